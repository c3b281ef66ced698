"""Parity of the HIP path with the CPU oracle (needs an MI355X).

EXACT mode evaluates Algorithm 1 literally in IEEE binary64 and must equal
the oracle bit for bit.  The default (fast) mode must match the oracle's
factor and the definition within the FP64 bound: relative residual and
relative distance to the oracle's factor both <= 1e-12.
"""
import json
import os

import numpy as np
import pytest

from gpu_util import RESID_TOL, print_case, problem, rel_diff, rel_residual_gpu, run_gpu

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def down_problem(orc, n, k, seed, ldl=None):
    """A factor that contains V V^T, so that downdating by V is well posed."""
    L, V = problem(n, k, seed, ldl=ldl)
    Lup, st, _ = orc.modify(L, V, +1)
    assert st == 0
    return Lup, V


def inputs_for(orc, n, k, seed, sigma, ldl=None):
    return problem(n, k, seed, ldl=ldl) if sigma > 0 else down_problem(orc, n, k, seed, ldl)


# ----------------------------------------------------------------- EXACT: bitwise
@pytest.mark.parametrize("n,k,sigma", [
    (1, 1, 1), (2, 3, -1), (31, 1, 1), (32, 16, 1), (33, 16, -1), (100, 5, 1),
    (129, 64, -1), (70, 70, 1), (257, 2, -1),
])
def test_exact_mode_is_bitwise_equal_to_oracle(orc, n, k, sigma):
    print_case("exact", n=n, k=k, sigma=sigma)
    L, V = inputs_for(orc, n, k, 1000 + n + k, sigma)
    ref, st, _ = orc.modify(L, V, sigma)
    assert st == 0
    out, gst, _, _ = run_gpu(L, V, sigma, exact=True)
    assert gst == 0
    assert np.array_equal(out, ref), "max |diff| = %g" % np.abs(out - ref).max()


def test_exact_mode_worked_example(orc):
    g = json.load(open(os.path.join(HERE, "golden", "p5_worked_example.json")))
    out, st, _, _ = run_gpu(np.array(g["L"]), np.array(g["V"]), g["sigma"], exact=True)
    assert st == 0
    assert np.array_equal(out, np.array(g["L_new"]))


# ----------------------------------------------------------------- FAST: tolerance
@pytest.mark.parametrize("n,k,sigma", [
    (1, 1, 1), (5, 2, -1), (64, 1, 1), (95, 16, -1), (200, 16, 1), (333, 7, -1),
    (512, 1, 1), (512, 1, -1), (300, 64, 1), (150, 65, -1), (1000, 32, 1),
])
def test_fast_mode_matches_oracle(orc, n, k, sigma):
    print_case("fast", n=n, k=k, sigma=sigma)
    L, V = inputs_for(orc, n, k, 2000 + n + k, sigma)
    ref, st, _ = orc.modify(L, V, sigma)
    assert st == 0
    out, gst, _, _ = run_gpu(L, V, sigma)
    assert gst == 0
    assert np.all(np.diag(out) > 0)
    assert rel_diff(out, ref) <= RESID_TOL
    assert rel_residual_gpu(out, L, V, sigma) <= RESID_TOL


@pytest.mark.parametrize("exact", [False, True])
def test_config1_update_then_downdate_restores_L(orc, exact):
    """n = 512, k = 1: update, then the matching downdate (the small config)."""
    print_case("config1", exact=exact)
    L, V = problem(512, 1, seed=1)
    up, st, _, _ = run_gpu(L, V, +1, exact=exact)
    assert st == 0
    back, st, _, _ = run_gpu(up, V, -1, exact=exact)
    assert st == 0
    ref_up, _, _ = orc.modify(L, V, +1)
    ref_back, _, _ = orc.modify(ref_up, V, -1)
    if exact:
        assert np.array_equal(up, ref_up) and np.array_equal(back, ref_back)
    assert rel_diff(back, L) <= 1e-13
    assert rel_diff(up, ref_up) <= RESID_TOL


def test_headline_shape_full_size(orc):
    """n = 5000, k = 16 (the headline shape): the whole factor against the oracle."""
    print_case("headline", n=5000, k=16)
    L, V = problem(5000, 16, seed=2)
    ref_up, st, _ = orc.modify(L, V, +1)
    assert st == 0
    up, st, _, _ = run_gpu(L, V, +1)
    assert st == 0
    assert rel_diff(up, ref_up) <= RESID_TOL
    assert rel_residual_gpu(up, L, V, +1) <= RESID_TOL
    back, st, _, _ = run_gpu(up, V, -1)
    assert st == 0
    ref_back, _, _ = orc.modify(ref_up, V, -1)
    assert rel_diff(back, ref_back) <= RESID_TOL
    assert rel_diff(back, L) <= 1e-12


# ----------------------------------------------------------------- memory outside the triangle
@pytest.mark.parametrize("exact", [False, True])
def test_lower_triangle_and_padding_untouched(orc, exact):
    n, ldl, k = 77, 83, 5
    L, V = problem(n, k, seed=5, ldl=ldl)
    L[:, n:] = np.nan
    L[np.tril_indices(n, -1)] = np.nan
    out, st, _, _ = run_gpu(L, V, +1, exact=exact)
    assert st == 0
    assert np.isnan(out[:, n:]).all()
    assert np.isnan(out[np.tril_indices(n, -1)]).all()
    ref, _, _ = orc.modify(L, V, +1)
    assert rel_diff(out, ref) <= RESID_TOL


# ----------------------------------------------------------------- trivial cases
@pytest.mark.parametrize("exact", [False, True])
def test_noops(orc, exact):
    import torch
    import paper_1011_1173_amd as chm
    L, _ = problem(40, 1, seed=6)
    out, st, _, _ = run_gpu(L, np.zeros((40, 0)), 1, exact=exact)
    assert st == 0 and np.array_equal(out, L)
    out, st, _, _ = run_gpu(L, np.zeros((40, 3)), -1, exact=exact)
    assert st == 0
    if exact:
        assert np.array_equal(out, L)
    else:
        assert rel_diff(out, L) <= 1e-15
    E = torch.zeros(0, 0, dtype=torch.float64, device="cuda")
    chm.update(E, torch.zeros(0, 2, dtype=torch.float64, device="cuda"), 1, exact=exact)


# ----------------------------------------------------------------- failures
@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("n,r,k", [(40, 0, 3), (40, 17, 3), (300, 150, 16), (100, 99, 70),
                                   (200, 63, 5), (200, 64, 5), (1000, 575, 16)])
def test_indefinite_downdate_reports_oracle_index(orc, exact, n, r, k):
    print_case("fail", n=n, r=r, k=k, exact=exact)
    L, _ = problem(n, 1, seed=33)
    V = np.zeros((n, k))
    V[:, 0] = 2.0 * L[r, :n]
    if k > 1:
        V[r:, 1] = 0.01
    _, ost, oinfo = orc.modify(L, V, -1)
    assert ost == orc.NOT_PD
    out, st, row, col = run_gpu(L, V, -1, exact=exact)
    assert st == orc.NOT_PD
    assert row * k + col == oinfo
    # rows before r saw V = 0: untouched in exact mode; in fast mode the
    # rotation with v = 0 has c = 1 and 1/c = 1 only to within an ulp
    if exact:
        assert np.array_equal(out[:r], L[:r])
    elif r > 0:
        assert np.abs(out[:r] - L[:r]).max() <= 1e-13 * np.abs(L).max()


def test_failure_in_later_column_pass_reports_first_index(orc):
    """k > 64: the failure sits in a column of the second 64-column pass but in
    an earlier row than a failure of the first pass; the earlier row wins."""
    n, k = 60, 70
    L, _ = problem(n, 1, seed=8)
    V = np.zeros((n, k))
    V[:, 65] = 2.0 * L[10, :n]   # fails at (10, 65)
    V[:, 3] = 2.0 * L[30, :n]    # fails at (30, 3)
    _, ost, oinfo = orc.modify(L, V, -1)
    assert ost == orc.NOT_PD and oinfo == 10 * k + 65
    for exact in (False, True):
        _, st, row, col = run_gpu(L, V, -1, exact=exact)
        assert st == orc.NOT_PD and (row, col) == (10, 65)


@pytest.mark.parametrize("exact", [False, True])
def test_bad_diagonal(orc, exact):
    L, V = problem(50, 4, seed=9)
    L[23, 23] = -2.0
    _, ost, oinfo = orc.modify(L, V, 1)
    assert ost == orc.BAD_DIAG
    _, st, row, col = run_gpu(L, V, 1, exact=exact)
    assert st == orc.BAD_DIAG and row * 4 + col == oinfo


def test_sync_entry_point_and_python_errors(orc):
    import torch
    import paper_1011_1173_amd as chm
    L, V = problem(64, 2, seed=10)
    Ld = torch.from_numpy(L).cuda()
    Vd = torch.from_numpy(V).cuda()
    st = chm._native.load().cholmod_update(
        __import__("ctypes").c_void_p(Ld.data_ptr()), __import__("ctypes").c_void_p(Vd.data_ptr()),
        64, 2, 64, 1, None)
    torch.cuda.synchronize()
    assert st == 0
    ref, _, _ = orc.modify(L, V, 1)
    assert rel_diff(Ld.cpu().numpy(), ref) <= RESID_TOL
    Vbad = torch.zeros(64, 1, dtype=torch.float64, device="cuda")
    Vbad[:, 0] = 2.0 * Ld[5]
    with pytest.raises(chm.NotPositiveDefinite) as ei:
        chm.update(Ld, Vbad, -1)
    assert (ei.value.row, ei.value.col) == (5, 0)


# ----------------------------------------------------------------- schedules agree bit for bit
@pytest.mark.parametrize("n,k,sigma", [
    (1, 1, 1), (2, 2, -1), (3, 16, 1), (17, 5, 1), (18, 16, -1), (20, 3, 1), (63, 8, -1),
    (64, 16, 1), (65, 1, -1), (100, 15, 1), (129, 16, -1), (257, 7, 1), (1000, 16, 1),
    (1500, 2, -1), (2049, 16, -1),
])
def test_chain_schedule_equals_row_schedule_bitwise(orc, n, k, sigma):
    """The owner schedule with every block applied by its rotations (64-row
    blocks, each run as a systolic chain by the workgroup owning its columns,
    which has applied the earlier blocks to them) and the per-row fast
    schedule run the same Compute/Apply arithmetic in the same per-element
    order: their results must be identical bit for bit (k <= 16: one pass in
    both).  The default, which applies blocks far from an owner by their
    block maps, agrees with both to the FP64 tolerance and with the oracle."""
    print_case("schedules", n=n, k=k, sigma=sigma)
    L, V = inputs_for(orc, n, k, 3000 + n + k, sigma)
    a, sa, _, _ = run_gpu(L, V, sigma, rotations=True)
    b, sb, _, _ = run_gpu(L, V, sigma, blocked=True)
    assert sa == 0 and sb == 0
    assert np.array_equal(a, b), "max |diff| = %g" % np.abs(a - b).max()
    c, sc, _, _ = run_gpu(L, V, sigma)
    assert sc == 0
    if n <= 384:  # a factor of 6 blocks or fewer has no block maps
        assert np.array_equal(a, c)
    ref, st, _ = orc.modify(L, V, sigma)
    assert st == 0
    assert rel_diff(c, ref) <= RESID_TOL and rel_diff(c, a) <= RESID_TOL


@pytest.mark.parametrize("sigma,scale", [(-1, 0.9), (-1, 0.5), (1, 3.0)])
def test_block_maps_with_large_rotations(orc, sigma, scale):
    """A rank-1 modification whose row-150 rotation is large: for a downdate
    by 0.9 times row 150 of L, 1/c = 2.3 there, so the map of block 2 has
    entries beyond the bound for maps and every owner applies that block by
    its rotations; for 0.5 (1/c = 1.15) and for an update the map is used.
    Either way the result is the oracle's within the FP64 tolerance (scaled by
    the downdate's conditioning, 1 / (1 - scale^2))."""
    n = 1000
    print_case("maps-large", sigma=sigma, scale=scale)
    L, _ = problem(n, 1, seed=3300)
    V = np.zeros((n, 1))
    V[:, 0] = scale * L[150, :n]
    a, sa, _, _ = run_gpu(L, V, sigma)
    assert sa == 0
    ref, st, _ = orc.modify(L, V, sigma)
    assert st == 0
    cond = 1.0 / (1.0 - scale * scale) if sigma < 0 else 1.0
    assert rel_diff(a, ref) <= RESID_TOL * cond
    b, sb, _, _ = run_gpu(L, V, sigma, rotations=True)
    assert sb == 0 and rel_diff(a, b) <= RESID_TOL * cond


@pytest.mark.parametrize("n,k,sigma", [(300, 33, 1), (200, 21, -1), (130, 47, 1),
                                       (1000, 40, 1), (1300, 64, -1)])
def test_passes_equal_consecutive_column_slices_bitwise(orc, n, k, sigma):
    """k > 16 runs in passes of 16 columns of V; pass p only rotates its own
    columns of the private copy of V, so one call equals consecutive calls on
    the 16-column slices of V, bit for bit (the last slice narrower).  At
    n = 1000 and 1300 the far blocks go by their maps, and a sweep may apply
    later passes' maps early (whatever it does, the result is the same)."""
    print_case("passes", n=n, k=k, sigma=sigma)
    L, V = inputs_for(orc, n, k, 3100 + n + k, sigma)
    a, sa, _, _ = run_gpu(L, V, sigma)
    assert sa == 0
    b = L.copy()
    for m0 in range(0, k, 16):
        b, sb, _, _ = run_gpu(b, np.ascontiguousarray(V[:, m0:m0 + 16]), sigma)
        assert sb == 0
    assert np.array_equal(a, b), "max |diff| = %g" % np.abs(a - b).max()
    ref, st, _ = orc.modify(L, V, sigma)
    assert st == 0 and rel_diff(a, ref) <= RESID_TOL
