"""FP32-storage mode (cholmod_update_f32s*) against the FP64 oracle.

L and V are stored in binary32; the rows of each diagonal block are evaluated
in binary64 and the Apply to the other blocks' columns in binary32.  The
oracle runs in binary64 on the same binary32 inputs (converted exactly), so
the comparison measures the error of the FP32-storage evaluation alone.
Bound: relative Frobenius distance to the oracle's factor <= 1e-5 (the
FP32-storage accuracy target), relative residual against the FP64 definition
<= 1e-5.
"""
import numpy as np
import pytest
import torch

from gpu_util import print_case, problem, rel_diff, rel_residual_gpu

pytestmark = pytest.mark.gpu
F32_TOL = 1e-5


def f32_problem(orc, n, k, seed, sigma, ldl=None):
    """Binary32 inputs; for a downdate the factor already contains V V^T."""
    L, V = problem(n, k, seed, ldl=ldl)
    V = V.astype(np.float32).astype(np.float64)
    if sigma < 0:
        L, st, _ = orc.modify(L, V, +1)
        assert st == 0
    L = L.astype(np.float32).astype(np.float64)
    return L, V


def run_f32(L, V, sigma):
    import paper_1011_1173_amd as chm
    Ld = torch.from_numpy(np.ascontiguousarray(L.astype(np.float32))).cuda()
    Vd = torch.from_numpy(np.ascontiguousarray(V.astype(np.float32))).cuda()
    st, row, col = chm.update_async(Ld, Vd, sigma).status()
    return Ld.cpu().numpy().astype(np.float64), st, row, col


@pytest.mark.parametrize("n,k,sigma", [
    (1, 1, 1), (3, 16, -1), (17, 5, 1), (64, 16, 1), (65, 1, -1), (129, 16, -1),
    (200, 33, 1), (300, 16, 1), (1000, 16, -1), (1100, 7, 1),
])
def test_f32s_matches_oracle(orc, n, k, sigma):
    print_case("f32s", n=n, k=k, sigma=sigma)
    L, V = f32_problem(orc, n, k, 4000 + n + k, sigma)
    ref, ost, _ = orc.modify(L, V, sigma)
    assert ost == 0
    out, st, _, _ = run_f32(L, V, sigma)
    assert st == 0
    assert rel_diff(out, ref) <= F32_TOL
    assert rel_residual_gpu(out, L, V, sigma) <= F32_TOL


def test_f32s_headline_shape(orc):
    """n = 5000, k = 16, update then downdate in FP32 storage."""
    n, k = 5000, 16
    print_case("f32s-headline", n=n, k=k)
    L, V = f32_problem(orc, n, k, 2, +1)
    ref, ost, _ = orc.modify(L, V, +1)
    assert ost == 0
    out, st, _, _ = run_f32(L, V, +1)
    assert st == 0
    d_up = rel_diff(out, ref)
    back, st2, _, _ = run_f32(out, V, -1)
    assert st2 == 0
    d_rt = rel_diff(back, L)
    print("f32s n=5000 k=16: rel diff to oracle %.3g, round trip %.3g" % (d_up, d_rt))
    assert d_up <= F32_TOL and d_rt <= F32_TOL


def test_f32s_failure_index_and_padding(orc):
    n, k, r, ldl = 150, 3, 77, 160
    print_case("f32s-fail", n=n, k=k, r=r)
    L, _ = problem(n, 1, seed=35, ldl=ldl)
    L = L.astype(np.float32).astype(np.float64)
    V = np.zeros((n, k))
    V[:, 0] = 2.0 * L[r, :n]
    V[r:, 1] = 0.01
    _, ost, oinfo = orc.modify(L, V, -1)
    assert ost == orc.NOT_PD
    L[:, n:] = np.nan
    out, st, row, col = run_f32(L, V, -1)
    assert st == orc.NOT_PD and row * k + col == oinfo
    assert np.isnan(out[:, n:]).all()
    # rows before the failure saw V = 0 only: unchanged up to FP32 rounding
    assert np.abs(out[:r, :n] - L[:r, :n]).max() <= 1e-6 * np.abs(L[:, :n]).max()


def test_f32s_rejects_modes_and_mixed_types():
    import paper_1011_1173_amd as chm
    L = torch.eye(8, dtype=torch.float32, device="cuda")
    V = torch.zeros(8, 1, dtype=torch.float32, device="cuda")
    with pytest.raises(chm.ArgumentError):
        chm.update(L, V, 1, exact=True)
    with pytest.raises(chm.ArgumentError):
        chm.update(L, V.double(), 1)
