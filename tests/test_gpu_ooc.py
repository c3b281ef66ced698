"""Out-of-core form (cholmod_update_ooc): the factor stays in host memory and
is streamed through the GPU in 64-row panels.  It runs the batched block-step
schedule, whose arithmetic is that of the single-factor fast schedule, so the
result must equal the in-core result bit for bit; failures report the same
(row, column)."""
import numpy as np
import pytest
import torch

from gpu_util import RESID_TOL, inputs, print_case, problem, rel_diff

pytestmark = pytest.mark.gpu


def incore(L, V, sigma):
    """The device entry point on a GPU copy, every block by its rotations (as
    the out-of-core form applies them); returns (L_new on host, status, row,
    col)."""
    import paper_1011_1173_amd as chm
    Ld, Vd = L.cuda(), V.cuda()
    st, row, col = chm.update_async(Ld, Vd, sigma, rotations=True).status()
    return Ld.cpu(), st, row, col


@pytest.mark.parametrize("n,k,sigma,ldl,pinned", [
    (1, 1, 1, None, False), (5, 3, -1, None, False), (64, 16, 1, None, True),
    (65, 4, -1, None, False), (200, 5, 1, 203, True), (300, 16, -1, None, False),
    (300, 33, 1, None, True), (1000, 16, 1, None, True), (3000, 16, -1, None, True),
    # pageable factors go through the library's pinned staging buffers: one
    # and two blocks over three passes (a panel is read again while its last
    # download may still wait to be unpacked), a ragged ldl, larger sizes
    (64, 33, 1, None, False), (100, 40, -1, None, False), (130, 17, 1, 131, False),
    (1000, 33, -1, 1003, False), (3000, 16, 1, None, False),
])
def test_ooc_equals_incore_bitwise(n, k, sigma, ldl, pinned):
    import paper_1011_1173_amd as chm
    print_case("ooc", n=n, k=k, sigma=sigma, ldl=ldl, pinned=pinned)
    L = inputs.spd_factor(n, 71, device="cuda", ldl=ldl).cpu()
    V = inputs.update_vectors(n, k, 71, device="cuda").cpu()
    if sigma < 0:  # a well-posed downdate: downdate by the V just added
        L, st, _, _ = incore(L, V, 1)
        assert st == 0
    ref, st, _, _ = incore(L, V, sigma)
    assert st == 0
    Lh = L.pin_memory() if pinned else L.clone()
    chm.update_ooc(Lh, V.cuda(), sigma)
    assert torch.equal(Lh, ref), "max |diff| = %g" % float((Lh - ref).abs().max())


def test_ooc_matches_oracle(orc):
    """Small case against the serial FP64 oracle, to the fast-mode bound."""
    import paper_1011_1173_amd as chm
    print_case("ooc-oracle", n=150, k=7)
    L, V = problem(150, 7, seed=72)
    ref, st, _ = orc.modify(L, V, 1)
    assert st == 0
    Lh = torch.from_numpy(L.copy())
    chm.update_ooc(Lh, torch.from_numpy(V).cuda(), 1)
    assert rel_diff(Lh.numpy(), ref) <= RESID_TOL


@pytest.mark.parametrize("pinned", [True, False])
def test_ooc_f32_storage_equals_incore_bitwise(pinned):
    import paper_1011_1173_amd as chm
    n, k = 500, 16
    print_case("ooc-f32s", n=n, k=k, pinned=pinned)
    L = inputs.spd_factor(n, 73, device="cuda").float().cpu()
    V = inputs.update_vectors(n, k, 73, device="cuda").float().cpu()
    ref, st, _, _ = incore(L, V, 1)
    assert st == 0
    Lh = L.pin_memory() if pinned else L.clone()
    chm.update_ooc(Lh, V.cuda(), 1)
    assert torch.equal(Lh, ref)


def test_ooc_caller_workspace_reused():
    """Two calls in a row with one caller workspace, the second smaller."""
    import paper_1011_1173_amd as chm
    print_case("ooc-ws", n=400, k=9)
    ws = torch.empty(chm.workspace_bytes_ooc(400, 9), dtype=torch.uint8, device="cuda")
    for n, k in ((400, 9), (130, 4)):
        L = inputs.spd_factor(n, 74 + n, device="cuda").cpu()
        V = inputs.update_vectors(n, k, 74 + n, device="cuda").cpu()
        ref, st, _, _ = incore(L, V, 1)
        Lh = L.clone()
        chm.update_ooc(Lh, V.cuda(), 1, workspace=ws)
        assert st == 0 and torch.equal(Lh, ref)


@pytest.mark.parametrize("n,r,k", [(200, 63, 5), (200, 64, 5), (300, 150, 16), (130, 129, 20)])
def test_ooc_failure_reports_incore_index(n, r, k):
    import paper_1011_1173_amd as chm
    print_case("ooc-fail", n=n, r=r, k=k)
    L, _ = problem(n, 1, seed=75)
    V = np.zeros((n, k))
    V[:, 0] = 2.0 * L[r, :n]
    if k > 1:
        V[r:, 1] = 0.01
    L, V = torch.from_numpy(L), torch.from_numpy(V)
    _, st, row, col = incore(L, V, -1)
    assert st == chm.NotPositiveDefinite.status
    Lh = L.clone()
    with pytest.raises(chm.NotPositiveDefinite) as ei:
        chm.update_ooc(Lh, V.cuda(), -1)
    assert (ei.value.row, ei.value.col) == (row, col)
    # rows before the failing block's step never changed beyond rounding of v = 0
    assert float((Lh[:r] - L[:r]).abs().max()) <= 1e-13 * float(L.abs().max())


def test_ooc_trivial_sizes():
    import paper_1011_1173_amd as chm
    print_case("ooc-trivial")
    L = inputs.spd_factor(40, 76).clone()
    before = L.clone()
    chm.update_ooc(L, torch.zeros(40, 0, dtype=torch.float64, device="cuda"), 1)
    assert torch.equal(L, before)
    E = torch.zeros(0, 0, dtype=torch.float64)
    chm.update_ooc(E, torch.zeros(0, 3, dtype=torch.float64, device="cuda"), 1)


def test_ooc_four_passes_ragged():
    """k = 64 (four 16-column passes, every panel streamed four times), ragged n."""
    import paper_1011_1173_amd as chm
    n, k = 1000, 64
    print_case("ooc-k64", n=n, k=k)
    L = inputs.spd_factor(n, 77, device="cuda").cpu()
    V = inputs.update_vectors(n, k, 77, device="cuda").cpu()
    ref, st, _, _ = incore(L, V, 1)
    assert st == 0
    Lh = L.pin_memory()
    chm.update_ooc(Lh, V.cuda(), 1)
    assert torch.equal(Lh, ref)
