"""Factors with more 64-row blocks than the GPU has compute units.

The fast schedule launches one workgroup per block and a workgroup fills a
compute unit, so at n = 17000 (266 blocks on 256 CUs) the last workgroups
start only after the first ones have finished and then catch up on every
earlier block.  The result must still equal the per-row schedule bit for bit,
and the modified factor must satisfy L~^T L~ = L^T L + sigma V V^T (checked
with random probes, O(n^2) on the GPU).  Everything stays on the device.
"""
import pytest
import torch

from gpu_util import inputs, print_case

pytestmark = pytest.mark.gpu


def probe_residual(Ln, L, V, sigma, nprobe=4, seed=0):
    """||U~^T U~ X - (U^T U + sigma V V^T) X|| / ||(U^T U + sigma V V^T) X||."""
    n = L.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    X = torch.randn(n, nprobe, generator=g, device="cuda", dtype=torch.float64)
    U = torch.triu(L[:, :n])
    Un = torch.triu(Ln[:, :n])
    # (U^T Y) as (Y^T U)^T with the small operand made contiguous
    lhs = ((Un @ X).T.contiguous() @ Un).T
    rhs = ((U @ X).T.contiguous() @ U).T + sigma * (V @ (V.T.contiguous() @ X))
    return float(torch.linalg.norm(lhs - rhs) / torch.linalg.norm(rhs))


@pytest.mark.parametrize("n,k,sigma", [(17000, 16, 1), (16500, 5, 1)])
def test_more_workgroups_than_compute_units(n, k, sigma):
    import paper_1011_1173_amd as chm
    print_case("scale", n=n, k=k, sigma=sigma)
    L = inputs.spd_factor(n, seed=61, device="cuda")
    V = inputs.update_vectors(n, k, seed=61, device="cuda")
    a = L.clone()
    st, _, _ = chm.update_async(a, V, sigma, rotations=True).status()
    assert st == 0
    b = L.clone()
    st, _, _ = chm.update_async(b, V, sigma, blocked=True).status()
    assert st == 0
    assert torch.equal(a, b), "max |diff| = %g" % float((a - b).abs().max())
    assert probe_residual(a, L, V, sigma) <= 1e-12
    # the default (far blocks by their maps) agrees to the FP64 tolerance
    c = L.clone()
    st, _, _ = chm.update_async(c, V, sigma).status()
    assert st == 0
    assert float(torch.linalg.norm(c - a) / torch.linalg.norm(a)) <= 1e-12
    assert probe_residual(c, L, V, sigma) <= 1e-12
    a = c
    # and back: the matching downdate restores L to rounding
    st, _, _ = chm.update_async(a, V, -sigma).status()
    assert st == 0
    assert float(torch.linalg.norm(a - L) / torch.linalg.norm(L)) <= 1e-12


def test_f32_storage_more_workgroups_than_compute_units():
    import paper_1011_1173_amd as chm
    n, k = 17000, 16
    print_case("scale-f32s", n=n, k=k)
    L64 = inputs.spd_factor(n, seed=62, device="cuda")
    V64 = inputs.update_vectors(n, k, seed=62, device="cuda")
    ref = L64.clone()
    st, _, _ = chm.update_async(ref, V64, +1).status()
    assert st == 0
    L = L64.float()
    st, _, _ = chm.update_async(L, V64.float(), +1).status()
    assert st == 0
    d = float(torch.linalg.norm(L.double() - ref) / torch.linalg.norm(ref))
    assert d <= 1e-5, d


@pytest.mark.parametrize("f32", [False, True])
def test_pass_pairs_share_far_tiles_bitwise(f32):
    """With more blocks than compute units (n = 33000: 516 blocks), an even
    pass also applies the next pass's block maps to the far tiles it
    has at hand, for the blocks whose next-pass maps are published already,
    and the next pass resumes after them.  Every element goes through the
    same operations in the same order as without that sharing, so one k = 40
    call (passes 0+1 paired, pass 2 of 8 columns alone) equals consecutive
    calls on the 16-column slices of V (single passes, nothing paired) bit
    for bit -- for the update and for the matching downdate, with binary64
    storage and with binary32 storage (which carries V of the later pass in
    binary64 between the two)."""
    import paper_1011_1173_amd as chm
    n, k = 33000, 40
    print_case("pass-pairs", n=n, k=k, f32=f32)
    dt = torch.float32 if f32 else torch.float64
    L = inputs.spd_factor(n, seed=71, device="cuda").to(dt)
    V = inputs.update_vectors(n, k, seed=71, device="cuda").to(dt)
    one = L.clone()
    assert chm.update_async(one, V, 1).status()[0] == 0
    sl = L.clone()
    for m0 in range(0, k, 16):
        assert chm.update_async(sl, V[:, m0:m0 + 16].contiguous(), 1).status()[0] == 0
    assert torch.equal(one, sl), "max |diff| = %g" % float((one - sl).abs().max())
    tol = 1e-5 if f32 else 1e-12
    assert probe_residual(one.double(), L.double(), V.double(), 1) <= tol
    back = one.clone()
    assert chm.update_async(back, V, -1).status()[0] == 0
    for m0 in range(0, k, 16):
        assert chm.update_async(sl, V[:, m0:m0 + 16].contiguous(), -1).status()[0] == 0
    assert torch.equal(back, sl), "max |diff| = %g" % float((back - sl).abs().max())
    assert float(torch.linalg.norm((back - L).double()) / torch.linalg.norm(L.double())) <= tol
    del one, sl, back, L, V
    torch.cuda.empty_cache()
