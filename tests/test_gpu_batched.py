"""Batched modification (cholmod_update_batched) of uneven factors.

Each factor of a batch runs the same blocking and the same per-element
operations as the single-factor entry point of its storage type, so its
result must equal the single-factor result bit for bit; the single-factor
path itself is checked against the oracle elsewhere, and here again within
the FP64 (1e-12) or FP32-storage (1e-5) bound.
"""
import numpy as np
import pytest
import torch

from gpu_util import RESID_TOL, print_case, problem, rel_diff

pytestmark = pytest.mark.gpu
F32_TOL = 1e-5


def make_case(orc, n, k, sigma, f32, seed):
    L, V = problem(n, k, seed)
    if f32:
        V = V.astype(np.float32).astype(np.float64)
    if sigma < 0:
        L, st, _ = orc.modify(L, V, +1)
        assert st == 0
    if f32:
        L = L.astype(np.float32).astype(np.float64)
    return L, V


def to_dev(a, f32):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.float32 if f32 else np.float64))).cuda()


def run_both(cases, rotations=False):
    """cases: [(L, V, sigma, f32)] -> (single results, batched results, batched statuses)."""
    import paper_1011_1173_amd as chm
    single, stat1 = [], []
    for L, V, sg, f32 in cases:
        Ld, Vd = to_dev(L, f32), to_dev(V, f32)
        stat1.append(chm.update_async(Ld, Vd, sg, rotations=rotations).status())
        single.append(Ld.cpu().numpy().astype(np.float64))
    Ls = [to_dev(L, f32) for L, _, _, f32 in cases]
    Vs = [to_dev(V, f32) for _, V, _, f32 in cases]
    stats = chm.update_batched(Ls, Vs, [c[2] for c in cases])
    batched = [L.cpu().numpy().astype(np.float64) for L in Ls]
    return single, stat1, batched, stats


MIXED = [(1, 1, 1, False), (5, 3, -1, False), (63, 16, 1, True), (64, 16, -1, False),
         (65, 1, 1, False), (200, 17, -1, True), (130, 33, 1, False), (700, 16, 1, False),
         (333, 8, -1, True), (97, 2, 1, True)]


def test_batched_equals_single_bitwise(orc):
    print_case("batched-mixed", count=len(MIXED))
    cases = [make_case(orc, n, k, sg, f32, 5000 + i) + (sg, f32)
             for i, (n, k, sg, f32) in enumerate(MIXED)]
    single, stat1, batched, stats = run_both(cases)
    for i, ((L, V, sg, f32), a, b) in enumerate(zip(cases, single, batched)):
        assert stat1[i][0] == 0 and stats[i][0] == 0, (i, stat1[i], stats[i])
        assert np.array_equal(a, b), "factor %d: max |diff| %g" % (i, np.abs(a - b).max())
        ref, ost, _ = orc.modify(L, V, sg)
        assert ost == 0
        assert rel_diff(b, ref) <= (F32_TOL if f32 else RESID_TOL), i


def test_batched_failure_stays_in_its_factor(orc):
    print_case("batched-failure")
    n, k, r = 120, 3, 70
    Lf, _ = problem(n, 1, seed=41)
    Vf = np.zeros((n, k))
    Vf[:, 0] = 2.0 * Lf[r, :n]
    _, ost, oinfo = orc.modify(Lf, Vf, -1)
    assert ost == orc.NOT_PD
    cases = [make_case(orc, 150, 16, 1, False, 61) + (1, False),
             (Lf, Vf, -1, False),
             make_case(orc, 90, 5, -1, True, 62) + (-1, True)]
    single, stat1, batched, stats = run_both(cases)
    assert stats[0][0] == 0 and stats[2][0] == 0
    st, row, col = stats[1]
    assert st == orc.NOT_PD and row * k + col == oinfo
    assert np.array_equal(single[0], batched[0]) and np.array_equal(single[2], batched[2])
    assert np.array_equal(single[1][:r], batched[1][:r])


def test_batch_after_failed_batch_in_the_same_workspace(orc):
    """A batch whose workspace last held another batch's block maps (the same
    layout, so every map region is reused), among them the unusable maps of
    downdates that fail early, gives the single-factor results bit for bit."""
    import paper_1011_1173_amd as chm
    n, k, r = 1024, 16, 100  # 16 blocks: blocks 0..9 get maps
    print_case("batched-reused-workspace", n=n, k=k)
    first, second = [], []
    for i in range(6):
        if i % 2 == 0:  # fails at row r: the maps of later blocks are unusable
            Lf, _ = problem(n, 1, seed=900 + i)
            Vf = np.zeros((n, k))
            Vf[:, 0] = 2.0 * Lf[r, :n]
            first.append((Lf, Vf, -1))
        else:
            L, V = problem(n, k, seed=900 + i)
            first.append((L, V, 1))
        L, V = problem(n, k, seed=950 + i)
        second.append((L, V, 1))
    Ls = [to_dev(L, False) for L, _, _ in first]
    ws_bytes = int(chm._native.load().cholmod_workspace_bytes_batched(
        chm._descs(Ls, [to_dev(V, False) for _, V, _ in first], [s for _, _, s in first])[0],
        len(first)))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    st1 = chm.update_batched_async(Ls, [to_dev(V, False) for _, V, _ in first],
                                   [s for _, _, s in first], workspace=ws).statuses()
    assert [x[0] == orc.NOT_PD for x in st1] == [i % 2 == 0 for i in range(6)], st1
    Ls2 = [to_dev(L, False) for L, _, _ in second]
    st2 = chm.update_batched_async(Ls2, [to_dev(V, False) for _, V, _ in second],
                                   [1] * 6, workspace=ws).statuses()
    assert all(x[0] == 0 for x in st2), st2
    for i, (L, V, sg) in enumerate(second):
        Ld, Vd = to_dev(L, False), to_dev(V, False)
        assert chm.update_async(Ld, Vd, sg).status()[0] == 0
        assert torch.equal(Ld, Ls2[i]), i


def test_batched_uneven_pool(orc):
    """A smaller pool in the shape of the batched workload: n ~ U{64..1024},
    k ~ U{1..32}, half updates and half downdates, FP64 and FP32 storage."""
    rng = np.random.default_rng(7)
    count = 24
    print_case("batched-pool", count=count)
    cases = []
    for i in range(count):
        n = int(rng.integers(64, 1025))
        k = int(rng.integers(1, 33))
        sg = 1 if i % 2 == 0 else -1
        f32 = i % 3 == 0
        cases.append(make_case(orc, n, k, sg, f32, 7000 + i) + (sg, f32))
    single, stat1, batched, stats = run_both(cases)
    for i in range(count):
        assert stat1[i][0] == 0 and stats[i][0] == 0, i
        assert np.array_equal(single[i], batched[i]), i


def test_batches_back_to_back_equal_batches_in_turn(orc):
    """Two batches enqueued without waiting (the second is planned and its
    tables uploaded from the reused pinned buffer while the first may still
    run; factors 6..11 are in both) give what the two batches give one
    after the other, bit for bit."""
    import paper_1011_1173_amd as chm
    rng = np.random.default_rng(11)
    print_case("batched-back-to-back", count=18)
    cases = [make_case(orc, int(rng.integers(64, 1500)), int(rng.integers(1, 33)), 1, False,
                       7500 + i) for i in range(18)]
    Vb = [problem(L.shape[0], int(rng.integers(1, 33)), 7600 + i)[1]
          for i, (L, _) in enumerate(cases)]
    A, B = range(0, 12), range(6, 18)

    def run(wait):
        Ls = [to_dev(L, False) for L, _ in cases]
        VA = [to_dev(cases[i][1], False) for i in A]
        VB = [to_dev(Vb[i], False) for i in B]
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            pa = chm.update_batched_async([Ls[i] for i in A], VA, [1] * len(A), stream=st)
            sa = pa.statuses() if wait else None
            pb = chm.update_batched_async([Ls[i] for i in B], VB, [1] * len(B), stream=st)
        sa = sa if wait else pa.statuses()
        sb = pb.statuses()
        assert all(x[0] == 0 for x in sa + sb), (sa, sb)
        return [L.cpu().numpy() for L in Ls]

    inturn, b2b = run(True), run(False)
    for i in range(18):
        assert np.array_equal(inturn[i], b2b[i]), i


def test_every_tuned_plan_equals_single_bitwise(orc):
    """Every launch plan the autotuner may pick (queued with block maps: fewer
    workgroups, factor-major order, other poll levels) and the plans outside
    its set (stepped, queued without maps) leave each factor of the mixed
    batch bit for bit where the single-factor path does: the default
    single-factor path for a queued plan with maps, the single-factor path
    with every block by its rotations otherwise."""
    import paper_1011_1173_amd as chm
    from paper_1011_1173_amd import _native, tune
    cus = int(_native.load().cholmod_compute_units())
    assert cus > 0
    cases = [make_case(orc, n, k, sg, f32, 5100 + i) + (sg, f32)
             for i, (n, k, sg, f32) in enumerate(MIXED)]
    single_maps, _, _, _ = run_both(cases)
    single_rot, _, _, _ = run_both(cases, rotations=True)
    extra = [{"schedule": 0, "grid": 1, "order": 1, "poll": 1, "maps": 1},
             {"schedule": 0, "grid": 0, "order": 0, "poll": 2, "maps": 0},
             {"schedule": 1, "grid": 0, "order": 0, "poll": 2, "maps": 0}]
    for plan in tune.candidates(cus) + extra:
        print_case("batched-plan", **plan)
        Ls = [to_dev(L, f32) for L, _, _, f32 in cases]
        Vs = [to_dev(V, f32) for _, V, _, f32 in cases]
        stats = chm.update_batched(Ls, Vs, [c[2] for c in cases], plan=plan)
        maps = plan["schedule"] == 0 and plan.get("maps", 1) == 1
        single = single_maps if maps else single_rot
        for i, L in enumerate(Ls):
            assert stats[i][0] == 0, (plan, i, stats[i])
            assert np.array_equal(single[i], L.cpu().numpy().astype(np.float64)), (plan, i)


def test_tuner_writes_a_cache_the_library_loads(tmp_path):
    """The autotuner on one small bucket: it checks every candidate against
    the default plan bit for bit, writes the fastest to a plan cache, and the
    cache goes into the library's plan table."""
    import ctypes
    from paper_1011_1173_amd import _native, tune
    print_case("tuner")
    out = tmp_path / "plans.json"
    data = tune.tune(str(out), dtypes=("f64",), n_buckets=(0,), k_buckets=(0,), reps=1)
    assert len(data["entries"]) == 1
    e = data["entries"][0]
    assert (e["dtype"], e["n_bucket"], e["k_bucket"]) == (0, 0, 0)
    assert e["plan"]["schedule"] == 0 and e["plan"]["maps"] == 1
    assert e["ms"] > 0 and e["default_ms"] >= e["ms"]
    lib = _native.load()
    keep = _native.Plan()
    assert lib.cholmod_get_plan(_native.F64, 0, 0, ctypes.byref(keep)) == _native.OK
    try:
        assert tune.load_plans(str(out)) == 1
        got = _native.Plan()
        assert lib.cholmod_get_plan(_native.F64, 0, 0, ctypes.byref(got)) == _native.OK
        assert (got.schedule, got.grid, got.order, got.poll, got.maps) == tuple(
            e["plan"][f] for f in ("schedule", "grid", "order", "poll", "maps"))
    finally:
        lib.cholmod_set_plan(_native.F64, 0, 0, ctypes.byref(keep))
