"""Served mode (cholmod_server_*): results equal the same requests applied
one at a time through the single-factor entry points, bit for bit, and the
oracle's results within the FP64 (1e-12) or FP32-storage (1e-5) bound;
failures and oversized requests are reported per request."""
import numpy as np
import pytest
import torch

from gpu_util import RESID_TOL, oracle_sequences, print_case, problem, rel_diff

pytestmark = pytest.mark.gpu


def dev(a, f32):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.float32 if f32 else np.float64))).cuda()


def test_server_equals_sequential(orc):
    import paper_1011_1173_amd as chm
    rng = np.random.default_rng(11)
    shapes = [(300, False), (129, True), (64, False), (1000, False), (77, True)]
    print_case("server", factors=len(shapes))
    base = [problem(n, 1, 900 + i)[0] for i, (n, _) in enumerate(shapes)]
    # a request sequence: each factor gets updates, then downdates of some of them
    reqs = []
    for it in range(4):
        for f, (n, f32) in enumerate(shapes):
            k = int(rng.integers(1, 33))
            V = rng.standard_normal((n, k)) / np.sqrt(n)
            reqs.append((f, V, +1))
    for f, (n, f32) in enumerate(shapes):
        ups = [r for r in reqs if r[0] == f and r[2] > 0]
        reqs.append((f, ups[0][1], -1))
        reqs.append((f, ups[2][1], -1))
    # sequential reference through the single-factor path
    ref = [dev(b, f32) for b, (_, f32) in zip(base, shapes)]
    for f, V, sg in reqs:
        st, _, _ = chm.update_async(ref[f], dev(V, shapes[f][1]), sg).status()
        assert st == 0
    # served
    Ls = [dev(b, f32) for b, (_, f32) in zip(base, shapes)]
    with chm.Server(ws_bytes=64 << 20, max_batch=8) as srv:
        ids = [srv.add_factor(L) for L in Ls]
        tickets = [srv.submit(ids[f], dev(V, shapes[f][1]), sg) for f, V, sg in reqs]
        srv.drain()
        res = [srv.poll(t) for t in tickets]
    for (st, lat) in res:
        assert st == 0 and lat > 0.0
    for f in range(len(shapes)):
        a = ref[f].cpu().numpy()
        b = Ls[f].cpu().numpy()
        assert np.array_equal(a, b), "factor %d" % f
    # and against the oracle: the same requests in FP64 on the stored inputs
    # (FP32-storage factors: their binary32 values), bound 1e-12 / 1e-5
    starts, seqs = [], []
    for f, (b, (n, f32)) in enumerate(zip(base, shapes)):
        cast = (lambda a: a.astype(np.float32).astype(np.float64)) if f32 else (lambda a: a)
        starts.append(cast(b))
        seqs.append([(cast(V), sg) for ff, V, sg in reqs if ff == f])
    refs = oracle_sequences(orc, starts, seqs)
    for f, (n, f32) in enumerate(shapes):
        d = rel_diff(Ls[f].cpu().numpy().astype(np.float64), refs[f])
        assert d <= (1e-5 if f32 else RESID_TOL), (f, n, f32, d)


def test_server_reports_failures_per_request(orc):
    import paper_1011_1173_amd as chm
    print_case("server-fail")
    n, r = 100, 40
    L, _ = problem(n, 1, seed=71)
    Vbad = np.zeros((n, 2))
    Vbad[:, 0] = 2.0 * L[r, :n]
    _, ost, oinfo = orc.modify(L, Vbad, -1)
    assert ost == orc.NOT_PD
    L2, V2 = problem(200, 16, seed=72)
    big = torch.zeros(5000, 5000, dtype=torch.float64, device="cuda")
    big.diagonal().fill_(1.0)
    # a 1 MiB budget: the two small requests fit together; the n = 5000,
    # k = 16 request needs about 3.3 MB of workspace and can never run
    with chm.Server(ws_bytes=1 << 20, max_batch=4) as srv:
        a = srv.add_factor(dev(L, False))
        b = srv.add_factor(dev(L2, False))
        c = srv.add_factor(big)
        t1 = srv.submit(a, dev(Vbad, False), -1)
        t2 = srv.submit(b, dev(V2, False), +1)
        t3 = srv.submit(c, torch.zeros(5000, 16, dtype=torch.float64, device="cuda"), +1)
        srv.drain()
        s1, s2, s3 = srv.poll(t1), srv.poll(t2), srv.poll(t3)
    assert s1[0] == chm.ERR_NOT_PD
    assert s2[0] == 0
    assert s3[0] == chm.ERR_ARG  # its workspace exceeds the server's whole HBM budget


def test_server_rejects_overflowing_sizes():
    """Sizes whose byte counts overflow are refused when the factor is
    registered or the request submitted, so no request can wait in a queue
    that no batch will ever take it from (drain would never return)."""
    import ctypes
    import paper_1011_1173_amd as chm
    from paper_1011_1173_amd import _native
    print_case("server-overflow")
    lib = _native.load()
    L = torch.eye(100, dtype=torch.float64, device="cuda")
    V = torch.zeros(100, 1, dtype=torch.float64, device="cuda")
    with chm.Server(ws_bytes=1 << 20, max_batch=4) as srv:
        fid = ctypes.c_int32(-1)
        assert lib.cholmod_server_add_factor(srv._h, ctypes.c_void_p(L.data_ptr()), 100, 1 << 62,
                                             chm.F64, ctypes.byref(fid)) == chm.ERR_ARG
        a = srv.add_factor(L)
        t = ctypes.c_uint64(0)
        assert lib.cholmod_server_submit(srv._h, a, ctypes.c_void_p(V.data_ptr()), 1 << 60, 1,
                                         ctypes.byref(t)) == chm.ERR_ARG
        ok = srv.submit(a, V, +1)
        srv.drain()
        assert srv.poll(ok)[0] == 0
    # V = 0 leaves the identity factor unchanged
    assert torch.allclose(L, torch.eye(100, dtype=torch.float64, device="cuda"), atol=1e-15)


def test_server_batches_overlap_on_the_device(orc):
    """Requests that arrive while a long batch runs are launched at once on
    another stream and finish while it is still running; each result equals
    the same request applied alone (bit for bit) and the oracle's."""
    import time
    import paper_1011_1173_amd as chm
    from gpu_util import inputs
    print_case("server-overlap")
    nbig, ksmall = 16384, 4
    Lbig = inputs.spd_factor(nbig, 91, device="cuda")
    Vbig = inputs.update_vectors(nbig, 32, 91, device="cuda")
    smalls = [problem(300 + 17 * i, ksmall, 920 + i) for i in range(4)]
    alone = []
    for L, V in smalls:
        Ld, Vd = dev(L, False), dev(V, False)
        st, _, _ = chm.update_async(Ld, Vd, +1).status()
        assert st == 0
        alone.append(Ld.cpu().numpy())
    Ls = [dev(L, False) for L, _ in smalls]
    Vs = [dev(V, False) for _, V in smalls]
    torch.cuda.synchronize()
    with chm.Server(ws_bytes=1 << 30, max_batch=16, streams=4) as srv:
        big = srv.add_factor(Lbig)
        ids = [srv.add_factor(L) for L in Ls]
        tb = srv.submit(big, Vbig, +1)
        time.sleep(0.002)  # the big batch is on the GPU
        ts = [srv.submit(i, V, +1) for i, V in zip(ids, Vs)]
        small_res, big_done_first = [], False
        for t in ts:
            while True:
                r = srv.poll(t)
                if r is not None:
                    break
                time.sleep(2e-5)
            small_res.append(r)
        # every small request is done: the big one must still be running
        rb = srv.poll(tb)
        big_done_first = rb is not None
        srv.drain()
        if rb is None:
            rb = srv.poll(tb)
    assert all(r[0] == 0 for r in small_res) and rb[0] == 0
    assert not big_done_first, "the small requests waited for the long batch"
    lat_small = max(r[1] for r in small_res)
    assert lat_small < rb[1], (lat_small, rb[1])
    for f, (L, V) in enumerate(smalls):
        out = Ls[f].cpu().numpy()
        assert np.array_equal(out, alone[f]), "factor %d differs from its result alone" % f
        ref, st, _ = orc.modify(L, V, +1)
        assert st == 0 and rel_diff(out, ref) <= RESID_TOL
