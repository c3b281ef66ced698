"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/cholmod_mi355x.h, and rejects bad arguments on the host
before any HIP call (so these run without a GPU and compute nothing)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cholmod_mi355x.h")


@pytest.fixture(scope="module")
def nat():
    from paper_1011_1173_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_1011_1173_amd import build
        build.build()
    _native.load()
    return _native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cholmod_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(nat):
    names = declared_functions()
    assert len(names) >= 7
    lib = ctypes.CDLL(nat.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(nat.EXPORTS) == names


def test_version_and_strings(nat):
    lib = nat.load()
    assert lib.cholmod_version() >= 100
    for code in (0, -1, -2, -3, -4):
        assert len(nat.status_string(code)) >= 2
    assert nat.status_string(12345) == "unknown status"


def test_decode_info(nat):
    assert nat.decode_info(nat.INFO_NONE, 16) == (0, -1, -1)
    # index 37 (row 2, col 5 with k = 16), code NOT_PD = 1
    assert nat.decode_info((37 << 2) | 1, 16) == (nat.ERR_NOT_PD, 2, 5)
    assert nat.decode_info((48 << 2) | 2, 16) == (nat.ERR_BAD_DIAG, 3, 0)


def test_workspace_bytes(nat):
    assert nat.workspace_bytes(-1, 4) == 0
    assert nat.workspace_bytes(4, -1) == 0
    assert nat.workspace_bytes(10, 2, 7) == 0
    a = nat.workspace_bytes(100, 16)
    b = nat.workspace_bytes(200, 16)
    c = nat.workspace_bytes(200, 32)
    assert 0 < a < b < c
    assert a % 256 == 0 and b % 256 == 0
    assert nat.workspace_bytes(100, 16, nat.F32S) < a
    # private copy of V plus one rotation record per row and column
    assert a >= 100 * 16 * 8 + 100 * 16 * 32
    assert nat.workspace_bytes(0, 0) > 0


FAKE = ctypes.c_void_p(0x100000)  # never dereferenced: validation fails first


def _ex(nat, L=FAKE, V=FAKE, n=8, k=2, ldl=8, sigma=1, flags=0, ws=FAKE, wsb=1 << 20,
        info=FAKE):
    return nat.load().cholmod_update_ex(L, V, n, k, ldl, sigma, flags, ws, wsb, info, None)


@pytest.mark.parametrize("kw", [
    dict(n=-1), dict(k=-1), dict(ldl=7), dict(ldl=0, n=0), dict(sigma=0), dict(sigma=2),
    dict(L=None), dict(V=None), dict(ws=None), dict(wsb=16), dict(info=None),
    dict(info=ctypes.c_void_p(0x100004)), dict(ws=ctypes.c_void_p(0x100010)), dict(flags=64),
])
def test_bad_arguments_rejected_on_host(nat, kw):
    assert _ex(nat, **kw) == nat.ERR_ARG


def test_bad_arguments_sync_and_async(nat):
    lib = nat.load()
    assert lib.cholmod_update(FAKE, FAKE, 8, 2, 4, 1, None) == nat.ERR_ARG
    assert lib.cholmod_update(FAKE, FAKE, 8, 2, 8, 0, None) == nat.ERR_ARG
    assert lib.cholmod_update(None, FAKE, 8, 2, 8, 1, None) == nat.ERR_ARG
    assert lib.cholmod_update_async(FAKE, None, 8, 2, 8, 1, FAKE, 1 << 20, FAKE, None) == nat.ERR_ARG
    assert lib.cholmod_update_async(FAKE, FAKE, 8, 2, 8, -1, FAKE, 10, FAKE, None) == nat.ERR_ARG


@pytest.mark.parametrize("kw", [
    dict(n=-1), dict(k=-1), dict(ldl=7), dict(sigma=0), dict(L=None), dict(V=None),
    dict(ws=None), dict(wsb=16), dict(info=None), dict(info=ctypes.c_void_p(0x100004)),
    dict(ws=ctypes.c_void_p(0x100010)),
])
def test_f32s_bad_arguments_rejected_on_host(nat, kw):
    a = dict(L=FAKE, V=FAKE, n=8, k=2, ldl=8, sigma=1, ws=FAKE, wsb=1 << 20, info=FAKE)
    a.update(kw)
    lib = nat.load()
    assert lib.cholmod_update_f32s_async(a["L"], a["V"], a["n"], a["k"], a["ldl"], a["sigma"],
                                         a["ws"], a["wsb"], a["info"], None) == nat.ERR_ARG
    assert lib.cholmod_update_f32s(FAKE, FAKE, 8, 2, 4, 1, None) == nat.ERR_ARG
    assert lib.cholmod_update_f32s(FAKE, None, 8, 2, 8, -1, None) == nat.ERR_ARG


def _desc(nat, n=8, k=2, ldl=None, sigma=1, dtype=0, L=0x100000, V=0x200000):
    return nat.Desc(L, V, n, k, n if ldl is None else ldl, sigma, dtype)


def test_batched_workspace_and_validation(nat):
    lib = nat.load()
    arr = (nat.Desc * 3)(_desc(nat), _desc(nat, n=100, k=33), _desc(nat, n=70, k=5, dtype=1))
    need = lib.cholmod_workspace_bytes_batched(arr, 3)
    single = sum(nat.workspace_bytes(n, k, t) for n, k, t in [(8, 2, 0), (100, 33, 0), (70, 5, 1)])
    assert need >= single and need % 256 == 0
    for bad in [dict(n=-1), dict(ldl=3), dict(sigma=0), dict(dtype=5), dict(L=None)]:
        b = (nat.Desc * 2)(_desc(nat), _desc(nat, **bad))
        assert lib.cholmod_workspace_bytes_batched(b, 2) == 0
        assert lib.cholmod_update_batched(b, 2, FAKE, 1 << 30, FAKE, None) == nat.ERR_ARG
    assert lib.cholmod_update_batched(arr, -1, FAKE, 1 << 30, FAKE, None) == nat.ERR_ARG
    assert lib.cholmod_update_batched(arr, 3, FAKE, need - 1, FAKE, None) == nat.ERR_ARG
    assert lib.cholmod_update_batched(arr, 3, FAKE, need, None, None) == nat.ERR_ARG
    assert lib.cholmod_update_batched(arr, 3, ctypes.c_void_p(0x100010), need, FAKE,
                                      None) == nat.ERR_ARG
    assert lib.cholmod_update_batched(arr, 0, None, 0, None, None) == nat.OK


def test_server_bad_config_rejected_on_host(nat):
    lib = nat.load()
    out = ctypes.c_void_p()
    for cfg in [nat.ServerCfg(16, 0, 0, 0, 0), nat.ServerCfg(1 << 20, -1, 0, 0, 0),
                nat.ServerCfg(1 << 20, 70000, 0, 0, 0), nat.ServerCfg(1 << 20, 0, 0, -1, 0),
                nat.ServerCfg(1 << 20, 0, 0, 17, 0)]:
        assert lib.cholmod_server_create(ctypes.byref(cfg), ctypes.byref(out)) == nat.ERR_ARG
    assert lib.cholmod_server_create(None, ctypes.byref(out)) == nat.ERR_ARG
    assert lib.cholmod_server_add_factor(None, FAKE, 4, 4, 0, None) == nat.ERR_ARG
    assert lib.cholmod_server_poll(None, 1, None, None) == nat.ERR_ARG
    assert lib.cholmod_server_drain(None) == nat.ERR_ARG
    assert lib.cholmod_server_destroy(None) == nat.ERR_ARG


def test_python_binding_rejects_bad_tensors():
    import torch
    import paper_1011_1173_amd as chm
    L = torch.eye(4, dtype=torch.float64)
    V = torch.ones(4, 1, dtype=torch.float64)
    with pytest.raises(chm.ArgumentError):
        chm.update(L, V, 1)  # CPU tensors are not accepted
    with pytest.raises(chm.ArgumentError):
        chm.update(L.float(), V.float(), 1)


def test_ooc_workspace_is_linear_in_n(nat):
    lib = nat.load()
    ws = lib.cholmod_workspace_bytes_ooc
    assert ws(-1, 4, nat.F64) == 0
    assert ws(10, -1, nat.F64) == 0
    assert ws(10, 4, 9) == 0
    a, b = ws(10_000, 16, nat.F64), ws(20_000, 16, nat.F64)
    assert 0 < a < b
    # O(n (64 + k)) device bytes: doubling n at most doubles it (plus alignment)
    assert b <= 2 * a + 4096
    # three 64-row panels of n elements dominate: at least 3 * 64 * n * 8 bytes
    assert a >= 3 * 64 * 10_000 * 8
    assert ws(10_000, 16, nat.F32S) < a


def test_ooc_bad_arguments_rejected_on_host(nat):
    lib = nat.load()
    p = ctypes.c_void_p
    host = (ctypes.c_double * 16)()
    info = ctypes.c_int64(0)
    dev = p(256)  # never dereferenced: the calls fail in validation
    call = lambda L, V, n, k, ldl, sg, dt, ws=None, wsb=0: lib.cholmod_update_ooc(
        L, V, n, k, ldl, sg, dt, ws, wsb, ctypes.byref(info), None)
    L = ctypes.cast(host, p)
    assert call(None, dev, 4, 2, 4, 1, nat.F64) == nat.ERR_ARG      # no L
    assert call(L, None, 4, 2, 4, 1, nat.F64) == nat.ERR_ARG        # no V
    assert call(L, dev, 4, 2, 3, 1, nat.F64) == nat.ERR_ARG         # ldl < n
    assert call(L, dev, 4, 2, 4, 0, nat.F64) == nat.ERR_ARG         # sigma
    assert call(L, dev, 4, 2, 4, 1, 5) == nat.ERR_ARG               # dtype
    assert call(L, dev, -1, 2, 4, 1, nat.F64) == nat.ERR_ARG        # n < 0
    assert call(L, dev, 4, 2, 4, 1, nat.F64, p(256), 16) == nat.ERR_ARG   # small workspace
    big = lib.cholmod_workspace_bytes_ooc(4, 2, nat.F64)
    assert call(L, dev, 4, 2, 4, 1, nat.F64, p(257), big) == nat.ERR_ARG  # misaligned
    # nothing to do: no HIP call, L untouched
    assert call(L, dev, 0, 2, 1, 1, nat.F64) == nat.OK
    assert call(L, dev, 4, 0, 4, 1, nat.F64) == nat.OK
    assert info.value == nat.INFO_NONE


def test_ooc_python_binding_rejects_bad_tensors():
    import torch
    import paper_1011_1173_amd as chm
    L = torch.eye(4, dtype=torch.float64)
    with pytest.raises(chm.ArgumentError):
        chm.update_ooc(L, torch.zeros(4, 2, dtype=torch.float64), 1)   # V on the host
    with pytest.raises(chm.ArgumentError):
        chm.update_ooc(L.float(), torch.zeros(4, 2, dtype=torch.float64), 1)


def test_batch_graph_bad_arguments_rejected_on_host(nat):
    lib = nat.load()
    p = ctypes.c_void_p
    h = p()
    d = nat.Desc(256, 256, 100, 4, 100, 1, nat.F64)
    arr = (nat.Desc * 1)(d)
    need = lib.cholmod_workspace_bytes_batched(arr, 1)
    assert need > 0
    assert lib.cholmod_batch_graph_create(arr, 0, p(256), need, p(256), ctypes.byref(h)) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_create(arr, 1, p(256), need - 1, p(256), ctypes.byref(h)) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_create(arr, 1, p(256), need, None, ctypes.byref(h)) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_create(arr, 1, p(257), need, p(256), ctypes.byref(h)) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_create(arr, 1, p(256), need, p(256), None) == nat.ERR_ARG
    bad = (nat.Desc * 1)(nat.Desc(256, 256, 100, 4, 99, 1, nat.F64))  # ldl < n
    assert lib.cholmod_batch_graph_create(bad, 1, p(256), need, p(256), ctypes.byref(h)) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_launch(None, None) == nat.ERR_ARG
    assert lib.cholmod_batch_graph_destroy(None) == nat.OK


def test_noalloc_rejects_oversized_problems_on_host(nat):
    """The allocation-free entry point refuses a problem whose workspace
    exceeds its fixed device array before any HIP call (fake non-null
    pointers: nothing is dereferenced)."""
    lib = nat.load()
    cap = lib.cholmod_noalloc_max_bytes()
    assert cap >= 1 << 20
    n, k = 60000, 16
    assert nat.workspace_bytes(n, k) > cap
    fake = ctypes.c_void_p(4096)
    assert lib.cholmod_update_noalloc(fake, fake, n, k, n, 1, fake, None) == nat.ERR_ARG
    # bad arguments as for the other entry points
    assert lib.cholmod_update_noalloc(fake, fake, 10, 2, 5, 1, fake, None) == nat.ERR_ARG
    assert lib.cholmod_update_noalloc(fake, fake, 10, 2, 10, 0, fake, None) == nat.ERR_ARG
    assert lib.cholmod_update_noalloc(fake, fake, 10, 2, 10, 1, None, None) == nat.ERR_ARG


def test_plan_table_on_host(nat):
    """Plan table and bucket functions: pure host code."""
    lib = nat.load()
    nb, kb = ctypes.c_int(-1), ctypes.c_int(-1)
    for (n, k, en, ek) in [(64, 1, 0, 0), (256, 16, 0, 0), (257, 17, 1, 1), (4096, 32, 2, 1),
                           (4097, 33, 3, 2), (16385, 65, 4, 3)]:
        assert lib.cholmod_plan_bucket(n, k, ctypes.byref(nb), ctypes.byref(kb)) == nat.OK
        assert (nb.value, kb.value) == (en, ek), (n, k)
    assert lib.cholmod_plan_bucket(-1, 1, None, None) == nat.ERR_ARG
    p = nat.Plan()
    assert lib.cholmod_get_plan(nat.F64, 2, 1, ctypes.byref(p)) == nat.OK
    assert p.maps == 1  # the default plan applies far blocks by their maps
    keep = nat.Plan(p.schedule, p.grid, p.order, p.poll, p.maps)
    q = nat.Plan(nat.SCHED_QUEUED, 128, nat.ORDER_FACTOR, 0)
    assert lib.cholmod_set_plan(nat.F64, 2, 1, ctypes.byref(q)) == nat.OK
    r = nat.Plan()
    assert lib.cholmod_get_plan(nat.F64, 2, 1, ctypes.byref(r)) == nat.OK
    assert (r.schedule, r.grid, r.order, r.poll) == (0, 128, 1, 0)
    assert lib.cholmod_set_plan(nat.F64, 2, 1, ctypes.byref(keep)) == nat.OK
    for bad in [nat.Plan(2, 0, 0, 2), nat.Plan(0, -1, 0, 2), nat.Plan(0, 0, 2, 2),
                nat.Plan(0, 0, 0, 3), nat.Plan(0, 0, 0, 2, 2)]:
        assert lib.cholmod_set_plan(nat.F64, 0, 0, ctypes.byref(bad)) == nat.ERR_ARG
    assert lib.cholmod_set_plan(7, 0, 0, ctypes.byref(q)) == nat.ERR_ARG
    assert lib.cholmod_set_plan(nat.F64, 5, 0, ctypes.byref(q)) == nat.ERR_ARG
    assert lib.cholmod_set_plan(nat.F64, 0, 4, ctypes.byref(q)) == nat.ERR_ARG
    assert lib.cholmod_get_plan(nat.F64, 0, 0, None) == nat.ERR_ARG


def test_plan_cache_file_loads(nat, tmp_path):
    """A plan cache in the tuner's format goes into the library's table."""
    import json
    from paper_1011_1173_amd import tune
    lib = nat.load()
    path = tmp_path / "plans.json"
    json.dump({"arch": "gfx950", "entries": [
        {"dtype": 1, "n_bucket": 3, "k_bucket": 2,
         "plan": {"schedule": 1, "grid": 0, "order": 0, "poll": 1}}]}, open(path, "w"))
    old = nat.Plan()
    assert lib.cholmod_get_plan(nat.F32S, 3, 2, ctypes.byref(old)) == nat.OK
    assert tune.load_plans(str(path)) == 1
    r = nat.Plan()
    assert lib.cholmod_get_plan(nat.F32S, 3, 2, ctypes.byref(r)) == nat.OK
    assert (r.schedule, r.poll) == (1, 1)
    assert lib.cholmod_set_plan(nat.F32S, 3, 2, ctypes.byref(old)) == nat.OK
    assert tune.load_plans(str(tmp_path / "missing.json")) == 0
