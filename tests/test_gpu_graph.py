"""Batches captured as a HIP graph (cholmod_batch_graph_*): every replay must
equal the directly launched batch bit for bit.  The graph is replayed several
times with the program's own eager work and synchronisations in between, and
each replay is checked."""
import pytest
import torch

from gpu_util import inputs, print_case

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_direct_batches():
    import paper_1011_1173_amd as chm
    shapes = [(300, 5, 1), (64, 16, -1), (1000, 16, 1), (129, 33, -1), (1, 2, 1), (500, 1, 1),
              (257, 20, 1), (700, 16, -1)]
    print_case("graph", factors=len(shapes))
    L0, V0, sg = [], [], []
    for f, (n, k, s) in enumerate(shapes):
        L = inputs.spd_factor(n, 80 + f, device="cuda")
        V = inputs.update_vectors(n, k, 80 + f, device="cuda")
        if s < 0:  # a well-posed downdate
            chm.update(L, V, 1)
        L0.append(L)
        V0.append(V)
        sg.append(s)
    # direct batch on copies
    ref = [L.clone() for L in L0]
    st = chm.update_batched(ref, V0, sg)
    assert all(x[0] == 0 for x in st), st
    # the graph works on its own buffers, refilled before each replay
    Lg = [L.clone() for L in L0]
    Vg = [V.clone() for V in V0]
    g = chm.BatchGraph(Lg, Vg, sg)
    other = inputs.spd_factor(200, 99, device="cuda")
    ov = inputs.update_vectors(200, 3, 99, device="cuda")
    try:
        for rep in range(4):
            for a, b in zip(Lg, L0):
                a.copy_(b)
            g.launch()
            sts = g.statuses()
            assert all(x[0] == 0 for x in sts), (rep, sts)
            for f, (a, b) in enumerate(zip(Lg, ref)):
                assert torch.equal(a, b), (rep, f, float((a - b).abs().max()))
            # eager work of the program between replays
            chm.update(other, ov, 1 if rep % 2 == 0 else -1)
            torch.cuda.synchronize()
    finally:
        g.close()


def test_graph_update_downdate_cycle_and_failure_status():
    """Two graphs (update, then the matching downdate) replayed alternately
    return L close to its start; a replay whose downdate fails reports the
    failing (row, column) like the direct batch."""
    import paper_1011_1173_amd as chm
    n, k = 400, 16
    print_case("graph-cycle", n=n, k=k)
    L = inputs.spd_factor(n, 90, device="cuda")
    V = inputs.update_vectors(n, k, 90, device="cuda")
    L0 = L.clone()
    up, down = chm.BatchGraph([L], [V], [1]), chm.BatchGraph([L], [V], [-1])
    try:
        for _ in range(3):
            up.launch()
            assert up.statuses()[0][0] == 0
            down.launch()
            assert down.statuses()[0][0] == 0
        assert float(torch.linalg.norm(L - L0) / torch.linalg.norm(L0)) <= 1e-13
        # make the downdate fail: V's first column now removes twice row 7
        V[:, 0] = 2.0 * L[7]
        Lf = L.clone()
        direct = chm.update_batched([Lf], [V], [-1])[0]
        down.launch()
        got = down.statuses()[0]
        assert direct[0] == chm.NotPositiveDefinite.status
        assert got == direct
    finally:
        up.close()
        down.close()


def test_graph_mixed_storage_and_closed_handle():
    """FP64 and FP32-storage factors in one captured batch; a closed graph
    refuses to launch."""
    import paper_1011_1173_amd as chm
    print_case("graph-mixed")
    shapes = [(300, 7, False), (450, 16, True), (65, 3, True), (900, 20, False)]
    Ls, Vs = [], []
    for f, (n, k, f32) in enumerate(shapes):
        dt = torch.float32 if f32 else torch.float64
        Ls.append(inputs.spd_factor(n, 95 + f, device="cuda").to(dt))
        Vs.append(inputs.update_vectors(n, k, 95 + f, device="cuda").to(dt))
    ref = [L.clone() for L in Ls]
    st = chm.update_batched(ref, Vs, [1] * len(Ls))
    assert all(x[0] == 0 for x in st)
    Lg = [L.clone() for L in Ls]
    g = chm.BatchGraph(Lg, Vs, [1] * len(Ls))
    g.launch()
    assert all(x[0] == 0 for x in g.statuses())
    for a, b in zip(Lg, ref):
        assert torch.equal(a, b)
    g.close()
    with pytest.raises(chm.ArgumentError):
        g.launch()
