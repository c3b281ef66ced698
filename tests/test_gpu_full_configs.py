"""The batched and served workloads at their full sizes, in the form the
benchmark times, against the single-factor path (which the parity tests pin
to the oracle) bit for bit:

* batched: 256 factors, n ~ U{64..4096}, k ~ U{1..32}, a mix of updates and
  downdates (a downdate removes a V added before, so A~ stays SPD), in FP64
  and in FP32 storage, through one cholmod_update_batched call; the four
  smallest and four largest factors are also checked against the oracle;
* served: a pool of 64 factors with n cycled over {1024, ..., 16384}, each
  receiving sliding-window request pairs (an update by a new V, then the
  downdate of the factor's oldest V) through the served mode; every factor
  must end exactly as the same requests applied one at a time, and every
  factor with n <= 4096 as the oracle applies them (within 1e-12)."""
import random

import numpy as np
import pytest
import torch

from gpu_util import RESID_TOL, inputs, oracle_sequences, print_case, rel_diff

pytestmark = pytest.mark.gpu


def new_v(gen, n, k, dt):
    return (torch.randn(n, k, generator=gen, device="cuda", dtype=torch.float64)
            / float(np.sqrt(n))).to(dt)


@pytest.mark.parametrize("f32", [False, True])
def test_batched_256_uneven_equals_single(orc, f32):
    import paper_1011_1173_amd as chm
    print_case("batched-256", f32=f32)
    dt = torch.float32 if f32 else torch.float64
    rng = random.Random(21)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2121)
    nf = 256
    ns = [rng.randint(64, 4096) for _ in range(nf)]
    L0, Vs, sg = [], [], []
    for f, n in enumerate(ns):
        L = inputs.spd_factor(n, 7000 + f, device="cuda").to(dt)
        V = new_v(gen, n, rng.randint(1, 32), dt)
        s = 1 if rng.random() < 0.5 else -1
        if s < 0:  # a downdate of a V added before
            st, _, _ = chm.update_async(L, V, 1).status()
            assert st == 0
        L0.append(L)
        Vs.append(V)
        sg.append(s)
    single = [L.clone() for L in L0]
    for L, V, s in zip(single, Vs, sg):
        chm.update_async(L, V, s)
    torch.cuda.synchronize()
    batched = [L.clone() for L in L0]
    stats = chm.update_batched(batched, Vs, sg)
    assert all(x[0] == 0 for x in stats), [x for x in stats if x[0] != 0][:4]
    for f in range(nf):
        assert torch.equal(single[f], batched[f]), "factor %d (n=%d)" % (f, ns[f])
    # the four smallest and the four largest factors against the oracle (FP64
    # on the stored inputs; FP32 storage within 1e-5)
    by_n = sorted(range(nf), key=lambda i: ns[i])
    pick = by_n[:4] + by_n[-4:]
    refs = oracle_sequences(orc, [L0[f].cpu().numpy().astype(np.float64) for f in pick],
                            [[(Vs[f].cpu().numpy().astype(np.float64), sg[f])] for f in pick])
    for f, ref in zip(pick, refs):
        d = rel_diff(batched[f].cpu().numpy().astype(np.float64), ref)
        assert d <= (1e-5 if f32 else RESID_TOL), (f, ns[f], d)


def test_served_pool_equals_sequential(orc):
    import paper_1011_1173_amd as chm
    sizes = [1024, 2048, 4096, 8192, 16384]
    nf = 64
    print_case("served-64", factors=nf, max_n=sizes[-1])
    rng = random.Random(22)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2222)
    ns = [sizes[f % len(sizes)] for f in range(nf)]
    base = [inputs.spd_factor(n, 8000 + f % len(sizes), device="cuda") for f, n in enumerate(ns)]
    # one prior V per factor, already added, then two sliding-window pairs each
    prior = [new_v(gen, n, rng.randint(1, 32), torch.float64) for n in ns]
    reqs = []  # (factor, V, sigma) in submission order
    window = [[v] for v in prior]
    for _ in range(2):
        for f, n in enumerate(ns):
            V = new_v(gen, n, rng.randint(1, 32), torch.float64)
            reqs.append((f, V, +1))
            reqs.append((f, window[f].pop(0), -1))
            window[f].append(V)
    ref = base  # modified in place by the sequential reference
    for f in range(nf):
        st, _, _ = chm.update_async(ref[f], prior[f], +1).status()
        assert st == 0
    served = [L.clone() for L in ref]
    waited = [L.clone() for L in ref]  # the same sequence, each call waited for
    for f, V, s in reqs:
        chm.update_async(ref[f], V, s)
    for f, V, s in reqs:
        assert chm.update_async(waited[f], V, s).status()[0] == 0
    torch.cuda.synchronize()
    with chm.Server(ws_bytes=1 << 30, max_batch=64) as srv:
        ids = [srv.add_factor(L) for L in served]
        tickets = [srv.submit(ids[f], V, s) for f, V, s in reqs]
        srv.drain()
        res = [srv.poll(t) for t in tickets]
    assert all(st == 0 for st, _ in res), [r for r in res if r[0] != 0][:4]

    def where(a, b):
        d = (a - b).abs()
        i = int(torch.nan_to_num(d, nan=float("inf")).argmax())
        return "max |diff| %.3e at (%d, %d), %d elements differ, NaN %d / %d" % (
            float(torch.nan_to_num(d, nan=float("inf")).max()), i // a.shape[1], i % a.shape[1],
            int((a != b).sum()), int(torch.isnan(a).sum()), int(torch.isnan(b).sum()))

    for f in range(nf):
        assert torch.equal(ref[f], waited[f]), "reference, factor %d (n=%d): %s" % (
            f, ns[f], where(ref[f], waited[f]))
        assert torch.equal(ref[f], served[f]), "factor %d (n=%d, k %s): %s" % (
            f, ns[f], [V.shape[1] for g, V, _ in reqs if g == f], where(ref[f], served[f]))
    # every factor with n <= 4096 against the oracle: the prior V, then its
    # request pairs in order, from the generator's factor
    small = [f for f in range(nf) if ns[f] <= 4096]
    starts = [inputs.spd_factor(ns[f], 8000 + f % len(sizes), device="cuda").cpu().numpy()
              for f in small]
    seqs = [[(prior[f].cpu().numpy(), +1)] + [(V.cpu().numpy(), s) for ff, V, s in reqs if ff == f]
            for f in small]
    refs = oracle_sequences(orc, starts, seqs)
    for f, r in zip(small, refs):
        d = rel_diff(served[f].cpu().numpy(), r)
        assert d <= RESID_TOL, (f, ns[f], d)
