"""Shared helpers for the GPU parity tests (inputs, residuals, comparisons)."""
import math
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1011_1173_amd import inputs  # noqa: E402

# FP64 acceptance bound for the relative residual ||L~^T L~ - A~||_F / ||A~||_F
# and for the relative distance to the oracle's factor (fast mode).
RESID_TOL = 1e-12


def problem(n, k, seed, ldl=None):
    """Seeded (L, V) as numpy arrays (L = upper factor of G^T G + n I, V ~
    N(0, 1)/sqrt(n)).  For a well-posed downdate by V, callers first add V V^T
    with the oracle's own update."""
    L = inputs.spd_factor(n, seed, ldl=ldl).numpy()
    V = inputs.update_vectors(n, k, seed).numpy()
    return L, V


def run_gpu(L, V, sigma, **kw):
    """Run the HIP path on copies of (L, V); return (L_new, status, row, col)."""
    import paper_1011_1173_amd as chm
    Ld = torch.from_numpy(np.ascontiguousarray(L)).cuda()
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    pend = chm.update_async(Ld, Vd, sigma, **kw)
    st, row, col = pend.status()
    return Ld.cpu().numpy(), st, row, col


def rel_residual_gpu(Lnew, L, V, sigma):
    """||U~^T U~ - (U^T U + sigma V V^T)||_F / ||.||_F with library FP64 GEMMs."""
    n = L.shape[0]
    dev = "cuda" if torch.cuda.is_available() else "cpu"
    U = torch.triu(torch.from_numpy(np.ascontiguousarray(L[:, :n])).to(dev))
    Un = torch.triu(torch.from_numpy(np.ascontiguousarray(Lnew[:, :n])).to(dev))
    Vt = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    At = U.T.contiguous() @ U + sigma * (Vt @ Vt.T.contiguous())
    R = Un.T.contiguous() @ Un - At
    return float(torch.linalg.norm(R) / torch.linalg.norm(At))


def rel_diff(a, b):
    a = np.triu(a[:, :a.shape[0]])
    b = np.triu(b[:, :b.shape[0]])
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def print_case(name, **kw):
    print("[case] %s %s" % (name, " ".join("%s=%s" % kv for kv in kw.items())), flush=True)


def oracle_sequences(orc, starts, seqs, workers=8):
    """Apply each factor's request sequence [(V, sigma), ...] to its starting
    factor with the oracle, in order; factors run in parallel host threads
    (the oracle releases the GIL).  Returns the final factors (numpy)."""
    from concurrent.futures import ThreadPoolExecutor

    def run(args):
        L, seq = args
        for V, sg in seq:
            L, st, _ = orc.modify(L, V, sg)
            assert st == 0
        return L

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(run, zip(starts, seqs)))
