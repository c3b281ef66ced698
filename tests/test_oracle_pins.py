"""Pins of the CPU oracle against facts that do not come from the oracle.

The oracle implements Algorithm 1 (CholeskyModifyB, rank k) of Walder 2010.
These tests tie it to the definition of the result (Section 1: the unique
upper factor of A + sigma V V^T), to closed forms, to invariants and to a
hand-worked example, chosen so that a slip anywhere in Compute or Apply (a
dropped term, a flipped sign, an old value used where the new one belongs,
a swapped index) fails at least one of them.  The last group plants such
slips in a pure-Python copy and checks that the pins catch each one.
"""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def rng_problem(n, k, seed, ldl=None):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    A = G.T @ G + n * np.eye(n)
    U = np.linalg.cholesky(A).T.copy()  # library factor, upper
    ldl = n if ldl is None else ldl
    L = np.zeros((n, ldl))
    L[:, :n] = U
    V = rng.standard_normal((n, k)) / math.sqrt(max(n, 1))
    return L, V


def chol_upper_textbook(A):
    """Plain textbook Cholesky written here (independent of the oracle's)."""
    n = len(A)
    U = [[0.0] * n for _ in range(n)]
    for i in range(n):
        d = A[i][i] - sum(U[p][i] * U[p][i] for p in range(i))
        U[i][i] = math.sqrt(d)
        for j in range(i + 1, n):
            U[i][j] = (A[i][j] - sum(U[p][i] * U[p][j] for p in range(i))) / U[i][i]
    return np.array(U)


def target(L, V, sigma):
    n = L.shape[0]
    U = np.triu(L[:, :n])
    return U.T @ U + sigma * (V @ V.T)


def rel_residual(Lnew, L, V, sigma):
    n = L.shape[0]
    At = target(L, V, sigma)
    U = np.triu(Lnew[:, :n])
    return np.linalg.norm(U.T @ U - At) / np.linalg.norm(At)


# ---------------------------------------------------------------- P1 definition
@pytest.mark.parametrize("n,k,sigma", [(1, 1, 1), (2, 3, 1), (7, 1, -1), (16, 4, 1),
                                       (24, 2, -1), (40, 5, 1), (64, 16, -1), (33, 64, 1)])
def test_p1_matches_library_cholesky_of_target(orc, n, k, sigma):
    L, V = rng_problem(n, k, seed=100 + n + k)
    if sigma < 0:  # downdate of a factor that already contains V V^T
        L[:, :n] = np.linalg.cholesky(target(L, V, +1)).T
    Lnew, st, info = orc.modify(L, V, sigma)
    assert st == 0 and info == -1
    ref = np.linalg.cholesky(target(L, V, sigma)).T
    assert np.all(np.diag(Lnew) > 0)
    np.testing.assert_allclose(np.triu(Lnew), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("n,k,sigma", [(5, 2, 1), (12, 3, -1), (20, 1, 1)])
def test_p1_matches_textbook_cholesky(orc, n, k, sigma):
    L, V = rng_problem(n, k, seed=7 * n + k)
    if sigma < 0:
        L[:, :n] = np.linalg.cholesky(target(L, V, +1)).T
    Lnew, st, _ = orc.modify(L, V, sigma)
    assert st == 0
    ref = chol_upper_textbook(target(L, V, sigma).tolist())
    np.testing.assert_allclose(np.triu(Lnew), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_oracle_cholesky_matches_library(orc):
    L, _ = rng_problem(50, 1, seed=3)
    A = L.T @ L
    U = orc.cholesky_upper(A)
    np.testing.assert_allclose(U, np.linalg.cholesky(A).T, rtol=0, atol=1e-12 * np.abs(U).max())


def test_target_matrix_matches_numpy(orc):
    L, V = rng_problem(30, 3, seed=4, ldl=33)
    L[:, 30:] = np.nan
    L[np.tril_indices(30, -1)] = np.nan
    for s in (1, -1):
        At = orc.target_matrix(L, V, s)
        U = np.triu(np.nan_to_num(L[:, :30]))
        np.testing.assert_allclose(At, U.T @ U + s * V @ V.T, rtol=1e-14, atol=1e-12)


# ---------------------------------------------------------------- P2 residual
@pytest.mark.parametrize("n,k", [(100, 1), (200, 16), (300, 64), (129, 17)])
def test_p2_residual_and_positive_diagonal(orc, n, k):
    L, V = rng_problem(n, k, seed=n + k)
    up, st, _ = orc.modify(L, V, +1)
    assert st == 0
    assert rel_residual(up, L, V, +1) <= 1e-12
    assert np.all(np.diag(up) > 0)
    down, st, _ = orc.modify(up, V, -1)
    assert st == 0
    assert rel_residual(down, up, V, -1) <= 1e-12
    assert np.all(np.diag(down) > 0)


# ---------------------------------------------------------------- P3 rank k == k x rank 1
@pytest.mark.parametrize("n,k,sigma", [(40, 5, 1), (40, 5, -1), (97, 16, 1), (10, 64, 1)])
def test_p3_rank_k_equals_k_sequential_rank_1_bitwise(orc, n, k, sigma):
    L, V = rng_problem(n, k, seed=11 * n + k)
    if sigma < 0:
        L[:, :n] = np.linalg.cholesky(target(L, V, +1)).T
    a, sa, _, Wa = orc.modify(L, V, sigma, return_w=True)
    b, sb, _, Wb = orc.modify(L, V, sigma, seq=True, return_w=True)
    assert sa == sb == 0
    assert np.array_equal(a, b)
    assert np.array_equal(Wa, Wb)


# ---------------------------------------------------------------- P4 round trip
@pytest.mark.parametrize("n,k", [(60, 1), (150, 16), (64, 33)])
def test_p4_update_then_downdate_returns_L(orc, n, k):
    L, V = rng_problem(n, k, seed=5 * n + k)
    up, st, _ = orc.modify(L, V, +1)
    assert st == 0
    back, st, _ = orc.modify(up, V, -1)
    assert st == 0
    rel = np.abs(np.triu(back) - np.triu(L)).max() / np.abs(L).max()
    assert rel <= 1e-13


# ---------------------------------------------------------------- P5 worked example
def test_p5_hand_worked_example_is_exact(orc):
    g = json.load(open(os.path.join(HERE, "golden", "p5_worked_example.json")))
    L = np.array(g["L"])
    V = np.array(g["V"])
    Lnew, st, _, W = orc.modify(L, V, g["sigma"], return_w=True)
    assert st == 0
    assert np.array_equal(Lnew, np.array(g["L_new"]))
    assert np.array_equal(W, np.array(g["W_final"]))


# ---------------------------------------------------------------- P6 closed form, L = I
@pytest.mark.parametrize("n,sigma", [(50, 1), (50, -1), (300, 1)])
def test_p6_identity_closed_form(orc, n, sigma):
    rng = np.random.default_rng(n)
    v = rng.standard_normal(n) / math.sqrt(n) * (0.5 if sigma < 0 else 1.0)
    if sigma < 0:
        assert 1 - np.sum(v * v) > 0.1
    L = np.eye(n)
    Lnew, st, _ = orc.modify(L, v.reshape(n, 1), sigma)
    assert st == 0
    tau = np.concatenate([[0.0], np.cumsum(v * v)])  # tau[i+1] = sum_{r<=i} v_r^2
    expect = np.zeros((n, n))
    for i in range(n):
        expect[i, i] = math.sqrt((1 + sigma * tau[i + 1]) / (1 + sigma * tau[i]))
        denom = math.sqrt((1 + sigma * tau[i]) * (1 + sigma * tau[i + 1]))
        expect[i, i + 1:] = sigma * v[i] * v[i + 1:] / denom
    np.testing.assert_allclose(Lnew, expect, rtol=0, atol=1e-14)


# ---------------------------------------------------------------- P7 row scaling
@pytest.mark.parametrize("r,alpha,sigma", [(0, 0.7, 1), (13, 1.3, 1), (29, 0.6, -1), (5, 0.25, -1)])
def test_p7_row_scaling_closed_form(orc, r, alpha, sigma):
    L, _ = rng_problem(30, 1, seed=9)
    v = alpha * L[r, :].copy()  # V = alpha * (row r of L)^T; zero for columns < r
    Lnew, st, _ = orc.modify(L, v.reshape(-1, 1), sigma)
    assert st == 0
    expect = L.copy()
    expect[r, :] *= math.sqrt(1 + sigma * alpha * alpha)
    # rows before r see v = 0 exactly and must be untouched bit for bit
    assert np.array_equal(Lnew[:r], L[:r])
    np.testing.assert_allclose(Lnew, expect, rtol=0, atol=1e-13 * np.abs(L).max())


# ---------------------------------------------------------------- P8 trivial cases
def test_p8_zero_V_is_bitwise_noop(orc):
    L, _ = rng_problem(37, 1, seed=1)
    for s in (1, -1):
        out, st, _ = orc.modify(L, np.zeros((37, 4)), s)
        assert st == 0 and np.array_equal(out, L)


def test_p8_empty_and_n1(orc):
    out, st, _ = orc.modify(np.zeros((0, 1)), np.zeros((0, 3)), 1)
    assert st == 0 and out.shape == (0, 1)
    L, V = rng_problem(8, 1, seed=2)
    out, st, _ = orc.modify(L, np.zeros((8, 0)), 1)
    assert st == 0 and np.array_equal(out, L)
    # n = 1: L~ = sqrt(L^2 + sigma |V|^2); 3-4-5 and 5-12-13 keep every step exact
    out, st, _ = orc.modify(np.array([[3.0]]), np.array([[4.0, 12.0]]), 1)
    assert st == 0 and out[0, 0] == 13.0
    out, st, _ = orc.modify(np.array([[5.0]]), np.array([[3.0]]), -1)
    assert st == 0 and out[0, 0] == 4.0


def test_bad_arguments(orc):
    L = np.eye(3)
    V = np.ones((3, 1))
    assert orc.modify(L, V, 0)[1] == orc.ARG
    assert orc.modify(L, V, 2)[1] == orc.ARG


# ---------------------------------------------------------------- P9 homogeneity
@pytest.mark.parametrize("e", [-3, 5, 20])
def test_p9_power_of_two_scaling_is_bitwise(orc, e):
    L, V = rng_problem(45, 7, seed=21)
    a, _, _ = orc.modify(L, V, 1)
    b, _, _ = orc.modify(L * 2.0 ** e, V * 2.0 ** e, 1)
    assert np.array_equal(a * 2.0 ** e, b)


# ---------------------------------------------------------------- P10 failure
@pytest.mark.parametrize("r", [0, 1, 17, 39])
def test_p10_indefinite_downdate_reports_first_failure(orc, r):
    L, _ = rng_problem(40, 1, seed=33)
    k = 3
    V = np.zeros((40, k))
    V[:, 0] = 2.0 * L[r, :]  # t = L_rr^2 (1 - 4) < 0 at (r, 0)
    V[:, 1] = 0.01           # other columns are harmless
    V[:r, 1] = 0.0
    out, st, info = orc.modify(L, V, -1)
    assert st == orc.NOT_PD
    assert info == r * k + 0
    # rows before r had v = 0 in every column: untouched
    assert np.array_equal(out[:r], L[:r])
    out, st, info = orc.modify(L, V, -1, seq=True)
    assert st == orc.NOT_PD and info == r * k + 0


def test_bad_diagonal(orc):
    L, V = rng_problem(10, 2, seed=4)
    L[6, 6] = -1.0
    _, st, info = orc.modify(L, V, 1)
    assert st == orc.BAD_DIAG and info == 6 * 2 + 0
    L[6, 6] = np.nan
    _, st, info = orc.modify(L, V, 1)
    assert st == orc.BAD_DIAG and info == 12


def test_singular_downdate_is_reported(orc):
    # A~ = 0 exactly in the first pivot: t = 1 - 1 = 0 is not > 0
    L = np.eye(3)
    V = np.zeros((3, 1))
    V[0, 0] = 1.0
    _, st, info = orc.modify(L, V, -1)
    assert st == orc.NOT_PD and info == 0


# ---------------------------------------------------------------- P11 untouched memory
def test_p11_lower_triangle_and_padding_untouched(orc):
    n, ldl = 23, 29
    L, V = rng_problem(n, 4, seed=8, ldl=ldl)
    L[:, n:] = np.nan
    L[np.tril_indices(n, -1)] = np.nan
    out, st, _ = orc.modify(L, V, 1)
    assert st == 0
    assert np.isnan(out[:, n:]).all()
    assert np.isnan(out[np.tril_indices(n, -1)]).all()
    assert not np.isnan(out[np.triu_indices(n)]).any()


# ---------------------------------------------------------------- P12 second form
@pytest.mark.parametrize("n,k,sigma", [(40, 5, 1), (33, 2, -1), (64, 16, 1)])
def test_p12_corrected_modifyA_equals_modifyB_bitwise(orc, n, k, sigma):
    L, V = rng_problem(n, k, seed=n * k)
    if sigma < 0:
        L[:, :n] = np.linalg.cholesky(target(L, V, +1)).T
    a, sa, _ = orc.modify(L, V, sigma)
    b, sb, _ = orc.modify_colA(L, V, sigma)
    assert sa == sb == 0
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- the pins catch slips
def _py_modify(L, V, sigma, slip=None):
    """Pure-Python CholeskyModifyB with an optional planted slip."""
    L = L.copy()
    W = V.copy()
    n, k = W.shape
    for i in range(n):
        cs = []
        for m in range(k):
            l, v = L[i, i], W[i, m]
            t = l * l + (sigma * v * v if slip != "drop_sigma" else v * v)
            w = math.sqrt(t)
            c = w / l if slip != "c_new_diag" else w / w
            s = v / l if slip != "s_over_w" else v / w
            L[i, i] = w
            cs.append((c, s))
        for j in range(i + 1, n):
            for m in range(k):
                c, s = cs[m]
                old = L[i, j]
                if slip == "sign_apply":
                    L[i, j] = (L[i, j] - sigma * s * W[j, m]) / c
                else:
                    L[i, j] = (L[i, j] + sigma * s * W[j, m]) / c
                if slip == "old_L_in_V":
                    W[j, m] = c * W[j, m] - s * old
                elif slip == "transposed":
                    W[j, m] = c * W[j, m] - s * L[j, i]
                else:
                    W[j, m] = c * W[j, m] - s * L[i, j]
    return L


@pytest.mark.parametrize("slip", [None, "drop_sigma", "c_new_diag", "s_over_w", "sign_apply",
                                  "old_L_in_V", "transposed"])
def test_pins_detect_planted_slips(orc, slip):
    n, k = 12, 3
    L, V = rng_problem(n, k, seed=77)
    caught = []
    for sigma in (1, -1):
        L0 = L.copy()
        if sigma < 0:
            L0[:, :n] = np.linalg.cholesky(target(L, V, +1)).T
        out = _py_modify(L0, V, sigma, slip)
        ref = np.linalg.cholesky(target(L0, V, sigma)).T
        caught.append(not np.allclose(np.triu(out), ref, rtol=0, atol=1e-12 * np.abs(ref).max()))
    if slip is None:
        assert not any(caught)
        # the clean Python copy also agrees with the C oracle to rounding
        c_out, _, _ = orc.modify(L, V, 1)
        np.testing.assert_allclose(_py_modify(L, V, 1), c_out, rtol=0, atol=1e-14 * np.abs(L).max())
    else:
        assert any(caught), "pin P1 did not catch slip %s" % slip
