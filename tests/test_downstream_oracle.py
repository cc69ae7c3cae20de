"""Pins of the post-processing oracle (Sec. IV-E; oracle/downstream_oracle.py)
against values fixed by hand or by the mathematics, each shown to reject a
plausibly broken copy of the function kept here as a fixture.  CPU only."""
import math

import numpy as np
import pytest

from oracle import downstream_oracle as D


# ---- broken copies (each must fail at least one pin) ------------------------

def pcc_uncentred(V):
    """cosine similarity of the rows (centering forgotten)"""
    V = np.asarray(V, dtype=np.float64)
    n = np.linalg.norm(V, axis=1)
    n = np.where(n > 0, n, 1.0)
    return (V / n[:, None]) @ (V / n[:, None]).T


def similarity_unsquared(U, idx, gamma):
    n = len(idx)
    return np.array([[math.exp(-gamma * np.linalg.norm(U[idx[i]] - U[idx[j]])) for j in range(n)] for i in range(n)])


def rwr_untransposed(S, target, c=0.15, iters=100):
    """A~ r instead of A~^T r"""
    A = np.asarray(S, dtype=np.float64).copy()
    np.fill_diagonal(A, 0.0)
    At = A / A.sum(axis=1, keepdims=True)
    q = np.zeros(A.shape[0])
    q[target] = 1.0
    r = q.copy()
    for _ in range(iters):
        r = (1 - c) * (At @ r) + c * q
    return r


def top_k_unstable(values, exclude, k):
    """ties to the higher index"""
    order = sorted((i for i in range(len(values)) if i != exclude), key=lambda i: (-values[i], -i))
    return order[:k]


# ---- pins --------------------------------------------------------------------

V_HAND = np.array([[1.0, 2.0, 3.0],    # a
                   [1.0, 0.0, -1.0],   # b: centred b = -centred a
                   [2.0, 2.0, 5.0],    # c: centred (-1, -1, 2)
                   [4.0, 4.0, 4.0]])   # d: constant (no correlation defined)


def _pcc_pins(f):
    C = f(V_HAND)
    # by hand: corr(a, b) = -1; corr(a, c) = 3 / sqrt(2 * 6); corr(b, c) = -3 / sqrt(12)
    assert abs(C[0, 1] + 1.0) < 1e-14
    assert abs(C[0, 2] - 3.0 / math.sqrt(12.0)) < 1e-14
    assert abs(C[1, 2] + 3.0 / math.sqrt(12.0)) < 1e-14
    assert np.all(C[3] == 0.0) and np.all(C[:, 3] == 0.0)
    assert np.allclose(np.diag(C)[:3], 1.0, atol=1e-15)
    # invariance: row a scaled by -2.5 and shifted by 7 flips the sign of its correlations
    V2 = V_HAND.copy()
    V2[0] = -2.5 * V2[0] + 7.0
    C2 = f(V2)
    assert np.allclose(C2[0, 1:3], -C[0, 1:3], atol=1e-14)


def test_feature_pcc_pins():
    _pcc_pins(D.feature_pcc)
    with pytest.raises(AssertionError):
        _pcc_pins(pcc_uncentred)


U_HAND = [np.zeros((3, 2)), np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]]),
          2.0 * np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])]


def _sim_pins(f):
    S = f(U_HAND, [0, 1, 2], 0.01)
    # ||U1 - U0||^2 = 2, ||U2 - U0||^2 = 8, ||U2 - U1||^2 = 2 (Eq. 9 with gamma = 0.01)
    assert abs(S[0, 1] - math.exp(-0.02)) < 1e-15
    assert abs(S[0, 2] - math.exp(-0.08)) < 1e-15
    assert abs(S[1, 2] - math.exp(-0.02)) < 1e-15
    assert np.all(np.diag(S) == 1.0) and np.array_equal(S, S.T)


def test_similarity_pins():
    _sim_pins(D.similarity)
    with pytest.raises(AssertionError):
        _sim_pins(similarity_unsquared)


def _topk_pins(f):
    assert f([0.5, 0.9, 0.9, 0.1, 0.7], 1, 3) == [2, 4, 0]
    assert f([0.3, 0.3, 0.3, 0.3], 0, 2) == [1, 2]
    assert f([1.0, 2.0], 1, 5) == [0]


def test_top_k_pins():
    _topk_pins(D.top_k)
    with pytest.raises(AssertionError):
        _topk_pins(top_k_unstable)


def _rwr_pins(f):
    c = 0.15
    # two nodes: r0 = c + (1 - c) r1, r1 = (1 - c) r0 (fixed point), converged
    # to (1 - c)^100 after 100 steps
    r = f(np.array([[1.0, 0.4], [0.4, 1.0]]), 0, c, 100)
    r0 = c / (1.0 - (1.0 - c) ** 2)
    assert abs(r[0] - r0) < 1e-6 and abs(r[1] - (1.0 - c) * r0) < 1e-6
    # three nodes of unequal degree: the fixed point of r = (1 - c) A~^T r + c q,
    # A~ the row-normalised adjacency worked out by hand
    S = np.array([[1.0, 0.8, 0.1], [0.8, 1.0, 0.5], [0.1, 0.5, 1.0]])
    At = np.array([[0.0, 0.8 / 0.9, 0.1 / 0.9], [0.8 / 1.3, 0.0, 0.5 / 1.3], [0.1 / 0.6, 0.5 / 0.6, 0.0]])
    q = np.array([0.0, 0.0, 1.0])
    star = np.linalg.solve(np.eye(3) - (1.0 - c) * At.T, c * q)
    r = f(S, 2, c, 200)
    assert np.abs(r - star).max() < 1e-12
    # probability mass is kept (every row of A has a positive sum)
    assert abs(np.sum(f(S, 1, c, 37)) - 1.0) < 1e-14


def test_rwr_pins():
    _rwr_pins(D.rwr)
    with pytest.raises(AssertionError):
        _rwr_pins(rwr_untransposed)


def test_rwr_isolated_node_keeps_zero_row():
    """A node with no edges (all similarities 0) gives no mass to anyone: with
    it as the target, r = c q after every step."""
    S = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.7], [0.0, 0.7, 1.0]])
    r = D.rwr(S, 0, 0.15, 10)
    assert np.allclose(r, [0.15, 0.0, 0.0], atol=0.0)
