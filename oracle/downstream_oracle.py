"""FP64 CPU oracle of the post-processing the paper applies to DPar2's factors
(Jang & Kang, arXiv 2203.12798, Sec. IV-E "Discovery").

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path never calls it and
shares no code with it.

  feature_pcc    Sec. IV-E, feature similarity: Pearson correlation coefficient
                 between the latent vectors V(i,:) of every pair of features
  similarity     Eq. 9: sim(s_i, s_j) = exp(-gamma ||U_si - U_sj||_F^2) between
                 slices of the same length
  top_k          the k most similar items (k-nearest neighbours of Sec. IV-E)
  rwr            random walk with restart on the similarity graph (Eqs. 10-11):
                 A(i,j) = sim(s_i, s_j) for i != j, 0 on the diagonal;
                 r <- (1 - c) A~^T r + c q with A~ the row-normalised A

Readings where the paper is silent (also listed in the design notes):
  * a feature whose latent vector is constant (zero variance) has no defined
    correlation: its row and column of the PCC matrix are 0 (its diagonal
    entry too);
  * the RWR iteration starts from r = q; a node whose row of A sums to zero
    keeps a zero row in A~;
  * ranking ties go to the lower index; the target itself is excluded from
    its own top-k.
"""
from __future__ import annotations

import numpy as np


def feature_pcc(V: np.ndarray) -> np.ndarray:
    """Pearson correlation between rows of V (J x R): C[a, b] =
    sum_r (V[a,r] - mean_a)(V[b,r] - mean_b) / sqrt(sum (V[a]-mean_a)^2 sum (V[b]-mean_b)^2)."""
    V = np.asarray(V, dtype=np.float64)
    J, R = V.shape
    C = np.zeros((J, J))
    means = [sum(V[a, r] for r in range(R)) / R for a in range(J)]
    dev = [[V[a, r] - means[a] for r in range(R)] for a in range(J)]
    ss = [sum(d * d for d in dev[a]) for a in range(J)]
    for a in range(J):
        for b in range(J):
            if ss[a] > 0.0 and ss[b] > 0.0:
                C[a, b] = sum(dev[a][r] * dev[b][r] for r in range(R)) / np.sqrt(ss[a] * ss[b])
    return C


def similarity(U: list, idx, gamma: float) -> np.ndarray:
    """Eq. 9 between the slices listed in idx (all of the same number of
    rows): S[i, j] = exp(-gamma ||U[idx[i]] - U[idx[j]]||_F^2)."""
    n = len(idx)
    S = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            Di = np.asarray(U[idx[i]], dtype=np.float64) - np.asarray(U[idx[j]], dtype=np.float64)
            S[i, j] = np.exp(-gamma * float(np.sum(Di * Di)))
    return S


def top_k(values, exclude: int, k: int):
    """Indices of the k largest values, the entry `exclude` left out; ties go
    to the lower index."""
    order = sorted((i for i in range(len(values)) if i != exclude), key=lambda i: (-values[i], i))
    return order[:k]


def rwr(S: np.ndarray, target: int, c: float = 0.15, iters: int = 100) -> np.ndarray:
    """Random walk with restart (Eqs. 10-11) on the graph with adjacency
    A(i,j) = S(i,j) for i != j and A(i,i) = 0; A~ is A with each row divided
    by its sum (zero rows stay zero); q = e_target; r starts at q and takes
    `iters` steps of r <- (1 - c) A~^T r + c q."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    A = S.copy()
    np.fill_diagonal(A, 0.0)
    d = A.sum(axis=1)
    At = np.zeros_like(A)
    for i in range(n):
        if d[i] > 0.0:
            At[i] = A[i] / d[i]
    q = np.zeros(n)
    q[target] = 1.0
    r = q.copy()
    for _ in range(iters):
        r = (1.0 - c) * (At.T @ r) + c * q
    return r
