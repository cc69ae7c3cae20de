"""Comparison helpers shared by the GPU parity tests (gauge handling only)."""
import numpy as np


def model_tensor(H, V, W):
    """H S_k V^T for all k: (K, R, J).  Invariant to column scaling/sign gauges."""
    return np.einsum("ir,kr,jr->kij", H, W, V)


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def canonical(H, V, W):
    """Unit-norm columns of H and V (scale into W); the largest-magnitude entry
    of each V and H column positive (sign into W)."""
    H = np.array(H, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    nh = np.linalg.norm(H, axis=0)
    nv = np.linalg.norm(V, axis=0)
    H, V, W = H / nh, V / nv, W * (nh * nv)[None, :]
    for M in (V, H):
        s = np.sign(M[np.argmax(np.abs(M), axis=0), np.arange(M.shape[1])])
        s[s == 0] = 1
        M *= s[None, :]
        W *= s[None, :]
    return H, V, W


def match_columns(A, B):
    """Signs that best align the columns of A with those of B."""
    s = np.sign(np.sum(A * B, axis=0))
    s[s == 0] = 1
    return s
