"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds no arithmetic of the DPar2 method itself: it only draws
irregular tensors with PARAFAC2 structure (Definition 1 of the paper; the
reformulated model with U_k = Q_k H of the PARAFAC2-ALS section), the Gaussian
test matrices Omega that the randomized SVD (Alg. 1) draws, and initial
factors (Alg. 3 starts from caller-chosen H, V, S_k).  Both sides receive the
same float32 arrays, so any difference between them comes from the method.

Layout of an irregular tensor {X_k}, k = 0..K-1, X_k in R^{I_k x J}:
  slab     float32 (N, J) row-major, N = sum_k I_k, slice k = rows
           offsets[k] .. offsets[k+1]-1
  offsets  int64 (K+1,), offsets[0] = 0, non-decreasing
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class IrregularTensor:
    slab: np.ndarray          # float32 (N, J)
    offsets: np.ndarray       # int64 (K+1,)
    H: np.ndarray | None = None   # generating factors (float64), when known
    V: np.ndarray | None = None
    W: np.ndarray | None = None

    @property
    def K(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def J(self) -> int:
        return int(self.slab.shape[1])

    @property
    def N(self) -> int:
        return int(self.slab.shape[0])

    @property
    def rows(self) -> np.ndarray:
        return np.diff(self.offsets)

    def slice(self, k: int) -> np.ndarray:
        return self.slab[self.offsets[k]:self.offsets[k + 1]]


def _orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Haar-like random column-orthonormal matrix (QR of a Gaussian matrix,
    columns signed so that diag(R) > 0)."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))


def _offsets(rows: np.ndarray) -> np.ndarray:
    off = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(rows, out=off[1:])
    return off


def parafac2(rows, J: int, rank: int, seed, *, noise_abs: float = 0.0,
             noise_rel: float = 0.0, col_scale_decades: tuple | None = None,
             w_range=(0.5, 1.5)) -> IrregularTensor:
    """X_k = Q_k H diag(W(k,:)) V^T (optionally times diag(c) over columns)
    plus Gaussian noise.

    Q_k: random column-orthonormal I_k x rank; H (rank x rank), V (J x rank)
    i.i.d. N(0,1); W (K x rank) i.i.d. U(w_range).
    noise_abs: i.i.d. N(0, noise_abs^2) added to every entry.
    noise_rel: per-column N(0, (noise_rel * rms_j)^2), rms_j the RMS of clean
               column j over all slices.
    col_scale_decades=(lo, hi): column j scaled by 10^U(lo, hi).
    """
    rng = np.random.default_rng(seed)
    rows = np.asarray(rows, dtype=np.int64)
    K = rows.shape[0]
    off = _offsets(rows)
    N = int(off[-1])
    H = rng.standard_normal((rank, rank))
    V = rng.standard_normal((J, rank))
    W = rng.uniform(w_range[0], w_range[1], size=(K, rank))
    if col_scale_decades is not None:
        c = 10.0 ** rng.uniform(col_scale_decades[0], col_scale_decades[1], size=J)
        Vs = V * c[:, None]
    else:
        Vs = V
    slab = np.empty((N, J), dtype=np.float32)
    colsq = np.zeros(J)
    for k in range(K):
        Q = _orthonormal(rng, int(rows[k]), rank)
        Xk = (Q @ (H * W[k][None, :])) @ Vs.T
        slab[off[k]:off[k + 1]] = Xk
        colsq += np.einsum("ij,ij->j", Xk, Xk)
    if noise_rel > 0.0:
        std = noise_rel * np.sqrt(colsq / max(N, 1))
        for k in range(K):
            blk = slab[off[k]:off[k + 1]]
            blk += (rng.standard_normal(blk.shape, dtype=np.float32)
                    * std[None, :].astype(np.float32))
    if noise_abs > 0.0:
        for k in range(K):
            blk = slab[off[k]:off[k + 1]]
            blk += np.float32(noise_abs) * rng.standard_normal(blk.shape, dtype=np.float32)
    return IrregularTensor(slab=slab, offsets=off, H=H, V=Vs, W=W)


# ---------------------------------------------------------------------------
# Workloads.  Each stands in for one shape the paper evaluates on (its real
# datasets are not available); sizes follow the configurations the build is
# measured on.
# ---------------------------------------------------------------------------

def small_parity(seed: int = 1, K: int = 64, J: int = 32, rank: int = 5,
                 imin: int = 50, imax: int = 200, noise: float = 0.01) -> IrregularTensor:
    """K=64 slices, J=32, I_k ~ U{50..200}, rank-5 PARAFAC2 + N(0, 0.01^2)."""
    rng = np.random.default_rng([seed, 101])
    rows = rng.integers(imin, imax + 1, size=K)
    return parafac2(rows, J, rank, seed, noise_abs=noise)


def stock_like_rows(K: int, seed: int, median: float = 1500.0, sigma: float = 0.7,
                    lo: int = 200, hi: int = 8000) -> np.ndarray:
    """Row counts I_k = clip(round(exp(N(ln median, sigma^2))), lo, hi): a
    long-tailed length mix like daily stock histories of uneven age."""
    rng = np.random.default_rng([seed, 202])
    r = np.exp(rng.normal(math.log(median), sigma, size=K))
    return np.clip(np.round(r), lo, hi).astype(np.int64)


def stock_like(seed: int = 2, K: int = 4000, J: int = 88, rank: int = 10,
               median: float = 1500.0) -> IrregularTensor:
    """US-Stock-shaped tensor: K=4000 stocks x J=88 features, lognormal
    history lengths in [200, 8000] (median 1500), rank-10 PARAFAC2 with
    feature scales spread over 1e-2..1e3 and 5% per-feature Gaussian noise."""
    rows = stock_like_rows(K, seed, median=median)
    return parafac2(rows, J, rank, seed, noise_rel=0.05, col_scale_decades=(-2.0, 3.0))


def uniform_rows(K: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 303])
    return rng.integers(lo, hi + 1, size=K).astype(np.int64)


def exact_parafac2(seed: int, K: int, J: int, rank: int, imin: int, imax: int) -> IrregularTensor:
    """Noise-free PARAFAC2 tensor (every slice has rank `rank` exactly)."""
    return parafac2(uniform_rows(K, imin, imax, seed), J, rank, seed)


# ---------------------------------------------------------------------------
# Random inputs the method draws: Gaussian test matrices and initial factors.
# ---------------------------------------------------------------------------

def omegas(J: int, L: int, KR: int, L2: int | None = None, seed: int = 0):
    """Omega_1 (J x L) for the per-slice randomized SVDs (one matrix shared by
    all slices) and Omega_2 (KR x L2) for the second-stage randomized SVD,
    both i.i.d. N(0,1), drawn in that order from default_rng(seed), rounded to
    float32."""
    L2 = L if L2 is None else L2
    rng = np.random.default_rng(seed)
    om1 = rng.standard_normal((J, L)).astype(np.float32)
    om2 = rng.standard_normal((KR, L2)).astype(np.float32)
    return om1, om2


def init_factors(J: int, K: int, R: int, seed: int = 7):
    """H = I_R, V ~ N(0,1) (J x R) from default_rng(seed), W = 1 (K x R);
    all float64 (S_k = diag(W(k,:)))."""
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((J, R))
    return np.eye(R), V, np.ones((K, R))


# ---------------------------------------------------------------------------
# Low-precision encodings of a slab (input formats, not part of the method):
# the GPU reads the encoded bytes, the oracle the decoded values.
# ---------------------------------------------------------------------------

def round_bf16(x: np.ndarray) -> np.ndarray:
    """float32 values rounded to the nearest bfloat16 (ties to even), as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def encode_bf16(x: np.ndarray) -> np.ndarray:
    """uint16 bfloat16 bit patterns of x (round to nearest even)."""
    return (round_bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def decode_bf16(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def _e4m3_table() -> np.ndarray:
    """Values of the 256 OCP fp8 e4m3fn codes (bias 7, S.1111.111 = NaN)."""
    v = np.zeros(256)
    for c in range(256):
        s, e, m = c >> 7, (c >> 3) & 15, c & 7
        if e == 15 and m == 7:
            v[c] = np.nan
            continue
        mag = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
        v[c] = -mag if s else mag
    return v


E4M3 = _e4m3_table()
E4M3_MAX = 448.0


def encode_fp8(slab: np.ndarray, offsets: np.ndarray):
    """Per-slice scaled fp8 e4m3 codes: scale_k = 2^ceil(log2(amax_k / 448))
    (a power of two, so decode(code) * scale_k is exact in float32), codes the
    nearest representable value of x / scale_k (ties to the even code).
    Returns (uint8 codes N x J, float32 scales K)."""
    x = np.asarray(slab, dtype=np.float64)
    K = len(offsets) - 1
    scale = np.ones(K, dtype=np.float32)
    pos = E4M3[:127]                       # codes 0x00..0x7E, increasing
    codes = np.zeros(x.shape, dtype=np.uint8)
    for k in range(K):
        blk = x[offsets[k]:offsets[k + 1]]
        amax = float(np.max(np.abs(blk))) if blk.size else 0.0
        sc = 2.0 ** math.ceil(math.log2(amax / E4M3_MAX)) if amax > 0 else 1.0
        scale[k] = sc
        a = np.minimum(np.abs(blk) / sc, E4M3_MAX)
        i = np.clip(np.searchsorted(pos, a), 1, 126)
        lo, hi = pos[i - 1], pos[i]
        pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & ((i & 1) == 0))
        c = np.where(pick_hi, i, i - 1).astype(np.uint8)
        c = np.where(a <= 0, 0, c).astype(np.uint8)
        codes[offsets[k]:offsets[k + 1]] = c | np.where(blk < 0, 0x80, 0).astype(np.uint8)
    return codes, scale


def decode_fp8(codes: np.ndarray, offsets: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """float32 values decode(code) * scale_k (exact: scales are powers of two)."""
    v = E4M3[np.asarray(codes, dtype=np.uint8)].astype(np.float32)
    rows = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    return (v * np.asarray(scale, dtype=np.float32)[rows][:, None]).astype(np.float32)
