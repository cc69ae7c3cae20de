#!/usr/bin/env python3
"""Derives the parity bounds of the GPU tests from a CPU emulation of the slab
pass's rounding, and writes them to parity_bounds.json next to this file.

TEST INFRASTRUCTURE: calls only the FP64 oracle and the seeded generators.

What the emulation models.  The whole-row slab pass of the library forms the
sketch Y = X Omega_1 (Alg. 1's first product) with float32-level error, then
represents Y and X in 22-bit fixed point per column of each 64-row tile (the
power of two 2^(22 - e) with |column| < 2^e in that tile, round to nearest
even) and forms Y^T Y and Y^T X of those rounded values exactly.  Everything
after the Gram and the projection runs in FP64 (Cholesky whitening,
B_k = R^-T (Y^T X), the small SVD, the second stage and the iteration), so
the GPU's compressed data are, to FP64 rounding, the exact randomized SVD of
the rounded pair (Yq, Xq).  This script computes exactly that with NumPy
(Yq, Xq as described; Y rounded to float32 after an FP64 product), runs the
oracle's second stage and iteration on it, and compares with the plain
oracle on the same inputs.  With a power step (q = 1) the next sketch matrix
of each slice is its right singular basis of B rounded to float32, as the
library writes it for the second slab pass.  The deviations it reports are what the GPU's
arithmetic is expected to produce; the tests allow a factor SAFETY above the
largest deviation seen over the cases of one check (and never less than the
floor given per check).

Usage:  python tests/golden/derive_parity_bounds.py   (about a minute)
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dpar2_oracle as O  # noqa: E402

TM = 64            # rows per tile of the slab pass
ITEM = 16384       # longest work item (rows); longer slices are cut evenly
FRAC_BITS = 22     # fixed-point bits per tile column
SAFETY = 4.0


def tile_round(A: np.ndarray, starts) -> np.ndarray:
    """22-bit fixed point per column of each 64-row tile, tiles starting at
    every item start and every 64 rows after it."""
    out = np.empty_like(A, dtype=np.float64)
    for s0, s1 in starts:
        for r0 in range(s0, s1, TM):
            r1 = min(r0 + TM, s1)
            blk = np.asarray(A[r0:r1], dtype=np.float64)
            m = np.max(np.abs(blk), axis=0)
            e = np.where(m > 0, np.floor(np.log2(np.where(m > 0, m, 1.0))) + 1, 0)
            sc = 2.0 ** (FRAC_BITS - e)
            out[r0:r1] = np.round(blk * sc[None, :]) / sc[None, :]   # numpy rounds half to even
    return out


def item_ranges(n: int):
    nc = max(1, (n + ITEM - 1) // ITEM)
    return [(n * c // nc, n * (c + 1) // nc) for c in range(nc)]


def emulated_stage1(Xk: np.ndarray, omega: np.ndarray, R: int, q: int = 0):
    """(A_k, sigma, C_k) as the slab pass and the per-slice FP64 completion
    compute them: exact randomized SVD of the rounded (Y, X) pair.  With q
    power steps, each step's sketch matrix is the slice's right singular
    basis of B (all L columns; those of a singular value below 64 eps of the
    largest set to zero) rounded to float32, as the completion writes it for
    the next slab pass."""
    X = np.asarray(Xk, dtype=np.float64)
    starts = item_ranges(X.shape[0])
    Xq = tile_round(X, starts)
    om = np.asarray(omega, dtype=np.float64)
    for step in range(q + 1):
        Y = (X @ om).astype(np.float32).astype(np.float64)
        Yq = tile_round(Y, starts)
        G = Yq.T @ Yq
        P = Yq.T @ Xq
        Rc = np.linalg.cholesky(G).T            # G = Rc^T Rc
        B = np.linalg.solve(Rc.T, P)            # Q^T X with Q = Yq Rc^-1
        Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
        if step < q:
            keep = s > 64.0 * np.finfo(np.float64).eps * s[0]
            om = (Vt.T * keep[None, :]).astype(np.float32).astype(np.float64)
    V = Vt[:R].T
    sg = np.sign(V[np.argmax(np.abs(V), axis=0), np.arange(R)])
    sg[sg == 0] = 1.0
    A = (Yq @ np.linalg.solve(Rc, Ut[:, :R])) * sg[None, :]
    return A, s[:R], V * sg[None, :]


def emulated_dpar2(X, R, om1, om2, H0, V0, W0, iters, q=0):
    K, J = X.K, X.J
    A, C, Bd = [], [], np.zeros((K, R))
    xn = np.zeros(K)
    for k in range(K):
        Xk = X.slice(k)
        a, s, c = emulated_stage1(Xk, om1, R, q)
        A.append(a)
        C.append(c)
        Bd[k] = s
        xn[k] = float(np.sum(np.asarray(Xk, dtype=np.float64) ** 2))
    M = np.zeros((J, K * R))
    for k in range(K):
        M[:, k * R:(k + 1) * R] = C[k] * Bd[k][None, :]
    D, E, F = O.randomized_svd(M, R, om2, 0)
    comp = O.Compressed(A=A, Bdiag=Bd, C=C, M=M, D=D, E=E, F=F, xnorm2=xn)
    st = O.als_compressed(comp, H0, V0, W0, iters)
    U = O.output_U(comp, st)
    # the library's fitness (Sec. IV-A) never revisits the slab: it uses
    # A_k^T X_k = (C_k B_k)^T, which holds for the represented slab, so
    # sum_k ||X_k - U_k S_k V^T||^2 = sum_k ||X_k||^2
    #   - 2 sum_k tr(V S_k H^T Psi_k^T (C_k B_k)^T) + sum_k ||H S_k V^T||^2
    res = float(np.sum(xn))
    for k in range(K):
        Psi = st.Z[k] @ st.P[k].T
        CB = C[k] * Bd[k][None, :]
        res -= 2.0 * float(np.trace(st.V @ np.diag(st.W[k]) @ st.H.T @ Psi.T @ CB.T))
        Gk = st.H @ np.diag(st.W[k]) @ st.V.T
        res += float(np.sum(Gk * Gk))
    return comp, st, U, 1.0 - res / float(np.sum(xn))


def canonical(H, V, W):
    H, V, W = (np.array(a, dtype=np.float64) for a in (H, V, W))
    nh, nv = np.linalg.norm(H, axis=0), np.linalg.norm(V, axis=0)
    H, V, W = H / nh, V / nv, W * (nh * nv)[None, :]
    for Mx in (V, H):
        s = np.sign(Mx[np.argmax(np.abs(Mx), axis=0), np.arange(Mx.shape[1])])
        s[s == 0] = 1
        Mx *= s[None, :]
        W *= s[None, :]
    return H, V, W


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def row_rel(a, b):
    """max over rows of ||a_i - b_i|| / ||b_i||"""
    nb = np.linalg.norm(b, axis=1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.where(nb > 0, nb, 1.0)))


def outlier_tile(seed=4):
    """The small parity tensor with row 10 of slice 0 scaled by 1e4: one row
    dominates every column of its 64-row tile."""
    X = synth.small_parity(seed=seed)
    slab = X.slab.copy()
    slab[X.offsets[0] + 10] *= np.float32(1e4)
    return synth.IrregularTensor(slab=slab, offsets=X.offsets)


def c4_rank20(seed=41):
    """A batching-form tensor at the largest rank: K=24, J=128, I_k in
    [32, 600], rank 20 + N(0, 0.05^2), R=20, L=30."""
    rows = synth.uniform_rows(24, 32, 600, seed)
    return synth.parafac2(rows, 128, 20, seed, noise_abs=0.05)


def rank20_long_j(seed=520):
    """Rank 20 at J = 520 (the second stage's J-long steps on one wave per
    64 rows, the wide slab pass at L = 30): K=12, I_k in [60, 200],
    N(0, 0.02^2) noise, R=20, L=30."""
    rows = synth.uniform_rows(12, 60, 200, seed)
    return synth.parafac2(rows, 520, 20, seed, noise_abs=0.02)


def rank_r(R):
    """Rank-R data for the rank instantiations R = 12 and 28: K=20, J=48,
    I_k in [40, 160], N(0, 0.02^2) noise."""
    def make():
        rows = synth.uniform_rows(20, 40, 160, R)
        return synth.parafac2(rows, 48, R, R + 100, noise_abs=0.02)
    return make


def large_rank(K, lo, hi, J, R, seed):
    """Ranks above 32 (one slice per 64-lane group in the iteration, the
    slab pass's four 16-column tiles of Y, the 64-lane factorisations of the
    L x L and L2 x L2 matrices): K slices with I_k in [lo, hi], rank-R
    PARAFAC2 + N(0, 0.02^2)."""
    def make():
        rows = synth.uniform_rows(K, lo, hi, seed)
        return synth.parafac2(rows, J, R, seed, noise_abs=0.02)
    return make


# name -> (tensor factory, R, L, iterations); the GPU tests use the same cases
CASES = {
    "small_parity": (lambda: synth.small_parity(), 5, 15, 100),
    "stock_like_K120": (lambda: synth.stock_like(K=120), 10, 20, 32),
    "outlier_tile": (outlier_tile, 5, 15, 40),
    "rank20_J128": (c4_rank20, 20, 30, 30),
    "rank20_J520": (rank20_long_j, 20, 30, 30),
    "rank12_J48": (rank_r(12), 12, 22, 20),
    "rank28_J48": (rank_r(28), 28, 32, 20),
    "rank40_J600": (large_rank(30, 60, 200, 600, 40, 4040), 40, 50, 10),
    "rank40_J96": (large_rank(40, 40, 150, 96, 40, 4041), 40, 40, 10),
    "rank50_L60_J300": (large_rank(24, 70, 250, 300, 50, 5060), 50, 60, 10),
}


def wide_case(K, J, R, lo, hi, seed, kind="f32"):
    """The chunked slab pass's parity tensors: K slices with I_k in [lo, hi],
    rank-R PARAFAC2 + N(0, 0.02^2); kind "bf16" / "fp8": the slab as the
    library reads it after encoding (the oracle runs on the decoded values)."""
    def make():
        X = synth.parafac2(synth.uniform_rows(K, lo, hi, seed), J, R, seed, noise_abs=0.02)
        if kind == "bf16":
            return synth.IrregularTensor(slab=synth.decode_bf16(synth.encode_bf16(X.slab)), offsets=X.offsets)
        if kind == "fp8":
            codes, scale = synth.encode_fp8(X.slab, X.offsets)
            return synth.IrregularTensor(slab=synth.decode_fp8(codes, X.offsets, scale), offsets=X.offsets)
        return X
    return make


# one power step (q = 1): name -> (tensor factory, R, L, iterations, Omega_1
# rounded to bf16); tests/test_gpu_wide.py uses the same cases.  From a random
# start the early iterations of ALS amplify the difference between the FP32
# sketch matrices of the power step and the oracle's FP64 ones, so the error
# trace gets a bound of its own here.
POWER_CASES = {
    "wide_q1_J517": (wide_case(9, 517, 4, 40, 300, 517), 4, 12, 30, False),
    "wide_q1_J2049_fp8": (wide_case(8, 2049, 5, 40, 200, 2057, "fp8"), 5, 12, 30, True),
    "wide_q1_J2049_bf16": (wide_case(8, 2049, 5, 40, 200, 2057, "bf16"), 5, 12, 30, True),
}


def measure_power(name):
    make, R, L, iters, om_bf16 = POWER_CASES[name]
    X = make()
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    if om_bf16:
        om1 = synth.round_bf16(om1)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters, q=1)
    comp, st, U, fit = emulated_dpar2(X, R, om1, om2, H0, V0, W0, iters, q=1)
    c = ref.comp
    Hg, Vg, Wg = canonical(st.H, st.V, st.W)
    Hr, Vr, Wr = canonical(ref.state.H, ref.state.V, ref.state.W)
    model = lambda H, V, W: np.einsum("ir,kr,jr->kij", H, W, V)
    e, er = np.asarray(st.errors), np.asarray(ref.state.errors)
    return {
        "sigma": float(np.max(np.abs(comp.Bdiag - c.Bdiag) / c.Bdiag)),
        "M": rel(comp.M, c.M),
        "errors": float(np.max(np.abs(e - er) / er)),
        "V": rel(Vg, Vr),
        "W": rel(Wg, Wr),
        "model": rel(model(st.H, st.V, st.W), model(ref.state.H, ref.state.V, ref.state.W)),
        "U": rel(np.concatenate(U), np.concatenate(ref.U)),
        "fit": abs(fit - ref.fit),
    }


def measure(name):
    make, R, L, iters = CASES[name]
    X = make()
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    comp, st, U, fit = emulated_dpar2(X, R, om1, om2, H0, V0, W0, iters)
    c = ref.comp
    s = np.sign(np.sum(comp.D * c.D, axis=0))
    Hg, Vg, Wg = canonical(st.H, st.V, st.W)
    Hr, Vr, Wr = canonical(ref.state.H, ref.state.V, ref.state.W)
    model = lambda H, V, W: np.einsum("ir,kr,jr->kij", H, W, V)
    return {
        "sigma": float(np.max(np.abs(comp.Bdiag - c.Bdiag) / c.Bdiag)),
        "M": rel(comp.M, c.M),
        "M_rows": row_rel(comp.M, c.M),
        "D": rel(comp.D * s, c.D),
        "F": rel(comp.F * s, c.F),
        "E": float(np.max(np.abs(comp.E - c.E) / c.E)),
        "V": rel(Vg, Vr),
        "V_rows": row_rel(Vg, Vr),
        "W": rel(Wg, Wr),
        "model": rel(model(st.H, st.V, st.W), model(ref.state.H, ref.state.V, ref.state.W)),
        "U": rel(np.concatenate(U), np.concatenate(ref.U)),
        "fit": abs(fit - ref.fit),
    }


# ---------------------------------------------------------------------------
# PARAFAC2-ALS on the uncompressed slices (Alg. 2) as the library computes it:
# per iteration Z'_k = X_k V (float32-level, V rounded to float32), the exact
# Gram and projection of the 22-bit fixed-point pair (Z'_k, X_k), then FP64:
# T = S_k H^T, G = T^T Z'^T Z' T, Y_k = G^{-1/2} T^T Z'^T X_k (= Q_k^T X_k with
# Q_k the polar factor of Z'_k T), the CP-ALS sweep, and the error in closed
# form e = sum ||X_k||^2 - 2 sum W.G3 + sum W (H^T H * V^T V) W^T.
# ---------------------------------------------------------------------------

def emulated_plain(X, R, H0, V0, W0, iters, tol=-1.0):
    K = X.K
    Xs = [np.asarray(X.slice(k), dtype=np.float64) for k in range(K)]
    xn = sum(float(np.sum(x * x)) for x in Xs)
    Xq = [tile_round(x, item_ranges(x.shape[0])) for x in Xs]
    H, V, W = (np.array(a, dtype=np.float64) for a in (H0, V0, W0))
    errors, Ulast = [], None
    for _ in range(iters):
        V32 = V.astype(np.float32).astype(np.float64)
        Y = np.zeros((R, X.J, K))
        Us = []
        for k in range(K):
            Zp = (Xs[k] @ V32).astype(np.float32).astype(np.float64)
            Zq = tile_round(Zp, item_ranges(Zp.shape[0]))
            T = np.diag(W[k]) @ H.T
            G = T.T @ (Zq.T @ Zq) @ T
            lam, E = np.linalg.eigh(0.5 * (G + G.T))
            Gm = E @ np.diag(1.0 / np.sqrt(lam)) @ E.T
            Y[:, :, k] = Gm @ T.T @ (Zq.T @ Xq[k])
            Us.append((Zp, T @ Gm))
        H = O.unfold(Y, 0) @ O.khatri_rao(W, V) @ O.pinv((W.T @ W) * (V.T @ V))
        H = O.normalize_columns(H)
        V = O.unfold(Y, 1) @ O.khatri_rao(W, H) @ O.pinv((W.T @ W) * (H.T @ H))
        V = O.normalize_columns(V)
        G3 = O.unfold(Y, 2) @ O.khatri_rao(V, H)
        W = G3 @ O.pinv((V.T @ V) * (H.T @ H))
        e = xn - 2.0 * float(np.sum(W * G3)) + float(np.sum((W @ ((H.T @ H) * (V.T @ V))) * W))
        errors.append(e)
        Ulast = [Zp @ Th @ H for Zp, Th in Us]
        if tol >= 0.0 and len(errors) >= 2 and errors[-2] - errors[-1] < tol * errors[-2]:
            break
    return H, V, W, errors, Ulast, 1.0 - errors[-1] / xn


def plain_ragged(J):
    def make():
        rows = np.array([7, 260, 64, 65, 130, 9, 200, 31, 100, 77, 12, 250], dtype=np.int64)
        return synth.parafac2(rows, J, 4, J + 5, noise_abs=0.02)
    return make


# name -> (tensor factory, R, iterations, tol); tests/test_gpu_plain.py uses the same cases
PLAIN_CASES = {
    "plain_small_parity": (lambda: synth.small_parity(), 5, 30, -1.0),
    "plain_stock_K60": (lambda: synth.stock_like(K=60), 10, 60, 1e-2),
    "plain_ragged_J300": (plain_ragged(300), 4, 20, -1.0),
    "plain_ragged_J40": (plain_ragged(40), 4, 20, -1.0),
    "plain_rank40_J300": (large_rank(20, 50, 200, 300, 40, 4042), 40, 10, -1.0),
}


def measure_plain(name):
    make, R, iters, tol = PLAIN_CASES[name]
    X = make()
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.als_plain(X.slab, X.offsets, R, H0, V0, W0, iters, tol=tol)
    H, V, W, errs, U, fit = emulated_plain(X, R, H0, V0, W0, iters, tol=tol)
    assert len(errs) == len(ref.errors), (name, len(errs), len(ref.errors))
    Hg, Vg, Wg = canonical(H, V, W)
    Hr, Vr, Wr = canonical(ref.H, ref.V, ref.W)
    model = lambda H_, V_, W_: np.einsum("ir,kr,jr->kij", H_, W_, V_)
    return {
        "errors": float(np.max(np.abs(np.asarray(errs) - np.asarray(ref.errors)) / np.asarray(ref.errors))),
        "model": rel(model(H, V, W), model(ref.H, ref.V, ref.W)),
        "V": rel(Vg, Vr), "W": rel(Wg, Wr), "HtH": rel(Hg.T @ Hg, Hr.T @ Hr),
        "U": rel(np.concatenate(U), np.concatenate(ref.U)),
        "fit": abs(fit - ref.fit),
    }


# per check: the floor of the bound (where the emulation gives less)
FLOORS = {"sigma": 1e-6, "M": 1e-6, "M_rows": 1e-6, "D": 1e-6, "F": 1e-6, "E": 1e-6, "V": 1e-6,
          "V_rows": 1e-6, "W": 1e-6, "model": 1e-6, "U": 1e-6, "fit": 1e-8, "errors": 1e-6, "HtH": 1e-6}


def main():
    out = {"safety": SAFETY, "cases": {}, "bounds": {}}
    for name in CASES:
        m = measure(name)
        out["cases"][name] = m
        print(name, {k: f"{v:.2e}" for k, v in m.items()}, flush=True)
    for name in POWER_CASES:
        m = measure_power(name)
        out["cases"][name] = m
        print(name, {k: f"{v:.2e}" for k, v in m.items()}, flush=True)
    for name in PLAIN_CASES:
        m = measure_plain(name)
        out["cases"][name] = m
        print(name, {k: f"{v:.2e}" for k, v in m.items()}, flush=True)
    for name, m in out["cases"].items():
        out["bounds"][name] = {k: float(max(FLOORS[k], SAFETY * v)) for k, v in m.items()}
    with open(os.path.join(HERE, "parity_bounds.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
