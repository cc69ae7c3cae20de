"""FP64 CPU oracle for DPar2 (Jang & Kang, "DPar2: Fast and Scalable PARAFAC2
Decomposition for Irregular Dense Tensors", arXiv 2203.12798).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path (libdpar2 and its
Python binding) never calls it and shares no code with it.

Everything here is plain NumPy/LAPACK in float64, written step by step in the
paper's order and notation so that it can be read against the paper:

  randomized_svd     Alg. 1 (randomized SVD, after Halko et al.), Sec. II-B
  compress           Sec. III-B: first stage (Eq. 4, per-slice randomized SVD),
                     M = ||_k C_k B_k, second stage (Eq. 5), F^(k) (Eqs. 6-7)
                     (first_stage and second_stage separately)
  als_compressed     Alg. 3 iteration: Eq. 8 (SVD of F^(k) E D^T V S_k H^T),
                     implicit Y_k (Sec. III-D), Lemmas 1-3 (G^(1), G^(2),
                     G^(3)), pseudoinverse updates, S_k = diag(W(k,:)),
                     convergence error of Sec. III-E
  dpar2              Alg. 3 end to end, U_k = A_k Z_k P_k^T H
  fitness            the fitness of Sec. IV-A against the original slices
  als_plain          Alg. 2 (PARAFAC2-ALS of Kiers et al.) on uncompressed X_k
  partition          Alg. 4 (greedy number partitioning of slices to threads)
  preprocessed_size  the preprocessed-size theorem of Sec. III-G

Readings where the paper is silent (each also listed in the design notes):
  * one Gaussian Omega_1 (J x L) is shared by all slices and one Omega_2
    (KR x L2) is used for the second stage; both are inputs;
  * L = R + s columns; the power exponent q uses the stabilised form
    (re-orthonormalise between applications of A and A^T), applied to the
    first stage only;
  * QR is Householder with diag(R) > 0 (the Q of any QR algorithm after that
    sign rule);
  * truncated SVD = full SVD of the small matrix, keep the leading R triplets;
    each singular pair is signed so that the largest-magnitude entry of its
    right singular vector is positive (the paper fixes no sign; the sign of a
    column of M = ||_k C_k B_k changes the second-stage sketch M Omega_2, so
    both implementations must agree on it);
  * "normalize H / V" = scale each column to unit 2-norm (norms < 1e-300 are
    left alone); the following least-squares update absorbs the scale;
  * pseudoinverse = Moore-Penrose with cutoff R * eps * sigma_max;
  * stop when e_{t-1} - e_t < tol * e_{t-1} (tol < 0: run max_iter);
  * U_k uses the Z_k, P_k of the last Q-step and the final H.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses

import numpy as np

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------------------
# Small helpers (definitions only)
# ---------------------------------------------------------------------------

def qr_pos(Y: np.ndarray):
    """Thin QR (Householder, LAPACK) with the sign rule diag(R) > 0."""
    Q, Rm = np.linalg.qr(Y)
    s = np.sign(np.diag(Rm))
    s[s == 0] = 1.0
    return Q * s[None, :], Rm * s[:, None]


def pinv(G: np.ndarray) -> np.ndarray:
    """Moore-Penrose pseudoinverse, singular values below R*eps*sigma_max
    treated as zero (the dagger of Lemmas 1-3)."""
    return np.linalg.pinv(G, rcond=G.shape[0] * EPS)


def normalize_columns(A: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns ("Normalize H", "Normalize V" in Alg. 3)."""
    n = np.linalg.norm(A, axis=0)
    n = np.where(n < 1e-300, 1.0, n)
    return A / n[None, :]


# ---------------------------------------------------------------------------
# Alg. 1: randomized SVD
# ---------------------------------------------------------------------------

def randomized_svd(A: np.ndarray, R: int, omega: np.ndarray, q: int = 0):
    """Alg. 1.  A (I x J), omega (J x L) Gaussian test matrix, L = R + s.

    Y = (A A^T)^q A Omega   (stabilised: re-orthonormalise between products)
    Q R = Y                 (QR factorisation)
    B = Q^T A               (L x J)
    B = U~ Sigma V^T        (SVD, truncated at rank R)
    return U = Q U~[:, :R], sigma[:R], V[:, :R]
    """
    A = np.asarray(A, dtype=np.float64)
    Y = A @ np.asarray(omega, dtype=np.float64)
    for _ in range(q):
        Q, _ = qr_pos(Y)
        Z, _ = qr_pos(A.T @ Q)
        Y = A @ Z
    Q, _ = qr_pos(Y)
    B = Q.T @ A
    Ut, s, Vt = np.linalg.svd(B, full_matrices=False)
    U, V = Q @ Ut[:, :R], Vt[:R].T
    # sign gauge: the largest-magnitude entry of each right singular vector is
    # positive (first such entry on ties); U changes sign with it
    sg = np.sign(V[np.argmax(np.abs(V), axis=0), np.arange(R)])
    sg[sg == 0] = 1.0
    return U * sg[None, :], s[:R], V * sg[None, :]


# ---------------------------------------------------------------------------
# Sec. III-B: two-stage compression
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Compressed:
    A: list            # A_k (I_k x R), column-orthonormal
    Bdiag: np.ndarray  # (K, R) singular values of each slice (diag of B_k)
    C: list            # C_k (J x R)
    M: np.ndarray      # (J, K R) = ||_k C_k B_k
    D: np.ndarray      # (J, R)
    E: np.ndarray      # (R,)  diagonal of E
    F: np.ndarray      # (K R, R); F^(k) = F[kR:(k+1)R]
    xnorm2: np.ndarray  # (K,) ||X_k||_F^2

    def Fk(self, k: int) -> np.ndarray:
        R = self.F.shape[1]
        return self.F[k * R:(k + 1) * R]


def partition(rows, T: int):
    """Alg. 4: careful distribution of work.  Sort the row counts in
    descending order (stable), then give each slice to the set whose row sum
    is currently smallest (lowest index on ties).  Returns (sets, sums)."""
    rows = np.asarray(rows)
    sets = [[] for _ in range(T)]
    S = np.zeros(T, dtype=np.int64)
    L_ind = np.argsort(-rows, kind="stable")
    L_val = rows[L_ind]
    for k in range(rows.shape[0]):
        t_min = int(np.argmin(S))
        sets[t_min].append(int(L_ind[k]))
        S[t_min] += int(L_val[k])
    return sets, S


def first_stage(slab: np.ndarray, offsets: np.ndarray, R: int, omega1: np.ndarray, q: int = 0,
                threads: int = 1):
    """Sec. III-B, first stage: randomized SVD of every slice at rank R,
    X_k ~ A_k B_k C_k^T (Eq. 4), slices spread over `threads` workers by
    Alg. 4.  Returns (A, Bdiag, C, xnorm2)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    K = offsets.shape[0] - 1
    A = [None] * K
    C = [None] * K
    Bd = np.zeros((K, R))
    xn = np.zeros(K)

    def one(k):
        Xk = np.asarray(slab[offsets[k]:offsets[k + 1]], dtype=np.float64)
        A[k], Bd[k], C[k] = randomized_svd(Xk, R, omega1, q)
        xn[k] = np.sum(Xk * Xk)

    if threads <= 1:
        for k in range(K):
            one(k)
    else:
        sets, _ = partition(np.diff(offsets), threads)

        def run(ks):
            for k in ks:
                one(k)
        with _cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, sets))
    return A, Bd, C, xn


def second_stage(A, Bd, C, xn, omega2: np.ndarray) -> Compressed:
    """Sec. III-B, second stage: M = ||_k C_k B_k (J x KR) and its randomized
    SVD M ~ D E F^T (Eq. 5); F^(k) = rows kR..kR+R-1 of F (Eqs. 6-7)."""
    K, R = Bd.shape
    J = C[0].shape[0]
    M = np.zeros((J, K * R))
    for k in range(K):
        M[:, k * R:(k + 1) * R] = C[k] * Bd[k][None, :]
    D, E, F = randomized_svd(M, R, omega2, 0)
    return Compressed(A=list(A), Bdiag=Bd, C=list(C), M=M, D=D, E=E, F=F, xnorm2=xn)


def compress(slab: np.ndarray, offsets: np.ndarray, R: int, omega1: np.ndarray,
             omega2: np.ndarray, q: int = 0, threads: int = 1) -> Compressed:
    """Sec. III-B: the first stage over all slices, then the second stage."""
    return second_stage(*first_stage(slab, offsets, R, omega1, q, threads), omega2)


# ---------------------------------------------------------------------------
# Alg. 3 iteration (Secs. III-C .. III-E)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class AlsState:
    H: np.ndarray
    V: np.ndarray
    W: np.ndarray
    Z: np.ndarray      # (K, R, R) left singular vectors of T_k (last Q-step)
    P: np.ndarray      # (K, R, R) right singular vectors of T_k
    errors: list       # e_t after each iteration
    iters: int


def q_step(c: Compressed, H, V, W):
    """Eq. 8: SVD of T_k = F^(k) E D^T V S_k H^T (R x R) = Z_k Sigma_k P_k^T."""
    K = W.shape[0]
    R = H.shape[0]
    E = np.diag(c.E)
    Z = np.zeros((K, R, R))
    P = np.zeros((K, R, R))
    for k in range(K):
        T = c.Fk(k) @ E @ c.D.T @ V @ np.diag(W[k]) @ H.T
        Zk, _, Pkt = np.linalg.svd(T)
        Z[k] = Zk
        P[k] = Pkt.T
    return Z, P


def implicit_Y(c: Compressed, Z, P):
    """Factor of Y_k = P_k Z_k^T F^(k) E D^T (Sec. III-D): returns the R x R
    matrices P_k Z_k^T F^(k); Y_k itself is never formed."""
    K = Z.shape[0]
    return np.stack([P[k] @ Z[k].T @ c.Fk(k) for k in range(K)])


def g1(c: Compressed, Yf, W, V):
    """Lemma 1: G1(:,r) = (sum_k W(k,r) P_k Z_k^T F^(k)) E D^T V(:,r)."""
    R = V.shape[1]
    EDtV = np.diag(c.E) @ c.D.T @ V
    G = np.zeros((R, R))
    for r in range(R):
        S = np.einsum("k,kij->ij", W[:, r], Yf)
        G[:, r] = S @ EDtV[:, r]
    return G


def g2(c: Compressed, Z, P, W, H):
    """Lemma 2: G2(:,r) = D E sum_k W(k,r) F^(k)T Z_k P_k^T H(:,r)."""
    K, R = W.shape
    J = c.D.shape[0]
    DE = c.D @ np.diag(c.E)
    G = np.zeros((J, R))
    for r in range(R):
        acc = np.zeros(R)
        for k in range(K):
            acc += W[k, r] * (c.Fk(k).T @ Z[k] @ P[k].T @ H[:, r])
        G[:, r] = DE @ acc
    return G


def g3(c: Compressed, Yf, V, H):
    """Lemma 3: G3(k,r) = vec(P_k Z_k^T F^(k))^T (E D^T V(:,r) kron H(:,r)),
    vec stacking columns."""
    K = Yf.shape[0]
    R = H.shape[0]
    EDtV = np.diag(c.E) @ c.D.T @ V
    G = np.zeros((K, R))
    vecs = Yf.transpose(0, 2, 1).reshape(K, R * R)   # column-major vec per k
    for r in range(R):
        G[:, r] = vecs @ np.kron(EDtV[:, r], H[:, r])
    return G


def compressed_error(c: Compressed, Yf, H, V, W) -> float:
    """Sec. III-E: e = sum_k || P_k Z_k^T F^(k) E D^T - H S_k V^T ||_F^2,
    with explicit R x J matrices."""
    EDt = np.diag(c.E) @ c.D.T
    e = 0.0
    for k in range(W.shape[0]):
        Dk = Yf[k] @ EDt - H @ np.diag(W[k]) @ V.T
        e += float(np.sum(Dk * Dk))
    return e


def als_compressed(c: Compressed, H0, V0, W0, max_iter: int, tol: float = -1.0,
                   callback=None) -> AlsState:
    """Alg. 3, the repeat loop: Q-step (Eq. 8), implicit Y_k, then one CP-ALS
    sweep through Lemmas 1-3 with normalised H and V, S_k = diag(W(k,:)),
    until max_iter or the error stops decreasing by more than tol (relative)."""
    H = np.array(H0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    W = np.array(W0, dtype=np.float64)
    errors = []
    Z = P = None
    it = 0
    for it in range(1, max_iter + 1):
        Z, P = q_step(c, H, V, W)
        Yf = implicit_Y(c, Z, P)
        H = g1(c, Yf, W, V) @ pinv((W.T @ W) * (V.T @ V))
        H = normalize_columns(H)
        V = g2(c, Z, P, W, H) @ pinv((W.T @ W) * (H.T @ H))
        V = normalize_columns(V)
        W = g3(c, Yf, V, H) @ pinv((V.T @ V) * (H.T @ H))
        e = compressed_error(c, Yf, H, V, W)
        errors.append(e)
        if callback is not None:
            callback(it, H, V, W, Z, P, e)
        if tol >= 0.0 and len(errors) >= 2 and errors[-2] - errors[-1] < tol * errors[-2]:
            break
    return AlsState(H=H, V=V, W=W, Z=Z, P=P, errors=errors, iters=it)


# ---------------------------------------------------------------------------
# End to end
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    comp: Compressed
    state: AlsState
    U: list            # U_k = A_k Z_k P_k^T H
    fit: float         # fitness against the original slices


def output_U(c: Compressed, st: AlsState):
    """Alg. 3 output: U_k = A_k Z_k P_k^T H."""
    return [c.A[k] @ st.Z[k] @ st.P[k].T @ st.H for k in range(len(c.A))]


def fitness(slab, offsets, U, W, V) -> float:
    """Sec. IV-A: 1 - sum_k ||X_k - U_k S_k V^T||^2 / sum_k ||X_k||^2."""
    num = 0.0
    den = 0.0
    for k in range(len(U)):
        Xk = np.asarray(slab[offsets[k]:offsets[k + 1]], dtype=np.float64)
        Rk = Xk - U[k] @ np.diag(W[k]) @ V.T
        num += float(np.sum(Rk * Rk))
        den += float(np.sum(Xk * Xk))
    return 1.0 - num / den


def dpar2(slab, offsets, R, omega1, omega2, H0, V0, W0, max_iter, tol=-1.0, q=0,
          threads=1) -> Result:
    """Alg. 3: compress once, iterate on the compressed data, recover U_k."""
    c = compress(slab, offsets, R, omega1, omega2, q=q, threads=threads)
    st = als_compressed(c, H0, V0, W0, max_iter, tol)
    U = output_U(c, st)
    return Result(comp=c, state=st, U=U, fit=fitness(slab, offsets, U, st.W, st.V))


# ---------------------------------------------------------------------------
# Alg. 2: PARAFAC2-ALS on the uncompressed slices (accuracy reference)
# ---------------------------------------------------------------------------

def unfold(T: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n matricisation (Kolda & Bader): columns ordered with the lower
    remaining mode index varying fastest."""
    return np.reshape(np.moveaxis(T, mode, 0), (T.shape[mode], -1), order="F")


def khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product A (.) B."""
    return np.stack([np.kron(A[:, r], B[:, r]) for r in range(A.shape[1])], axis=1)


@dataclasses.dataclass
class PlainResult:
    H: np.ndarray
    V: np.ndarray
    W: np.ndarray
    Q: list
    errors: list
    fit: float
    U: list


def als_plain(slab, offsets, R, H0, V0, W0, max_iter, tol=-1.0) -> PlainResult:
    """Alg. 2.  Q_k = Z'_k P'_k^T from the SVD of X_k V S_k H^T; Y_k = Q_k^T X_k
    stacked into Y (R x J x K); one CP-ALS sweep on Y with explicit unfoldings
    and Khatri-Rao products; S_k = diag(W(k,:)).  H and V are normalised as in
    Alg. 3 (a gauge that leaves the model unchanged).  The error is
    sum_k ||X_k - Q_k H S_k V^T||^2."""
    offsets = np.asarray(offsets)
    K = offsets.shape[0] - 1
    J = slab.shape[1]
    X = [np.asarray(slab[offsets[k]:offsets[k + 1]], dtype=np.float64) for k in range(K)]
    H = np.array(H0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    W = np.array(W0, dtype=np.float64)
    errors = []
    Q = None
    for _ in range(max_iter):
        Q = []
        for k in range(K):
            Zp, _, Ppt = np.linalg.svd(X[k] @ V @ np.diag(W[k]) @ H.T, full_matrices=False)
            Q.append(Zp[:, :R] @ Ppt[:R])
        Y = np.zeros((R, J, K))
        for k in range(K):
            Y[:, :, k] = Q[k].T @ X[k]
        H = unfold(Y, 0) @ khatri_rao(W, V) @ pinv((W.T @ W) * (V.T @ V))
        H = normalize_columns(H)
        V = unfold(Y, 1) @ khatri_rao(W, H) @ pinv((W.T @ W) * (H.T @ H))
        V = normalize_columns(V)
        W = unfold(Y, 2) @ khatri_rao(V, H) @ pinv((V.T @ V) * (H.T @ H))
        e = 0.0
        for k in range(K):
            Dk = X[k] - Q[k] @ H @ np.diag(W[k]) @ V.T
            e += float(np.sum(Dk * Dk))
        errors.append(e)
        if tol >= 0.0 and len(errors) >= 2 and errors[-2] - errors[-1] < tol * errors[-2]:
            break
    U = [Q[k] @ H for k in range(K)]
    return PlainResult(H=H, V=V, W=W, Q=Q, errors=errors,
                       fit=fitness(slab, offsets, U, W, V), U=U)


# ---------------------------------------------------------------------------
# Sec. III-G: size of the preprocessed data
# ---------------------------------------------------------------------------

def preprocessed_size(rows, J: int, R: int) -> int:
    """Number of stored values: A_k (I_k x R each), F^(k) (R x R each),
    E (R), D (J x R)."""
    rows = np.asarray(rows)
    K = rows.shape[0]
    return int(np.sum(rows) * R + K * R * R + R + J * R)
