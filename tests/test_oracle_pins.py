"""Pins for the FP64 oracle: each test checks it against something the paper or
the mathematics fixes (closed forms, identities, special cases, brute force,
a textbook re-derivation), never against itself.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(seed=11, K=6, J=9, rank=3, imin=12, imax=20, noise=0.0):
    rows = synth.uniform_rows(K, imin, imax, seed)
    return synth.parafac2(rows, J, rank, seed, noise_abs=noise)


# ---------------------------------------------------------------------------
# Alg. 1 (randomized SVD)
# ---------------------------------------------------------------------------

def test_rsvd_equals_truncated_svd_when_sketch_spans_range():
    """With L >= rank(A) the sketch spans range(A), so Alg. 1 returns the
    exact truncated SVD (Eckart-Young).  Reference: eigen-decomposition of
    A^T A, a different route to the same singular triplets."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 4)) @ np.diag([9.0, 5.0, 2.0, 0.7]) @ rng.standard_normal((4, 12))
    omega = rng.standard_normal((12, 6))
    U, s, V = O.randomized_svd(A, 3, omega)
    lam, Ev = np.linalg.eigh(A.T @ A)
    order = np.argsort(lam)[::-1]
    s_ref = np.sqrt(np.maximum(lam[order[:3]], 0))
    np.testing.assert_allclose(s, s_ref, rtol=1e-10)
    Vref = Ev[:, order[:3]]
    np.testing.assert_allclose(V @ V.T, Vref @ Vref.T, atol=1e-10)
    # U = A V / s
    np.testing.assert_allclose(U, A @ V / s[None, :], atol=1e-10)


def test_rsvd_full_sketch_is_exact_truncation():
    """L = J: the randomized SVD of a full-rank A is its exact rank-R
    truncation, residual^2 = sum of the trailing sigma^2."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 8))
    U, s, V = O.randomized_svd(A, 3, rng.standard_normal((8, 8)))
    lam = np.sort(np.linalg.eigvalsh(A.T @ A))[::-1]
    resid = A - U @ np.diag(s) @ V.T
    assert abs(np.sum(resid ** 2) - np.sum(lam[3:])) < 1e-10 * np.sum(lam)


def test_rsvd_projection_identity_and_orthonormality():
    """Alg. 1 gives U^T A = Sigma V^T for any sketch width (B = Q^T A exactly),
    with U and V column-orthonormal."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((50, 20))
    U, s, V = O.randomized_svd(A, 4, rng.standard_normal((20, 7)))
    np.testing.assert_allclose(U.T @ A, np.diag(s) @ V.T, atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(4), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(4), atol=1e-13)
    assert np.all(np.diff(s) <= 0)


def test_power_iteration_improves_capture():
    """(A A^T)^q A Omega with q = 1 captures the leading subspace at least as
    well as q = 0 on a slowly decaying spectrum (Halko et al.)."""
    rng = np.random.default_rng(3)
    Uo, _ = np.linalg.qr(rng.standard_normal((200, 60)))
    Vo, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    A = Uo @ np.diag(1.0 / np.arange(1, 61) ** 0.5) @ Vo.T
    om = rng.standard_normal((60, 8))
    r0 = np.linalg.norm(A - (lambda u, s, v: u @ np.diag(s) @ v.T)(*O.randomized_svd(A, 4, om, 0)))
    r1 = np.linalg.norm(A - (lambda u, s, v: u @ np.diag(s) @ v.T)(*O.randomized_svd(A, 4, om, 1)))
    opt = np.sqrt(np.sum((1.0 / np.arange(5, 61) ** 0.5) ** 2))
    assert opt <= r1 + 1e-12 and r1 <= r0 + 1e-12


def _rsvd_noop_power(A, R, omega, q=0):
    """A deliberately broken copy of Alg. 1 whose power loop changes nothing
    (the span stays that of A Omega).  Kept so that the power-step pin below
    is shown to reject it."""
    A = np.asarray(A, dtype=np.float64)
    Y = A @ np.asarray(omega, dtype=np.float64)
    for _ in range(q):
        Q, _ = O.qr_pos(Y)
        Z, _ = O.qr_pos(A.T @ Q)
    Q, _ = O.qr_pos(Y)
    Ut, s, Vt = np.linalg.svd(Q.T @ A, full_matrices=False)
    return Q @ Ut[:, :R], s[:R], Vt[:R].T


def _projector(M):
    Q, _ = np.linalg.qr(M)
    return Q @ Q.T


def _power_span_error(rsvd, q):
    """Distance between the range Alg. 1 returns with R = L (so that span(U)
    is the whole sketch span) and span((A A^T)^q A Omega) formed literally,
    without any re-orthonormalisation, on a well-conditioned A (singular
    values in [1, 2], so the literal product loses nothing)."""
    rng = np.random.default_rng(31)
    Uo, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    Vo, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    A = Uo @ np.diag(np.linspace(2.0, 1.0, 12)) @ Vo.T
    om = rng.standard_normal((12, 5))
    U, _, _ = rsvd(A, 5, om, q)
    Y = A @ om
    for _ in range(q):
        Y = A @ (A.T @ Y)
    return float(np.linalg.norm(U @ U.T - _projector(Y))), float(np.linalg.norm(U @ U.T - _projector(A @ om)))


@pytest.mark.parametrize("q", [1, 2])
def test_power_iteration_spans_literal_power_product(q):
    """Alg. 1 with q power steps: span(Y) = span((A A^T)^q A Omega).  The
    oracle's stabilised loop must reach the literal product's span (1e-10),
    which differs clearly from span(A Omega); a power loop that does nothing
    fails the same check."""
    err, vs_q0 = _power_span_error(O.randomized_svd, q)
    assert err < 1e-10, err
    assert vs_q0 > 1e-2, vs_q0            # q >= 1 really moves the subspace
    bad, _ = _power_span_error(_rsvd_noop_power, q)
    assert bad > 1e-2, bad


# ---------------------------------------------------------------------------
# Two-stage compression (Sec. III-B)
# ---------------------------------------------------------------------------

def test_compression_exact_on_noise_free_parafac2():
    """Noise-free rank-R PARAFAC2 slices: both randomized SVDs capture the
    whole range, so A_k F^(k) E D^T = X_k (Eq. 6) up to the float32 rounding
    of the stored slab (which is the only part of X_k outside rank R)."""
    X = _small(noise=0.0)
    R = 3
    om1, om2 = synth.omegas(X.J, 5, X.K * R)
    c = O.compress(X.slab, X.offsets, R, om1, om2)
    for k in range(X.K):
        Xk = X.slice(k).astype(np.float64)
        rec = c.A[k] @ c.Fk(k) @ np.diag(c.E) @ c.D.T
        assert np.linalg.norm(rec - Xk) <= 2.0 ** -22 * np.linalg.norm(Xk)
    np.testing.assert_allclose(c.D.T @ c.D, np.eye(R), atol=1e-12)
    np.testing.assert_allclose(c.F.T @ c.F, np.eye(R), atol=1e-12)
    for k in range(X.K):
        np.testing.assert_allclose(c.A[k].T @ c.A[k], np.eye(R), atol=1e-12)


def test_M_is_concatenation_of_CkBk():
    """M = ||_k C_k B_k, and the second stage factors M ~ D E F^T with block
    k of D E F^T equal to D E F^(k)T (Eqs. 5-7)."""
    X = _small(seed=12, noise=0.05)
    R = 3
    om1, om2 = synth.omegas(X.J, 6, X.K * R)
    c = O.compress(X.slab, X.offsets, R, om1, om2)
    for k in range(X.K):
        np.testing.assert_allclose(c.M[:, k * R:(k + 1) * R], c.C[k] * c.Bdiag[k][None, :], atol=0)
    DEF = c.D @ np.diag(c.E) @ c.F.T
    for k in range(X.K):
        np.testing.assert_allclose(DEF[:, k * R:(k + 1) * R], c.D @ np.diag(c.E) @ c.Fk(k).T, atol=1e-12)


def test_partition_threads_do_not_change_compression():
    """Alg. 4 only schedules work: the compressed result is the same for any
    number of threads."""
    X = _small(seed=13, K=9, noise=0.05)
    om1, om2 = synth.omegas(X.J, 5, X.K * 3)
    c1 = O.compress(X.slab, X.offsets, 3, om1, om2, threads=1)
    c3 = O.compress(X.slab, X.offsets, 3, om1, om2, threads=3)
    np.testing.assert_array_equal(c1.M, c3.M)
    np.testing.assert_array_equal(c1.F, c3.F)


# ---------------------------------------------------------------------------
# Lemmas 1-3 against the textbook MTTKRP on an explicit Y tensor
# ---------------------------------------------------------------------------

def test_lemmas_equal_naive_mttkrp():
    """G^(1) = Y_(1)(W kr V), G^(2) = Y_(2)(W kr H), G^(3) = Y_(3)(V kr H)
    written in index form on the explicit tensor Y(:,:,k) = P_k Z_k^T F^(k) E D^T."""
    X = _small(seed=14, noise=0.1)
    R = 3
    om1, om2 = synth.omegas(X.J, 5, X.K * R)
    c = O.compress(X.slab, X.offsets, R, om1, om2)
    rng = np.random.default_rng(5)
    H, V, W = rng.standard_normal((R, R)), rng.standard_normal((X.J, R)), rng.uniform(0.5, 1.5, (X.K, R))
    Z, P = O.q_step(c, H, V, W)
    Yf = O.implicit_Y(c, Z, P)
    Y = np.stack([Yf[k] @ np.diag(c.E) @ c.D.T for k in range(X.K)], axis=2)   # R x J x K
    G1 = np.einsum("ijk,kr,jr->ir", Y, W, V)
    G2 = np.einsum("ijk,kr,ir->jr", Y, W, H)
    G3 = np.einsum("ijk,jr,ir->kr", Y, V, H)
    np.testing.assert_allclose(O.g1(c, Yf, W, V), G1, rtol=1e-12, atol=1e-12 * np.abs(G1).max())
    np.testing.assert_allclose(O.g2(c, Z, P, W, H), G2, rtol=1e-12, atol=1e-12 * np.abs(G2).max())
    np.testing.assert_allclose(O.g3(c, Yf, V, H), G3, rtol=1e-12, atol=1e-12 * np.abs(G3).max())


def test_q_step_is_procrustes_on_uncompressed_form():
    """Eq. 8: A_k Z_k P_k^T is the orthonormal minimiser of
    ||A_k F^(k) E D^T - Q H S_k V^T||, i.e. the polar factor of
    (A_k F^(k) E D^T) V S_k H^T, here computed by a matrix square root."""
    X = _small(seed=15, noise=0.1)
    R = 3
    om1, om2 = synth.omegas(X.J, 5, X.K * R)
    c = O.compress(X.slab, X.offsets, R, om1, om2)
    rng = np.random.default_rng(6)
    H, V, W = rng.standard_normal((R, R)), rng.standard_normal((X.J, R)), rng.uniform(0.5, 1.5, (X.K, R))
    Z, P = O.q_step(c, H, V, W)
    for k in range(X.K):
        Mk = c.A[k] @ c.Fk(k) @ np.diag(c.E) @ c.D.T @ V @ np.diag(W[k]) @ H.T
        lam, Ev = np.linalg.eigh(Mk.T @ Mk)
        polar = Mk @ Ev @ np.diag(lam ** -0.5) @ Ev.T
        np.testing.assert_allclose(c.A[k] @ Z[k] @ P[k].T, polar, atol=1e-9)


# ---------------------------------------------------------------------------
# Iteration invariants
# ---------------------------------------------------------------------------

def _run_small(seed=16, noise=0.05, iters=30, K=8, J=10, rank=3):
    X = _small(seed=seed, noise=noise, K=K, J=J, rank=rank)
    R = rank
    om1, om2 = synth.omegas(X.J, R + 3, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    res = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    return X, res


def test_error_is_monotone_and_unitarily_invariant():
    """Each ALS sub-step is an exact minimiser, so e_t never increases; and
    e equals sum_k ||A_k F^(k) E D^T - Q_k H S_k V^T||^2 (Sec. III-E)."""
    X, res = _run_small()
    e = np.array(res.state.errors)
    assert np.all(np.diff(e) <= 1e-12 * e[:-1])
    c, st = res.comp, res.state
    tot = 0.0
    for k in range(X.K):
        Qk = c.A[k] @ st.Z[k] @ st.P[k].T
        d = c.A[k] @ c.Fk(k) @ np.diag(c.E) @ c.D.T - Qk @ st.H @ np.diag(st.W[k]) @ st.V.T
        tot += np.sum(d * d)
    Yf = O.implicit_Y(c, st.Z, st.P)
    e_last = O.compressed_error(c, Yf, st.H, st.V, st.W)
    assert abs(e_last - tot) <= 1e-10 * tot


def test_parafac2_constraint_and_orthonormal_Q():
    """U_k = Q_k H with Q_k^T Q_k = I, hence U_k^T U_k = H^T H for every k
    (Harshman's constraint)."""
    X, res = _run_small(seed=17)
    c, st = res.comp, res.state
    HtH = st.H.T @ st.H
    for k in range(X.K):
        Qk = c.A[k] @ st.Z[k] @ st.P[k].T
        np.testing.assert_allclose(Qk.T @ Qk, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(res.U[k].T @ res.U[k], HtH, atol=1e-12)


def test_substeps_are_minimisers():
    """Perturbing H, V or W after an update never lowers the compressed error
    (least-squares optimality of Lemma 1-3 updates)."""
    X, res = _run_small(seed=18, iters=5)
    c, st = res.comp, res.state
    Yf = O.implicit_Y(c, st.Z, st.P)
    e0 = O.compressed_error(c, Yf, st.H, st.V, st.W)
    rng = np.random.default_rng(7)
    for _ in range(10):
        dW = 1e-4 * rng.standard_normal(st.W.shape)
        assert O.compressed_error(c, Yf, st.H, st.V, st.W + dW) >= e0 - 1e-12 * e0


def test_fixed_point_at_ground_truth():
    """Exactly low-rank PARAFAC2 data started at the generating factors: the
    model is exact and stays exact, 1 - fitness < 1e-10."""
    X = synth.exact_parafac2(21, K=16, J=12, rank=4, imin=20, imax=40)
    R = 4
    om1, om2 = synth.omegas(X.J, 6, X.K * R)
    res = O.dpar2(X.slab, X.offsets, R, om1, om2, X.H, X.V, X.W, 10)
    # the slab is float32: the ground truth reproduces it to float32 rounding
    assert 1.0 - res.fit < 1e-10


def test_perturbed_truth_converges_to_exact_fit():
    """Start 1% away from the generating factors: ALS converges to fitness 1
    within 1e-10 on exactly low-rank data (64 slices, J=32, rank 5)."""
    X = synth.exact_parafac2(22, K=64, J=32, rank=5, imin=20, imax=40)
    R = 5
    rng = np.random.default_rng(8)
    H0 = X.H * (1 + 0.01 * rng.standard_normal(X.H.shape))
    V0 = X.V * (1 + 0.01 * rng.standard_normal(X.V.shape))
    W0 = X.W * (1 + 0.01 * rng.standard_normal(X.W.shape))
    om1, om2 = synth.omegas(X.J, 7, X.K * R)
    res = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, 200)
    assert 1.0 - res.fit < 1e-10


def test_single_slice_reduces_to_truncated_svd():
    """K = 1 and L = J: PARAFAC2 of one slice is its best rank-R approximation,
    fitness = sum_{i<=R} sigma_i^2 / sum sigma_i^2."""
    rng = np.random.default_rng(9)
    A = (rng.standard_normal((40, 6)) @ np.diag([10, 6, 3, 1, 0.5, 0.2]) @ rng.standard_normal((6, 6))).astype(np.float32)
    off = np.array([0, 40], dtype=np.int64)
    R = 3
    om1 = rng.standard_normal((6, 6)).astype(np.float32)
    om2 = rng.standard_normal((3, 3)).astype(np.float32)
    H0, V0, W0 = synth.init_factors(6, 1, R)
    res = O.dpar2(A, off, R, om1, om2, H0, V0, W0, 200)
    lam = np.sort(np.linalg.eigvalsh(A.astype(np.float64).T @ A.astype(np.float64)))[::-1]
    assert abs(res.fit - np.sum(lam[:R]) / np.sum(lam)) < 1e-9


def test_dpar2_matches_plain_parafac2_als_when_compression_is_exact():
    """On noise-free rank-R data both stages are exact, so Alg. 3 and Alg. 2
    (explicit unfoldings and Khatri-Rao products) follow the same trajectory
    (up to the float32 rounding of the slab, the only part outside rank R)."""
    X = synth.exact_parafac2(23, K=10, J=9, rank=3, imin=15, imax=30)
    R = 3
    om1, om2 = synth.omegas(X.J, 5, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    d = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, 15)
    p = O.als_plain(X.slab, X.offsets, R, H0, V0, W0, 15)
    e_d, e_p = np.array(d.state.errors), np.array(p.errors)
    np.testing.assert_allclose(e_d, e_p, rtol=1e-6, atol=1e-9 * e_p[0])
    np.testing.assert_allclose(d.state.V, p.V, atol=1e-8)
    np.testing.assert_allclose(d.state.W, p.W, rtol=1e-6, atol=1e-9)


def test_plain_als_monotone_and_K1_svd():
    X = _small(seed=24, noise=0.1)
    H0, V0, W0 = synth.init_factors(X.J, X.K, 3)
    p = O.als_plain(X.slab, X.offsets, 3, H0, V0, W0, 20)
    e = np.array(p.errors)
    assert np.all(np.diff(e) <= 1e-12 * e[:-1])


def test_true_fitness_from_compressed_factors():
    """sum_k ||X_k - U_k S_k V^T||^2 = sum ||X_k||^2 - 2 sum_k tr(V S_k H^T
    (Z_k P_k^T)^T (C_k B_k)^T) + sum_k W(k,:)(H^T H * V^T V)W(k,:)^T, using
    A_k^T X_k = (C_k B_k)^T: the fitness needs no second pass over the slab."""
    X, res = _run_small(seed=25, noise=0.1)
    c, st = res.comp, res.state
    R = st.H.shape[0]
    num = float(np.sum(c.xnorm2))
    HV = (st.H.T @ st.H) * (st.V.T @ st.V)
    for k in range(X.K):
        CB = c.M[:, k * R:(k + 1) * R]
        Psi = st.Z[k] @ st.P[k].T
        num -= 2 * np.trace(st.V @ np.diag(st.W[k]) @ st.H.T @ Psi.T @ CB.T)
        num += st.W[k] @ HV @ st.W[k]
    fit = 1 - num / float(np.sum(c.xnorm2))
    assert abs(fit - res.fit) < 1e-12


# ---------------------------------------------------------------------------
# Alg. 4 and the size theorem
# ---------------------------------------------------------------------------

def test_partition_hand_example():
    with open(os.path.join(GOLDEN, "alg4_partition.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        sets, sums = O.partition(np.array(case["rows"]), case["T"])
        assert sets == case["sets"]
        assert list(sums) == case["sums"]


def test_partition_lpt_bound_vs_brute_force():
    """Greedy LPT makespan <= (4/3 - 1/(3T)) * optimum (Graham), optimum by
    brute force over all assignments of <= 8 items."""
    rng = np.random.default_rng(10)
    for _ in range(30):
        n = int(rng.integers(3, 9))
        T = int(rng.integers(2, 4))
        rows = rng.integers(1, 50, size=n)
        _, sums = O.partition(rows, T)
        best = min(max(np.bincount(np.array(a), weights=rows, minlength=T))
                   for a in itertools.product(range(T), repeat=n))
        assert max(sums) <= (4 / 3 - 1 / (3 * T)) * best + 1e-9
        assert sum(sums) == rows.sum()


def test_preprocessed_size_and_ratio():
    """Sec. III-G size theorem and the compression ratio of Sec. IV-B:
    IJK / (IKR + KR^2 + JR) for equal I_k (E adds R values)."""
    X = _small(seed=26, K=5, J=11, rank=3, imin=20, imax=20)
    om1, om2 = synth.omegas(X.J, 5, X.K * 3)
    c = O.compress(X.slab, X.offsets, 3, om1, om2)
    stored = sum(a.size for a in c.A) + c.F.size + c.E.size + c.D.size
    assert O.preprocessed_size(X.rows, X.J, 3) == stored
    I, J, K, R = 20, 11, 5, 3
    ratio = I * J * K / (I * K * R + K * R * R + J * R)
    assert abs(ratio - 1 / (R / J + R * R / (I * J) + R / (I * K))) < 1e-12
