"""Pins for the warm-start oracle (CPU only): the analytic gradient against
central finite differences of the loss, the invariances that define the
features and the target gauge, and Adam's closed form in a degenerate case."""
import numpy as np
import pytest

from oracle import warm_oracle as WO


def _rand_orth(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def _problem(seed=0, K=7, R=4, J=9):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(WO.n_params(R)) * 0.2
    tok = rng.standard_normal((K, WO.n_features(R)))
    tH = rng.standard_normal((R, R))
    tH = tH.T @ tH
    tV = rng.standard_normal((R, R))
    tW = rng.standard_normal((K, R))
    return theta, tok, tH, tV, tW


def test_parameter_count():
    R = 10
    F, W = 55, 128
    assert WO.n_params(R) == W * F + W + W * W + W + 2 * (R * R * W + R * R) + R * 2 * W + R


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    """Central differences (step 1e-6) of the summed loss against the
    analytic gradient, on 60 random parameters of every block."""
    R = 4
    theta, tok, tH, tV, tW = _problem(seed, R=R)
    pH, pV, pW, cache = WO.forward(theta, tok, R)
    g = WO.backward(pH, pV, pW, tH, tV, tW, cache, R)

    def L(th):
        a, b, c, _ = WO.forward(th, tok, R)
        return sum(WO.loss(a, b, c, tH, tV, tW, R))

    rng = np.random.default_rng(seed + 10)
    at = 0
    for name, shp in WO.param_shapes(R):
        n = int(np.prod(shp))
        for i in rng.choice(n, size=min(n, 6), replace=False):
            e = np.zeros_like(theta)
            e[at + i] = 1e-6
            num = (L(theta + e) - L(theta - e)) / 2e-6
            assert abs(num - g[at + i]) <= 1e-6 * max(1.0, abs(num)), (name, i, num, g[at + i])
        at += n


def _compressed(seed=3, K=6, R=3, J=8):
    """F (KR x R) with orthonormal columns, E > 0, D (J x R) orthonormal."""
    rng = np.random.default_rng(seed)
    F = np.linalg.qr(rng.standard_normal((K * R, R)))[0]
    E = np.sort(rng.uniform(1.0, 5.0, R))[::-1]
    D = np.linalg.qr(rng.standard_normal((J, R)))[0]
    return F, E, D


def test_features_invariant_to_slice_rotations_and_basis_signs():
    """The first stage leaves a rotation O_k of each slice free (A_k O_k^T,
    O_k F^(k) give the same M), and the second stage leaves the signs of
    D's columns free (D diag(s), F diag(s)): the tokens must not change."""
    K, R = 6, 3
    F, E, D = _compressed(K=K, R=R)
    t0, e0 = WO.features(F, E, D, K, R)
    rng = np.random.default_rng(4)
    F2 = F.copy()
    for k in range(K):
        F2[k * R:(k + 1) * R] = _rand_orth(rng, R) @ F[k * R:(k + 1) * R]
    s = np.array([1.0, -1.0, -1.0])
    t1, e1 = WO.features(F2 * s, E, D * s, K, R)
    np.testing.assert_allclose(t1, t0, atol=1e-12)
    assert e1 == pytest.approx(e0)
    # mean trace of the tokens' Phi is R (normalisation by e_mean = ||E||^2 / K)
    iu = np.triu_indices(R)
    diag = [i for i, (a, b) in enumerate(zip(*iu)) if a == b]
    assert t0[:, diag].sum(axis=1).mean() == pytest.approx(R)


def _model_gram(H, V, W):
    """(H S_k V^T)^T (H S_k V^T) per slice: the part of the model that the
    free Q_k leaves identifiable."""
    return np.stack([V @ np.diag(w) @ H.T @ H @ np.diag(w) @ V.T for w in W])


def test_targets_fix_every_gauge_and_keep_the_model():
    """Column scalings (H r -> a H r, V r -> b V r, W r -> W r / (a b)), sign
    flips and a permutation of the components leave the targets unchanged,
    and the factors rebuilt from the targets (V = D' T_V, diag(S_k) from
    T_W, H^T H = T_H) give the same per-slice model Gram."""
    K, R, J = 6, 3, 8
    F, E, D = _compressed(K=K, R=R, J=J)
    rng = np.random.default_rng(5)
    H = rng.standard_normal((R, R))
    V = D @ rng.standard_normal((R, R))          # V in span(D)
    W = rng.uniform(0.5, 1.5, (K, R))
    e_mean = float(np.sum(E ** 2)) / K
    tH, tV, tW = WO.targets(H, V, W, D, e_mean, R)
    a = np.array([2.0, -0.5, 3.0])
    b = np.array([-1.5, 4.0, 0.25])
    perm = [2, 0, 1]
    H2, V2, W2 = (H * a)[:, perm], (V * b)[:, perm], (W / (a * b))[:, perm]
    for x, y in zip(WO.targets(H2, V2, W2, D, e_mean, R), (tH, tV, tW)):
        np.testing.assert_allclose(x, y, atol=1e-12)
    Ds, _ = WO.sign_basis(D)
    Vr = Ds @ tV
    Wr = tW * np.sqrt(e_mean / R)
    G = np.stack([Vr @ np.diag(w) @ tH @ np.diag(w) @ Vr.T for w in Wr])
    np.testing.assert_allclose(G, _model_gram(H, V, W), atol=1e-10)
    # the rebuilt V has unit columns, sorted by ||W(:, r)||
    np.testing.assert_allclose(np.linalg.norm(Vr, axis=0), 1.0, atol=1e-12)
    assert np.all(np.diff(np.linalg.norm(tW, axis=0)) <= 1e-12)
    np.testing.assert_allclose(np.diag(tH), 1.0, atol=1e-12)


def test_apply_inverts_targets():
    """apply(H_c, T_V, T_W) returns V = D' T_V and W = T_W sqrt(e_mean / R)."""
    K, R, J = 5, 3, 7
    F, E, D = _compressed(K=K, R=R, J=J)
    rng = np.random.default_rng(6)
    pH, pV, pW = rng.standard_normal((R, R)), rng.standard_normal((R, R)), rng.standard_normal((K, R))
    e_mean = 2.5
    H, V, W = WO.apply(pH, pV, pW, D, e_mean, R)
    Ds, _ = WO.sign_basis(D)
    np.testing.assert_allclose(Ds.T @ V, pV, atol=1e-12)
    np.testing.assert_allclose(W, pW * np.sqrt(e_mean / R))
    np.testing.assert_array_equal(H, pH)


def test_adam_without_moments_is_a_sign_step():
    """With beta1 = beta2 = 0 and eps -> 0, Adam moves every parameter by
    exactly lr against the sign of its gradient."""
    rng = np.random.default_rng(7)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = WO.adam(th, g, np.zeros(50), np.zeros(50), 1, 0.01, 0.0, 0.0, 1e-300)
    np.testing.assert_allclose(new, th - 0.01 * np.sign(g), atol=1e-15)
    np.testing.assert_allclose(m, g)
    np.testing.assert_allclose(v, g * g)
