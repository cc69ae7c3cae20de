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


# ---------------------------------------------------------------------------
# Forward pass: set-encoder structure, and Adam beyond the degenerate case
# ---------------------------------------------------------------------------

def _forward_sum_pool(theta, tok, R):
    """A deliberately broken copy of the forward pass that pools by summing
    instead of averaging; kept so that the pins below are shown to reject it."""
    P = WO.unpack(theta, R)
    x = np.asarray(tok, dtype=np.float64)
    K = x.shape[0]
    Z1 = np.maximum(x @ P["W1"].T + P["b1"], 0.0)
    Z2 = np.maximum(Z1 @ P["W2"].T + P["b2"], 0.0)
    p = Z2.sum(axis=0)
    pH = (P["WH"] @ p + P["bH"]).reshape(R, R)
    pV = (P["WV"] @ p + P["bV"]).reshape(R, R)
    cat = np.concatenate([Z2, np.broadcast_to(p, (K, WO.WIDTH))], axis=1)
    return pH, pV, cat @ P["Ww"].T + P["bw"], None


def _set_encoder_ok(fwd):
    """A set encoder with mean pooling: permuting the tokens permutes the
    per-slice head and leaves the pooled heads alone; repeating every token
    (the same set with each slice twice) changes neither pooled head."""
    R = 3
    theta, tok, *_ = _problem(5, K=6, R=R)
    pH, pV, pW, _ = fwd(theta, tok, R)
    perm = np.array([4, 0, 5, 2, 1, 3])
    qH, qV, qW, _ = fwd(theta, tok[perm], R)
    ok = np.allclose(qH, pH, atol=1e-12) and np.allclose(qV, pV, atol=1e-12) and \
        np.allclose(qW, pW[perm], atol=1e-12)
    dH, dV, dW, _ = fwd(theta, np.concatenate([tok, tok]), R)
    return ok and np.allclose(dH, pH, atol=1e-12) and np.allclose(dV, pV, atol=1e-12) and \
        np.allclose(dW, np.concatenate([pW, pW]), atol=1e-12)


def test_forward_is_a_mean_pooled_set_encoder():
    assert _set_encoder_ok(WO.forward)
    assert not _set_encoder_ok(_forward_sum_pool)


def _hand_network():
    """R = 1 (one feature per token) with every weight zero except a few, so
    the outputs can be worked out by hand (see the test)."""
    R = 1
    th = np.zeros(WO.n_params(R))
    P = WO.unpack(th, R)            # fill the blocks, then pack them back
    P["W1"][0, 0], P["W1"][1, 0] = 1.0, -1.0
    P["W2"][0, 0], P["W2"][0, 1], P["W2"][1, 0], P["W2"][1, 1] = 1.0, 1.0, -1.0, 2.0
    P["b2"][0], P["b2"][1] = -1.0, 0.5
    P["WH"][0, 0], P["WH"][0, 1], P["bH"][0] = 0.5, -1.0, 0.25
    P["WV"][0, 0], P["WV"][0, 1], P["bV"][0] = 2.0, 0.5, -1.0
    P["Ww"][0, 0], P["Ww"][0, WO.WIDTH], P["Ww"][0, WO.WIDTH + 1], P["bw"][0] = 1.0, 10.0, -1.0, 0.5
    return WO.pack(P, R), R


def test_forward_hand_computed_two_token_network():
    """Tokens 2 and -3.  Layer 1 (rows 1, -1 of W1): [2, 0] and [0, 3].
    Layer 2 (rows [1 1], [-1 2], bias [-1, 0.5]): [relu(1), relu(-1.5)] = [1, 0]
    and [relu(2), relu(6.5)] = [2, 6.5].  Mean pool p = [1.5, 3.25].
    pH = 0.5 * 1.5 - 3.25 + 0.25 = -2.25;  pV = 2 * 1.5 + 0.5 * 3.25 - 1 = 3.625;
    pW_k = Z2_k[0] + 10 p[0] - p[1] + 0.5 = 13.25 and 14.25."""
    th, R = _hand_network()
    pH, pV, pW, _ = WO.forward(th, np.array([[2.0], [-3.0]]), R)
    assert pH.shape == (1, 1) and pV.shape == (1, 1) and pW.shape == (2, 1)
    assert pH[0, 0] == -2.25 and pV[0, 0] == 3.625
    np.testing.assert_array_equal(pW[:, 0], [13.25, 14.25])
    sH, _, _, _ = _forward_sum_pool(th, np.array([[2.0], [-3.0]]), R)
    assert sH[0, 0] != -2.25


def _adam_no_bias_correction(theta, grad, m, v, step, lr, b1, b2, eps):
    """A deliberately broken Adam without the 1 - beta^t corrections."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    return theta - lr * m / (np.sqrt(v) + eps), m, v


def _constant_gradient_steps_are_sign_steps(adam):
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step (Kingma & Ba, Sec. 3), so with eps -> 0 each of the
    first steps moves every parameter by lr against the sign of g, for the
    usual beta1 = 0.9, beta2 = 0.999."""
    rng = np.random.default_rng(8)
    th0 = rng.standard_normal(40)
    g = rng.standard_normal(40) * 10.0 ** rng.uniform(-3, 3, 40)
    th, m, v = th0.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, 6):
        new, m, v = adam(th, g, m, v, t, 1e-2, 0.9, 0.999, 1e-300)
        if not np.allclose(new, th - 1e-2 * np.sign(g), rtol=0, atol=1e-12):
            return False
        th = new
    return True


def test_adam_bias_correction_with_usual_betas():
    assert _constant_gradient_steps_are_sign_steps(WO.adam)
    assert not _constant_gradient_steps_are_sign_steps(_adam_no_bias_correction)
