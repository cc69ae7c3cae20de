"""FP64 CPU oracle for the learned warm start of the DPar2 iteration.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark may
import this module; the product path never calls it and shares no code with
it.

The paper starts Alg. 3 from arbitrary factors.  This extension proposes the
starting H, V, W with a small set encoder that reads the compressed
representation of Sec. III-B (M ~ D E F^T, F^(k) = rows kR .. kR+R-1 of F).

  features     per slice, Phi_k = (F^(k) E)^T (F^(k) E) in the basis of D
               with each column of D signed so that its largest-magnitude
               entry is positive; Phi_k does not depend on the per-slice
               rotation that the first stage leaves free (A_k O_k^T, O_k
               F^(k) give the same M), so it is a property of the tensor.
               Token k = upper triangle of R * Phi_k / e_mean, with
               e_mean = ||E||^2 / K the mean slice energy (F^T F = I).
  targets      converged factors brought to one gauge: unit-norm columns of
               H and V (scale moved into W), V expressed in that basis of D
               (V~ = D^T V; V lies in span(D) after one V update, Lemma 2),
               each V~ column signed by its largest-magnitude entry, each
               column of W signed to a non-negative sum (flipping the same
               column of H), components sorted by ||W(:, r)|| descending.
               Targets: H^T H (only H^T H is identifiable: Q_k absorbs any
               rotation of H), V~, and W / sqrt(e_mean / R).
  forward      two ReLU layers of width 128 per token, mean pooling, and
               three linear heads: H (R x R) and V~ (R x R) from the pooled
               vector, W(k, :) from [token k ; pooled].
  loss         ||H^T H - T_H||^2 / R^2 + ||V~ - T_V||^2 / R^2
               + sum_k ||W_k - T_W,k||^2 / (K R).
  backward     gradient of that loss with respect to every parameter.
  apply        H = predicted H, V = D' V~, W = predicted W * sqrt(e_mean / R).
"""
import numpy as np

WIDTH = 128


def n_features(R):
    return R * (R + 1) // 2


def param_shapes(R):
    """Parameter blocks in storage order (row-major, float32 on the GPU)."""
    F, Hd, RR = n_features(R), WIDTH, R * R
    return [("W1", (Hd, F)), ("b1", (Hd,)), ("W2", (Hd, Hd)), ("b2", (Hd,)),
            ("WH", (RR, Hd)), ("bH", (RR,)), ("WV", (RR, Hd)), ("bV", (RR,)),
            ("Ww", (R, 2 * Hd)), ("bw", (R,))]


def n_params(R):
    return int(sum(np.prod(s) for _, s in param_shapes(R)))


def unpack(theta, R):
    out, at = {}, 0
    for name, shp in param_shapes(R):
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[at:at + n], dtype=np.float64).reshape(shp)
        at += n
    return out


def pack(grads, R):
    return np.concatenate([np.asarray(grads[name], dtype=np.float64).ravel() for name, _ in param_shapes(R)])


def sign_basis(D):
    """D with each column signed so that its largest-magnitude entry (lowest
    index on ties) is positive."""
    D = np.asarray(D, dtype=np.float64)
    idx = np.argmax(np.abs(D), axis=0)
    s = np.sign(D[idx, np.arange(D.shape[1])])
    s[s == 0] = 1.0
    return D * s, s


def features(F, E, D, K, R):
    """Tokens (K x R(R+1)/2) and e_mean from the compressed representation."""
    _, s = sign_basis(D)
    e_mean = float(np.sum(np.asarray(E, dtype=np.float64) ** 2)) / K
    iu = np.triu_indices(R)
    tok = np.empty((K, n_features(R)))
    for k in range(K):
        Fk = np.asarray(F[k * R:(k + 1) * R], dtype=np.float64) * E[None, :] * s[None, :]
        Phi = Fk.T @ Fk
        tok[k] = (R * Phi / e_mean)[iu]
    return tok, e_mean


def targets(H, V, W, D, e_mean, R):
    """(T_H, T_V, T_W) of converged factors in the gauge described above."""
    H = np.array(H, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    nH = np.linalg.norm(H, axis=0)
    nV = np.linalg.norm(V, axis=0)
    nH[nH == 0] = 1.0
    nV[nV == 0] = 1.0
    Hc, Vc, Wc = H / nH, V / nV, W * (nH * nV)
    Ds, _ = sign_basis(D)
    Vt = Ds.T @ Vc
    for r in range(R):
        i = int(np.argmax(np.abs(Vt[:, r])))
        if Vt[i, r] < 0:
            Vt[:, r] *= -1.0
            Wc[:, r] *= -1.0
        if Wc[:, r].sum() < 0:
            Hc[:, r] *= -1.0
            Wc[:, r] *= -1.0
    order = sorted(range(R), key=lambda r: (-np.linalg.norm(Wc[:, r]), r))
    Hc, Vt, Wc = Hc[:, order], Vt[:, order], Wc[:, order]
    return Hc.T @ Hc, Vt, Wc / np.sqrt(e_mean / R)


def forward(theta, tok, R):
    """Returns (pH (R x R), pV (R x R), pW (K x R), cache)."""
    P = unpack(theta, R)
    x = np.asarray(tok, dtype=np.float64)
    K = x.shape[0]
    Z1 = np.maximum(x @ P["W1"].T + P["b1"], 0.0)
    Z2 = np.maximum(Z1 @ P["W2"].T + P["b2"], 0.0)
    p = Z2.mean(axis=0)
    pH = (P["WH"] @ p + P["bH"]).reshape(R, R)
    pV = (P["WV"] @ p + P["bV"]).reshape(R, R)
    cat = np.concatenate([Z2, np.broadcast_to(p, (K, WIDTH))], axis=1)
    pW = cat @ P["Ww"].T + P["bw"]
    return pH, pV, pW, dict(x=x, Z1=Z1, Z2=Z2, p=p, cat=cat, P=P)


def loss(pH, pV, pW, tH, tV, tW, R):
    K = pW.shape[0]
    G = pH.T @ pH
    return (np.sum((G - tH) ** 2) / R ** 2, np.sum((pV - tV) ** 2) / R ** 2,
            np.sum((pW - tW) ** 2) / (K * R))


def backward(pH, pV, pW, tH, tV, tW, cache, R):
    """Gradient of the summed loss (flat, in storage order)."""
    P, x, Z1, Z2, p, cat = (cache[k] for k in ("P", "x", "Z1", "Z2", "p", "cat"))
    K = x.shape[0]
    dG = 2.0 * (pH.T @ pH - tH) / R ** 2
    dHp = pH @ (dG + dG.T)
    dV = 2.0 * (pV - tV) / R ** 2
    dW = 2.0 * (pW - tW) / (K * R)
    g = {}
    g["WH"] = np.outer(dHp.ravel(), p)
    g["bH"] = dHp.ravel()
    g["WV"] = np.outer(dV.ravel(), p)
    g["bV"] = dV.ravel()
    g["Ww"] = dW.T @ cat
    g["bw"] = dW.sum(axis=0)
    dp = P["WH"].T @ dHp.ravel() + P["WV"].T @ dV.ravel() + P["Ww"][:, WIDTH:].T @ dW.sum(axis=0)
    dZ2 = dW @ P["Ww"][:, :WIDTH] + dp[None, :] / K
    dA2 = dZ2 * (Z2 > 0)
    g["W2"] = dA2.T @ Z1
    g["b2"] = dA2.sum(axis=0)
    dA1 = (dA2 @ P["W2"]) * (Z1 > 0)
    g["W1"] = dA1.T @ x
    g["b1"] = dA1.sum(axis=0)
    return pack(g, R)


def adam(theta, grad, m, v, step, lr, b1, b2, eps):
    """One Adam step (Kingma & Ba, Alg. 1, with bias correction); returns
    the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def apply(pH, pV, pW, D, e_mean, R):
    """Initial factors (H, V, W) from the network outputs."""
    Ds, _ = sign_basis(D)
    return np.array(pH, dtype=np.float64), Ds @ pV, np.asarray(pW) * np.sqrt(e_mean / R)
