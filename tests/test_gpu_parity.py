"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs.  Tolerances: factors within 1e-5 relative (up to the sign and
scale gauges of PARAFAC2), fitness within 1e-4 absolute (tested tighter
where the arithmetic allows), and the compressed intermediates within the
FP32 rounding of the sketch."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import canonical, match_columns, model_tensor, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run_gpu(X, R, L, L2, iters, om1, om2, H0, V0, W0, tol=-1.0, want_U=False, trace=True, T=None,
             power_iters=0, wide_slab=False):
    torch = _torch()
    import paper_2203_12798_amd as d
    print(f"[gpu] K={X.K} J={X.J} N={X.N} R={R} L={L} L2={L2} iters={iters} q={power_iters}"
          f"{'' if T is None else ' dtype=' + str(T.dtype)}{' wide slab pass' if wide_slab else ''}", flush=True)
    if T is None:
        T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=L, sketch2=L2, max_iter=iters, tol=tol, power_iters=power_iters,
                  wide_slab=wide_slab)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_workspace(T, o)
    o1 = torch.from_numpy(om1).cuda()
    o2 = torch.from_numpy(om2).cuda()
    d.compress(T, o, o1, o2, ws)
    comp = d.compressed_view(T, o, ws)
    et = torch.zeros(max(iters, 1), dtype=torch.float64, device="cuda")
    d.als_step(T, o, f, iters, ws, err_trace=et if trace else None)
    d.fitness(T, o, f, ws)
    U = None
    if want_U:
        U = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
        d.output_U(T, o, f, U, ws)
    rep = d.report_read(T, o, ws)
    H, V, W = f.numpy()
    return dict(comp=comp, rep=rep, H=H, V=V, W=W, err=et.cpu().numpy()[:rep["iters"]],
                U=None if U is None else U.cpu().numpy())


def _check_compression(X, R, g, ref, tol_m=1e-6):
    """The slab pass forms the sketch Y = X Omega_1 with FP32-level error and then
    represents Y and X in 22-bit fixed point per column of each 64-row tile
    (error at most 2^-22 of that column's maximum); the Gram, the projection
    and everything after them are exact or FP64.  A CPU emulation of exactly
    this arithmetic differs from the FP64 oracle by at most 4.6e-7 (sigma, on
    the minimal-rows case) and 5.3e-7 (stock-shaped, K=120).  Bound: 1e-6
    relative."""
    c = ref.comp
    K, J = X.K, X.J
    np.testing.assert_allclose(g["comp"]["xnorm2"], c.xnorm2, rtol=1e-12)
    np.testing.assert_allclose(g["comp"]["sigma"], c.Bdiag, rtol=tol_m)
    Mg = g["comp"]["Mt"].T                                   # J x KR
    assert rel(Mg, c.M) < tol_m, rel(Mg, c.M)
    np.testing.assert_allclose(g["comp"]["E"], c.E, rtol=tol_m)
    s = match_columns(g["comp"]["D"], c.D)
    assert rel(g["comp"]["D"] * s, c.D) < tol_m
    assert rel(g["comp"]["F"] * s, c.F) < tol_m


def _check_errors(g, ref):
    """Per-iteration error e_t of Sec. III-E.  The GPU evaluates it in closed
    form, e0 - 2 sum W.G3 + sum W (H^T H * V^T V) W^T, whose cancellation
    leaves an absolute rounding error of a few eps64 * e0; the oracle forms
    the R x J residuals explicitly."""
    e_ref = np.asarray(ref.state.errors)
    e0 = float(np.sum(ref.comp.E ** 2))
    np.testing.assert_allclose(g["err"], e_ref, rtol=1e-6, atol=1e-12 * e0)


def _check_factors(g, ref, tol=1e-5):
    st = ref.state
    mg, mr = model_tensor(g["H"], g["V"], g["W"]), model_tensor(st.H, st.V, st.W)
    assert rel(mg, mr) < tol, rel(mg, mr)
    Hg, Vg, Wg = canonical(g["H"], g["V"], g["W"])
    Hr, Vr, Wr = canonical(st.H, st.V, st.W)
    assert rel(Vg, Vr) < tol, rel(Vg, Vr)
    assert rel(Wg, Wr) < tol, rel(Wg, Wr)
    assert rel(Hg.T @ Hg, Hr.T @ Hr) < tol


def test_small_parity_end_to_end():
    """64 slices, J=32, I_k in [50, 200], rank-5 PARAFAC2 + 0.01 noise, R=5,
    L=15, 100 iterations."""
    X = synth.small_parity()
    R, L, iters = 5, 15, 100
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True)
    _check_compression(X, R, g, ref)
    assert g["rep"]["iters"] == iters
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    Ug = g["U"]
    Ur = np.concatenate(ref.U, axis=0)
    assert rel(Ug, Ur) < 1e-5, rel(Ug, Ur)
    assert g["rep"]["warn_bits"] == 0


@pytest.mark.parametrize("exp2", [-110, 100])
def test_extreme_magnitudes_match_oracle(exp2):
    """The small-parity tensor times 2^-110 and times 2^100 (exact power-of-two
    scalings).  The slab pass scales each column of each 64-row tile by a
    power of two before its 22-bit fixed point; at 2^-110 every column maximum
    of X and of Y lies below 2^-104, where that power of two leaves the FP32
    range and the column is pre-multiplied by 2^64.  Every comparison is
    relative, as in the unscaled case."""
    X0 = synth.small_parity(seed=5)
    assert np.abs(X0.slab).max() < 32.0
    X = synth.IrregularTensor(slab=(X0.slab * np.float32(2.0 ** exp2)).astype(np.float32),
                              offsets=X0.offsets)
    R, L, iters = 5, 15, 40
    print(f"[gpu] magnitudes 2^{exp2}", flush=True)
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert g["rep"]["warn_bits"] == 0


def test_stock_like_scaled_down():
    """US-Stock-shaped slices (J=88, lognormal I_k, feature scales over
    1e-2..1e3, 5% noise), 120 slices, R=10, L=20, 32 iterations."""
    X = synth.stock_like(K=120)
    R, L, iters = 10, 20, 32
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-6


@pytest.mark.parametrize("case", ["minimal_rows", "odd_J_scalar_path", "long_slice_split", "rank_one"])
def test_ragged_edge_cases(case):
    """Slices with exactly L rows, tail tiles, J not a multiple of 4 (scalar
    loads), a slice longer than one work item (split and re-summed), R = 1."""
    if case == "minimal_rows":
        rows = np.array([12, 12, 64, 65, 127, 12, 200], dtype=np.int64)
        X, R, L = synth.parafac2(rows, 20, 4, 31, noise_abs=0.05), 4, 12
    elif case == "odd_J_scalar_path":
        rows = synth.uniform_rows(9, 40, 150, 32)
        X, R, L = synth.parafac2(rows, 37, 3, 32, noise_abs=0.05), 3, 7
    elif case == "long_slice_split":
        rows = np.array([40000, 300, 20000, 17], dtype=np.int64)
        X, R, L = synth.parafac2(rows, 16, 3, 33, noise_abs=0.05), 3, 8
    else:
        rows = synth.uniform_rows(6, 10, 80, 34)
        X, R, L = synth.parafac2(rows, 9, 1, 34, noise_abs=0.05), 1, 4
    iters = 25
    L2 = min(L, X.K * R)
    om1, om2 = synth.omegas(X.J, L, X.K * R, L2=L2)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L2, iters, om1, om2, H0, V0, W0, want_U=True)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-6
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5


def test_tolerance_stop_matches_oracle():
    X = synth.small_parity(seed=5)
    R, L, iters, tol = 5, 15, 200, 5e-3
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters, tol=tol)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, tol=tol)
    assert ref.state.iters < iters
    assert g["rep"]["iters"] == ref.state.iters
    assert g["rep"]["converged"]
    _check_errors(g, ref)


def test_resume_and_determinism():
    """Two identical runs agree bit for bit (every reduction has a fixed
    order, no floating-point atomics); 16 + 16 iterations equal 32 to 1e-9
    (a new call re-derives W^T W, V^T V and E D^T V from the factors it is
    given, with its own rounding)."""
    torch = _torch()
    import paper_2203_12798_amd as d
    X = synth.small_parity(seed=6)
    R, L = 5, 15
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=32)
    o1, o2 = torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda()
    outs = []
    for split in (False, False, True):
        f = d.Factors.from_numpy(H0, V0, W0)
        ws = d.alloc_workspace(T, o)
        d.compress(T, o, o1, o2, ws)
        if split:
            d.als_step(T, o, f, 16, ws)
            d.als_step(T, o, f, 16, ws)
        else:
            d.als_step(T, o, f, 32, ws)
        rep = d.report_read(T, o, ws)
        outs.append((f.numpy(), rep["err_last"], rep["iters"]))
    (Ha, Va, Wa), ea, ia = outs[0]
    (Hb, Vb, Wb), eb, ib = outs[1]
    assert ea == eb and ia == ib == 32
    assert np.array_equal(Ha, Hb) and np.array_equal(Va, Vb) and np.array_equal(Wa, Wb)
    (Hc, Vc, Wc), ec, ic = outs[2]
    assert ic == 32
    assert abs(ec - ea) <= 1e-9 * ea
    assert rel(model_tensor(Hc, Vc, Wc), model_tensor(Ha, Va, Wa)) < 1e-8


def test_exact_low_rank_reaches_fit_one():
    """Noise-free rank-R PARAFAC2 data from a 1%-perturbed start: the GPU path
    reaches fitness 1 within 1e-10, like the oracle."""
    X = synth.exact_parafac2(22, K=64, J=32, rank=5, imin=20, imax=40)
    R, L, iters = 5, 7, 200
    rng = np.random.default_rng(8)
    H0 = X.H * (1 + 0.01 * rng.standard_normal(X.H.shape))
    V0 = X.V * (1 + 0.01 * rng.standard_normal(X.V.shape))
    W0 = X.W * (1 + 0.01 * rng.standard_normal(X.W.shape))
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, trace=False)
    assert 1.0 - g["rep"]["fit_true"] < 1e-10, g["rep"]
