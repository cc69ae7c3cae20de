"""GPU parity (through the C ABI) on the configurations the other parity tests
leave out, with bounds derived from a CPU emulation of the slab pass's
rounding (tests/golden/derive_parity_bounds.py writes
tests/golden/parity_bounds.json: the largest deviation of the emulated
arithmetic from the FP64 oracle times a safety factor of 4, per check and
case), and per-row checks next to the Frobenius ones:

  * M (J x KR) and V (J x R) row by row: max_j ||row_gpu - row_ref|| /
    ||row_ref||, so that the small-scale feature rows of the stock-shaped
    tensor (feature scales over five decades) cannot hide behind the large
    ones;
  * a 64-row tile with one row 1e4 times larger than the rest of each of its
    columns (the 22-bit fixed point of that tile keeps few bits for the other
    rows);
  * rank 20 with L = 30 on a J = 128 tensor (the batching form's largest rank
    and widest J bucket; k_als_A<20>, k_slice_fin<30>, the second stage at
    L2 = 30), and on a J = 520 tensor (the wide slab pass at L = 30 and the
    second stage's J-long steps spread over 64-row waves);
  * float32 slabs with 128 < J <= 256 (the FP64 matrix-core Gram and
    projection), with 4-element and scalar loads;
  * the rank instantiations R = 12 (L = 22) and R = 28 (L = 32, four
    oversampled columns only);
  * the ranks above 32: R = 40 with L = 50 at J = 600 (the second stage's
    J-long steps), R = L = 40 at J = 96 (the chunked slab pass below the
    whole-row limit, taken for every J above L = 32) and R = 50 with L = 60
    at J = 300 (one slice per 64-lane block in the iteration, four
    16-column tiles of Y in the slab pass)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import canonical, match_columns, model_tensor, rel
from tests.golden.derive_parity_bounds import CASES
from tests.test_gpu_parity import _check_compression, _check_errors, _check_factors, _run_gpu

pytestmark = pytest.mark.gpu

BOUNDS = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "parity_bounds.json")))["bounds"]


def row_rel(a, b):
    nb = np.linalg.norm(b, axis=1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.where(nb > 0, nb, 1.0)))


@pytest.mark.parametrize("case", sorted(CASES))
def test_bounded_case(case):
    make, R, L, iters = CASES[case]
    X = make()
    b = BOUNDS[case]
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True)
    c = ref.comp
    # compression (first and second stage)
    np.testing.assert_allclose(g["comp"]["xnorm2"], c.xnorm2, rtol=1e-12)
    assert np.max(np.abs(g["comp"]["sigma"] - c.Bdiag) / c.Bdiag) < b["sigma"]
    Mg = g["comp"]["Mt"].T
    assert rel(Mg, c.M) < b["M"], rel(Mg, c.M)
    assert row_rel(Mg, c.M) < b["M_rows"], row_rel(Mg, c.M)
    assert np.max(np.abs(g["comp"]["E"] - c.E) / c.E) < b["E"]
    s = match_columns(g["comp"]["D"], c.D)
    assert rel(g["comp"]["D"] * s, c.D) < b["D"]
    assert rel(g["comp"]["F"] * s, c.F) < b["F"]
    # factors, U_k, fitness
    st = ref.state
    Hg, Vg, Wg = canonical(g["H"], g["V"], g["W"])
    Hr, Vr, Wr = canonical(st.H, st.V, st.W)
    assert rel(Vg, Vr) < b["V"], rel(Vg, Vr)
    assert row_rel(Vg, Vr) < b["V_rows"], row_rel(Vg, Vr)
    assert rel(Wg, Wr) < b["W"], rel(Wg, Wr)
    assert rel(model_tensor(g["H"], g["V"], g["W"]), model_tensor(st.H, st.V, st.W)) < b["model"]
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < b["U"]
    assert abs(g["rep"]["fit_true"] - ref.fit) < b["fit"]
    print(f"[coverage] {case}: M rows {row_rel(Mg, c.M):.2e} (bound {b['M_rows']:.1e}), "
          f"V rows {row_rel(Vg, Vr):.2e} (bound {b['V_rows']:.1e}), |dfit| {abs(g['rep']['fit_true'] - ref.fit):.1e}",
          flush=True)


@pytest.mark.parametrize("J", [200, 150])
def test_fp64_matrix_core_pass_matches_oracle(J):
    """float32 slab, 128 < J <= 256: the Gram and projection on the FP64
    matrix cores from the float32 sketch; J = 200 with 4-element loads,
    J = 150 with scalar loads; compression within the 1e-6 bound of the
    narrow path, factors within 1e-5, U_k, fitness within 1e-7."""
    rows = synth.uniform_rows(14, 40, 400, J)
    X = synth.parafac2(rows, J, 6, J, noise_abs=0.02)
    R, L, iters = 6, 16, 30
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert row_rel(g["comp"]["Mt"].T, ref.comp.M) < 1e-6
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5


def test_rank_deficient_sketch_takes_the_eigen_whitening():
    """Slices whose sketch Y_k = X_k Omega_1 has rank 5 < L = 8 (X_k of rank 5
    up to its float32 rounding, no noise: the Gram's last pivots sit at the
    rounding level, far below 1e-9 of its largest diagonal), between
    noisy rank-3 slices: those slices take the eigen form of the whitening.
    R = 3 < 5, so their leading triplets are well defined and the same
    tolerances as elsewhere apply: compression, factors, U_k, fitness."""
    rng = np.random.default_rng(23)
    J, R, L = 24, 3, 8
    X0 = synth.parafac2(synth.uniform_rows(20, 40, 120, 23), J, R, 23, noise_abs=0.02)
    slab = X0.slab.copy()
    deficient = [2, 7, 11, 18]
    for k in deficient:
        n = X0.offsets[k + 1] - X0.offsets[k]
        A = rng.standard_normal((n, 5))
        B = rng.standard_normal((J, 5)) * np.array([3.0, 2.2, 1.5, 0.8, 0.4])
        slab[X0.offsets[k]:X0.offsets[k + 1]] = (A @ B.T).astype(np.float32)
    X = synth.IrregularTensor(slab=slab, offsets=X0.offsets)
    iters = 30
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    # those slices' sketches have rank 5 up to the float32 rounding of the
    # slab: their Gram's sixth eigenvalue lies below 1e-12 of the largest,
    # far below the 1e-9 pivot threshold of the Cholesky whitening
    for k in deficient:
        Y = X.slab[X.offsets[k]:X.offsets[k + 1]].astype(np.float64) @ om1
        s = np.linalg.svd(Y, compute_uv=False)
        assert s[5] < 1e-6 * s[0]
    print("[gpu] eigen whitening", flush=True)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5
