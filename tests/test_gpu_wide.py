"""GPU parity of the wide slab pass (J above 256 for float32, above 128 for
bf16 / fp8: the sketch kernel writes Y, the projection kernel forms G and P
per 128-column chunk on the FP64 matrix cores), through the C ABI, against
the FP64 oracle.  Same tolerances as the narrow path; ragged tiles (rows not a
multiple of 64), J not a multiple of 4 (scalar loads) and of 128 (partial last
chunk), both sketch widths (L <= 16 and L > 16), the U output, a power step
and the low-precision inputs."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import rel
from tests.test_gpu_forms import _lp_tensor
from tests.test_gpu_parity import _check_compression, _check_errors, _check_factors, _run_gpu

pytestmark = pytest.mark.gpu

# error-trace bounds of the power-step cases, from the CPU emulation of the
# slab pass (tests/golden/derive_parity_bounds.py, POWER_CASES)
BOUNDS = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "parity_bounds.json")))["bounds"]


def _check_errors_power(g, ref, case):
    """Per-iteration error with one power step: the GPU keeps each slice's
    next sketch matrix in FP32 (the oracle in FP64), and the early iterations
    of ALS from a random start amplify that difference; the relative bound is
    the emulation's deviation of the trace times 4 (at least 1e-6)."""
    e_ref = np.asarray(ref.state.errors)
    e0 = float(np.sum(ref.comp.E ** 2))
    dev = float(np.max(np.abs(g["err"] - e_ref) / e_ref))
    print(f"[wide] {case}: error trace {dev:.2e} (bound {BOUNDS[case]['errors']:.1e})", flush=True)
    np.testing.assert_allclose(g["err"], e_ref, rtol=BOUNDS[case]["errors"], atol=1e-12 * e0)


def _case(K, J, R, lo, hi, seed, noise=0.02):
    rows = synth.uniform_rows(K, lo, hi, seed)
    return synth.parafac2(rows, J, R, seed, noise_abs=noise)


@pytest.mark.parametrize("J,R,L,q", [(300, 5, 15, 0), (2049, 10, 20, 0), (517, 4, 12, 1)])
def test_wide_float32_matches_oracle(J, R, L, q):
    """K = 9 slices of 40..300 rows: J = 300 (4-element loads, L <= 16),
    J = 2049 (the precision-form width: scalar loads, 17 chunks, L = 20),
    J = 517 with one power step."""
    X = _case(9, J, R, 40, 300, seed=J)
    iters = 30
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters, q=q)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, power_iters=q)
    _check_compression(X, R, g, ref)
    if q == 0:
        _check_errors(g, ref)
    else:
        _check_errors_power(g, ref, f"wide_q1_J{J}")
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5
    assert g["rep"]["warn_bits"] == 0


@pytest.mark.parametrize("kind,J,q", [("bf16", 200, 0), ("fp8", 2049, 0), ("fp8", 2049, 1), ("bf16", 2049, 1)])
def test_wide_low_precision_matches_oracle_on_decoded(kind, J, q):
    """bf16 slab with J = 200 and fp8 with J = 2049 (above the narrow limit
    of 128), and both at J = 2049 with one power step (the precision form's
    accuracy recovery; the power step's sketch matrices on the FP32 matrix
    cores): parity with the oracle on the decoded slab and the bf16-rounded
    Omega_1."""
    R, L = 5, 12
    X = _case(8, J, R, 40, 200, seed=J + 7 + q)
    iters = 30
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    om1 = synth.round_bf16(om1)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    T, dec = _lp_tensor(X, kind)
    Xd = synth.IrregularTensor(slab=dec, offsets=X.offsets, H=X.H, V=X.V, W=X.W)
    ref = O.dpar2(dec, X.offsets, R, om1, om2, H0, V0, W0, iters, q=q)
    g = _run_gpu(Xd, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, T=T, power_iters=q)
    _check_compression(Xd, R, g, ref)
    if q == 0:
        _check_errors(g, ref)
    else:
        _check_errors_power(g, ref, f"wide_q1_J{J}_{kind}")
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5


def test_long_j_second_stage_rank_deficient_matches_oracle():
    """The second stage's J-long steps on one wave per 64 rows (J >= 512) on
    a noise-free rank-3 tensor at J = 600, whose M has rank 3 < L2 = 8 up to
    the float32 rounding of the slab (both whitening passes of Y2 take the
    eigen form, as do the slices' own sketches): compression, error trace,
    factors and fitness against the oracle at the usual bounds.  (The seed
    gives an error trace about as sensitive to the compression as the other
    parity cases: a 1e-7 relative change of D and F moves it by at most 4e-7
    over 30 iterations in the oracle; some draws of this shape amplify it a
    hundredfold, beyond what a 1e-6 bound can test.)  Rank 20 with L = 30 at
    J = 520 is a bounded case of test_gpu_coverage."""
    X, R, L = _case(30, 600, 3, 40, 160, seed=601, noise=0.0), 3, 8
    iters = 30
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
