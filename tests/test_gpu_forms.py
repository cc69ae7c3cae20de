"""GPU parity of the power iteration of Alg. 1 (q = 1) and of the low-precision
slab inputs (bfloat16, fp8 e4m3 with per-slice power-of-two scales), through
the C ABI.

For bf16 / fp8 slabs the oracle runs on the decoded values and on Omega_1
rounded to bf16 -- exactly the inputs the GPU sketches with -- so the same
tolerances as the float32 path apply.  The accuracy cost of the encoding
itself is reported against the oracle on the original float32 data
(|delta fitness| <= 1e-3)."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import rel
from tests.test_gpu_parity import _check_compression, _check_errors, _check_factors, _run_gpu, _torch

pytestmark = pytest.mark.gpu


def _case(K=48, J=32, R=5, L=12, seed=41):
    rows = synth.uniform_rows(K, 40, 300, seed)
    X = synth.parafac2(rows, J, R, seed, noise_abs=0.02)
    return X, R, L


def _lp_tensor(X, kind):
    _torch()
    import paper_2203_12798_amd as d
    if kind == "bf16":
        bits = synth.encode_bf16(X.slab)
        return d.Tensor.from_numpy(bits, X.offsets, dtype=d.binding.DPAR2_BF16), synth.decode_bf16(bits)
    codes, scale = synth.encode_fp8(X.slab, X.offsets)
    T = d.Tensor.from_numpy(codes, X.offsets, dtype=d.binding.DPAR2_FP8_E4M3, scale=scale)
    return T, synth.decode_fp8(codes, X.offsets, scale)


def test_power_iteration_q1_matches_oracle():
    """q = 1 (stabilised power step; the slab is read twice) on float32."""
    X, R, L = _case()
    iters = 40
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters, q=1)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, power_iters=1)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_low_precision_slab_matches_oracle_on_decoded(kind):
    """bf16 / fp8 slab, sketch on the bf16 matrix cores: parity with the oracle
    on the decoded slab and the bf16-rounded Omega_1."""
    X, R, L = _case(seed=42 if kind == "bf16" else 43)
    iters = 40
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    om1 = synth.round_bf16(om1)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    T, dec = _lp_tensor(X, kind)
    Xd = synth.IrregularTensor(slab=dec, offsets=X.offsets, H=X.H, V=X.V, W=X.W)
    ref = O.dpar2(dec, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(Xd, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, T=T)
    _check_compression(Xd, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5
    # cost of the encoding: against the oracle on the original float32 slab
    ref32 = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    print(f"[forms] {kind}: fitness {g['rep']['fit_true']:.6f} vs float32 oracle {ref32.fit:.6f}", flush=True)
    assert abs(g["rep"]["fit_true"] - ref32.fit) < 1e-3


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_low_precision_with_power_step(kind):
    """bf16 / fp8 slab with q = 1: the first pass sketches with Omega_1 rounded
    to bf16 (as the oracle does), the power step's per-slice sketch matrices
    are split into three bf16 pieces (float32-level products, like a float32
    slab's), so the same bounds as the float32 power step apply against the
    oracle on the decoded slab."""
    X, R, L = _case(seed=44 if kind == "bf16" else 45)
    iters = 40
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    om1 = synth.round_bf16(om1)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    T, dec = _lp_tensor(X, kind)
    Xd = synth.IrregularTensor(slab=dec, offsets=X.offsets, H=X.H, V=X.V, W=X.W)
    ref = O.dpar2(dec, X.offsets, R, om1, om2, H0, V0, W0, iters, q=1)
    g = _run_gpu(Xd, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, T=T, power_iters=1)
    _check_compression(Xd, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    print(f"[forms] {kind} q=1: fitness {g['rep']['fit_true']:.8f} vs oracle {ref.fit:.8f}", flush=True)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5


@pytest.mark.parametrize("wide", [False, True])
def test_every_fp8_code_decodes_exactly(wide):
    """Every finite e4m3 code, both signs: slice k (of 8, 64 rows of J = 32)
    holds the codes 16 k .. 16 k + 15 (zero, the subnormals and every binade)
    with random signs, scaled by 2^(k - 4).  ||X_k||^2 of every slice equals
    the sum of the exactly decoded values (FP64 on both sides: 1e-13); within a
    slice the codes span two binades, so any code decoded wrongly moves its
    slice's sum by more than 1e-3.  Whole-row and 128-column-chunk passes."""
    torch = _torch()
    import paper_2203_12798_amd as d
    rng = np.random.default_rng(17)
    K, I, J = 8, 64, 32
    codes = np.zeros((K * I, J), dtype=np.uint8)
    for k in range(K):
        lo, hi = 16 * k, min(16 * k + 16, 127)          # 0x7f (NaN) excluded
        c = rng.integers(lo, hi, size=(I, J)).astype(np.uint8)
        codes[k * I:(k + 1) * I] = c | (rng.integers(0, 2, size=(I, J)) * 0x80).astype(np.uint8)
    offsets = np.arange(K + 1, dtype=np.int64) * I
    scale = np.exp2(np.arange(K) - 4.0).astype(np.float32)
    dec = synth.decode_fp8(codes, offsets, scale).astype(np.float64)
    ref = np.array([np.sum(dec[k * I:(k + 1) * I] ** 2) for k in range(K)])
    T = d.Tensor.from_numpy(codes, offsets, dtype=d.binding.DPAR2_FP8_E4M3, scale=scale)
    R, L = 4, 8
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=1, wide_slab=wide)
    om1, om2 = synth.omegas(J, L, K * R)
    ws = d.alloc_workspace(T, o)
    print(f"[gpu] fp8 codes wide={wide}", flush=True)
    d.compress(T, o, torch.from_numpy(synth.round_bf16(om1)).cuda(), torch.from_numpy(om2).cuda(), ws)
    got = d.compressed_view(T, o, ws)["xnorm2"]
    np.testing.assert_allclose(got, ref, rtol=1e-13)
