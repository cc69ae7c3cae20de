"""Streaming DPar2 on the GPU (dpar2_append, through the C ABI): slices
appended to a decomposed tensor get the first stage alone, the second stage
runs again over the whole M, Alg. 3 iterates from the given factors.

  * bit for bit equal to dpar2_decompose on the grown tensor from the same
    factors (the per-slice arithmetic is the same: the slab-pass items of a
    slice and their order do not depend on the other slices), for float32
    narrow and wide slabs, fp8 with per-slice scales, q = 1 and slices cut
    into several work items, and over two appends in a row (one of a single
    slice);
  * against the streaming oracle (which equals the batch oracle on the grown
    tensor) at the parity tolerances of the batch path;
  * a warm start from the previous factors reaches the stop rule in fewer
    iterations than the cold start and within 1e-4 of its fitness."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from oracle import stream_oracle as S
from tests._helpers import rel
from tests.test_gpu_forms import _lp_tensor
from tests.test_gpu_parity import _check_compression, _check_errors, _check_factors

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _views(d, T, K):
    """The first K slices of T (same device slab, offsets and scales)."""
    return d.Tensor(T.slab, T.offsets_dev, T.offsets_host[:K + 1].copy(), T.dtype, T.scale)


def _result(d, T, o, ws, f, U):
    H, V, W = f.numpy()
    return dict(comp=d.compressed_view(T, o, ws), rep=d.report_read(T, o, ws), H=H, V=V, W=W,
                U=None if U is None else U.cpu().numpy())


def _same(a, b):
    for k in ("H", "V", "W", "U"):
        if a[k] is not None or b[k] is not None:
            assert np.array_equal(a[k], b[k]), k
    for k in a["comp"]:
        assert np.array_equal(a["comp"][k], b["comp"][k]), k
    assert a["rep"] == b["rep"], (a["rep"], b["rep"])


def _stream_vs_full(X, T, R, L, iters, cuts, q=0, item_rows=0, wide=False, om1=None):
    """Decompose the first cuts[0] slices, append up to each next cut, and
    decompose all slices in one call; returns (streamed, full, inputs)."""
    torch = _torch()
    import paper_2203_12798_amd as d
    K = X.K
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, power_iters=q, item_rows=item_rows,
                  wide_slab=wide)
    if om1 is None:
        om1, om2 = synth.omegas(X.J, L, K * R)
    else:
        _, om2 = synth.omegas(X.J, L, K * R)
    H0, V0, W0 = synth.init_factors(X.J, K, R)
    o1, o2 = torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda()
    print(f"[gpu] stream K={K} J={X.J} R={R} L={L} q={q} cuts={cuts} item_rows={item_rows} wide={wide} "
          f"dtype={T.dtype}", flush=True)
    k0 = cuts[0]
    Tp = _views(d, T, k0)
    ws = d.alloc_workspace(Tp, o)
    d.decompose(Tp, o, o1, o2[:k0 * R].contiguous(), d.Factors.from_numpy(H0, V0, W0[:k0]), ws)
    for k1 in cuts[1:] + [K]:
        Tk = _views(d, T, k1)
        wsn = d.alloc_append_workspace(Tk, k0, o)
        f = d.Factors.from_numpy(H0, V0, W0[:k1])
        U = torch.zeros((int(Tk.offsets_host[-1]), R), dtype=torch.float64, device="cuda")
        d.append(Tk, k0, o, o1, o2[:k1 * R].contiguous(), ws, f, wsn, U=U)
        d.release(ws)
        ws, k0 = wsn, k1
    streamed = _result(d, T, o, ws, f, U)
    wsf = d.alloc_workspace(T, o)
    ff = d.Factors.from_numpy(H0, V0, W0)
    Uf = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    d.decompose(T, o, o1, o2, ff, wsf, U=Uf)
    full = _result(d, T, o, wsf, ff, Uf)
    d.release(ws)
    d.release(wsf)
    return streamed, full, (om1, om2, H0, V0, W0)


def test_append_equals_decompose_and_matches_oracle():
    """60 slices of 40..300 rows, J = 32, R = 5, L = 12, 40 iterations: 45
    decomposed, 15 appended.  Bit for bit the single-call decomposition;
    against the streaming oracle at the batch path's bounds."""
    _torch()
    import paper_2203_12798_amd as d
    X = synth.parafac2(synth.uniform_rows(60, 40, 300, 31), 32, 5, 31, noise_abs=0.02)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    R, L, iters = 5, 12, 40
    g, full, (om1, om2, H0, V0, W0) = _stream_vs_full(X, T, R, L, iters, [45])
    _same(g, full)
    off = np.asarray(X.offsets)
    prev = O.compress(X.slab[:off[45]], off[:46], R, om1, om2[:45 * R])
    ref = S.dpar2_append(prev, X.slab, X.offsets, 45, R, om1, om2, H0, V0, W0, iters)
    _check_compression(X, R, g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-7
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < 1e-5
    assert g["rep"]["warn_bits"] == 0


@pytest.mark.parametrize("kind", ["q1_cut_items", "wide_J300", "long_J600", "fp8", "rank40_J300"])
def test_two_appends_equal_decompose(kind):
    """Two appends in a row (20 -> 21 -> 48 slices, the first of a single
    slice): with q = 1 and 64-row work items (every slice cut into several
    items), with the wide slab pass at J = 300, at J = 600 (the second
    stage's J-long steps spread over 64-row waves), with an fp8 slab (the
    per-slice scales of the new slices), and at rank 40 (L = 50); bit for bit
    the single call."""
    _torch()
    import paper_2203_12798_amd as d
    if kind == "rank40_J300":
        X = synth.parafac2(synth.uniform_rows(48, 60, 200, 9), 300, 40, 9, noise_abs=0.02)
        T = d.Tensor.from_numpy(X.slab, X.offsets)
        g, full, _ = _stream_vs_full(X, T, 40, 50, 6, [20, 21])
        _same(g, full)
        return
    J = {"wide_J300": 300, "long_J600": 600}.get(kind, 24)
    X = synth.parafac2(synth.uniform_rows(48, 40, 260, 7), J, 4, 7, noise_abs=0.02)
    om1 = None
    if kind == "fp8":
        T, _ = _lp_tensor(X, "fp8")
        om1 = synth.round_bf16(synth.omegas(X.J, 10, X.K * 4)[0])
    else:
        T = d.Tensor.from_numpy(X.slab, X.offsets)
    g, full, _ = _stream_vs_full(X, T, 4, 10, 25, [20, 21], q=1 if kind == "q1_cut_items" else 0,
                                 item_rows=64 if kind == "q1_cut_items" else 0, om1=om1)
    _same(g, full)


def test_warm_start_after_append():
    """After appending 10 slices to 50, Alg. 3 from the previous H and V
    (and the mean of the previous W rows for the new slices) stops (tol
    1e-5) in fewer iterations than from the random start, at a fitness
    within 1e-4 of it."""
    torch = _torch()
    import paper_2203_12798_amd as d
    X = synth.parafac2(synth.uniform_rows(60, 40, 300, 41), 32, 5, 41, noise_abs=0.02)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    R, L = 5, 12
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=1000, tol=1e-5)
    o1, o2 = torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda()
    Tp = _views(d, T, 50)
    ws = d.alloc_workspace(Tp, o)
    fp = d.Factors.from_numpy(H0, V0, W0[:50])
    d.decompose(Tp, o, o1, o2[:50 * R].contiguous(), fp, ws, report=True)
    Hp, Vp, Wp = fp.numpy()
    wsn = d.alloc_append_workspace(T, 50, o)
    Ww = np.concatenate([Wp, np.repeat(Wp.mean(axis=0, keepdims=True), 10, axis=0)])
    print("[gpu] stream warm start", flush=True)
    warm = d.append(T, 50, o, o1, o2, ws, d.Factors.from_numpy(Hp, Vp, Ww), wsn, report=True)
    cold = d.append(T, 50, o, o1, o2, ws, d.Factors.from_numpy(H0, V0, W0), wsn, report=True)
    print(f"[stream] warm {warm['iters']} iterations fit {warm['fit_true']:.8f}; "
          f"cold {cold['iters']} iterations fit {cold['fit_true']:.8f}", flush=True)
    assert warm["status"] == 0 and cold["status"] == 0
    assert warm["iters"] < cold["iters"]
    assert abs(warm["fit_true"] - cold["fit_true"]) < 1e-4
    d.release(ws)
    d.release(wsn)
