"""The tiling of the slab pass and its autotuners, through the C ABI: results
with small items (long slices cut into many pieces) and with the
128-column-chunk pass below the whole-row limit match the FP64 oracle, and the
autotuners time every candidate and return the fastest."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests.test_gpu_parity import _check_compression, _check_errors, _check_factors, _run_gpu, _torch

pytestmark = pytest.mark.gpu


def _long_case():
    rows = np.array([3000, 70, 4100, 900, 2500, 64])
    return synth.parafac2(rows, 24, 4, 61, noise_abs=0.02)


@pytest.mark.parametrize("item_rows", [64, 640])
def test_small_items_match_oracle(item_rows):
    """Slices of 64..4100 rows cut into items of at most 64 or 640 rows
    (up to 65 items per slice, summed per slice in the completion)."""
    torch = _torch()
    import paper_2203_12798_amd as d
    X = _long_case()
    R, L, iters = 4, 10, 25
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    print(f"[gpu] item_rows={item_rows}", flush=True)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, item_rows=item_rows)
    ws = d.alloc_workspace(T, o)
    f = d.Factors.from_numpy(H0, V0, W0)
    d.compress(T, o, torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda(), ws)
    comp = d.compressed_view(T, o, ws)
    et = torch.zeros(iters, dtype=torch.float64, device="cuda")
    d.als_step(T, o, f, iters, ws, err_trace=et)
    d.fitness(T, o, f, ws)
    rep = d.report_read(T, o, ws)
    H, V, W = f.numpy()
    g = dict(comp=comp, rep=rep, H=H, V=V, W=W, err=et.cpu().numpy()[:rep["iters"]])
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(rep["fit_true"] - ref.fit) < 1e-7


def test_autotuner_returns_fastest_candidate():
    torch = _torch()
    import paper_2203_12798_amd as d
    from paper_2203_12798_amd import binding as b
    X = _long_case()
    R, L = 4, 10
    print("[gpu] autotune", flush=True)
    om1, _ = synth.omegas(X.J, L, X.K * R)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    cands = (256, 1024, 4096, 0)
    ws = d.alloc_workspace(T, d.Options(rank=R, sketch=L, sketch2=L, max_iter=5, item_rows=256))
    best, times = b.autotune_item_rows(T, d.Options(rank=R, sketch=L, sketch2=L, max_iter=5),
                                       torch.from_numpy(om1).cuda(), ws, candidates=cands)
    print(f"[autotune] {times} -> {best}", flush=True)
    assert best in cands
    assert all(t > 0 for t in times.values())
    assert times[best] == min(times.values())


@pytest.mark.parametrize("case", ["small_parity", "stock_like"])
def test_chunked_slab_pass_below_limit_matches_oracle(case):
    """DPAR2_FLAG_WIDE_SLAB with J below the whole-row limit: J = 32, L = 15
    (one partial 128-column chunk, one 16-column L-tile) and the stock-shaped
    J = 88, L = 20 (two L-tiles), with the U output; the same bounds as the
    whole-row pass."""
    if case == "small_parity":
        X, R, L, iters = synth.small_parity(seed=9), 5, 15, 40
    else:
        X, R, L, iters = synth.stock_like(K=60, seed=4), 10, 20, 32
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    g = _run_gpu(X, R, L, L, iters, om1, om2, H0, V0, W0, want_U=True, wide_slab=True)
    _check_compression(X, R, g, ref)
    _check_errors(g, ref)
    _check_factors(g, ref)
    assert abs(g["rep"]["fit_true"] - ref.fit) < 1e-6
    assert np.linalg.norm(g["U"] - np.concatenate(ref.U, axis=0)) <= 1e-5 * np.linalg.norm(np.concatenate(ref.U))
    assert g["rep"]["warn_bits"] == 0


def test_slab_autotuner_chooses_among_passes_and_item_sizes():
    """dpar2_autotune_slab over (item_rows, chunked) pairs: every candidate is
    timed and the index of the fastest is returned."""
    torch = _torch()
    import paper_2203_12798_amd as d
    from paper_2203_12798_amd import binding as b
    X = _long_case()
    R, L = 4, 10
    print("[gpu] slab autotune", flush=True)
    om1, _ = synth.omegas(X.J, L, X.K * R)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    cands = [(256, False), (4096, False), (256, True), (0, True)]
    ws = d.alloc_workspace(T, d.Options(rank=R, sketch=L, sketch2=L, max_iter=5, item_rows=256, wide_slab=True))
    best, times = b.autotune_slab(T, d.Options(rank=R, sketch=L, sketch2=L, max_iter=5),
                                  torch.from_numpy(om1).cuda(), ws, cands)
    print(f"[autotune] {list(zip(cands, times))} -> {best}", flush=True)
    assert best in cands
    assert all(t > 0 for t in times)
    assert times[cands.index(best)] == min(times)
