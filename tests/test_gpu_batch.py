"""Batched decomposition through the C ABI: every tensor of a batch must come
out bit for bit as dpar2_decompose leaves it when run alone (the kernels
partition work per tensor, so no sum crosses tensors and every partial sum
has the same blocking), including tensors that stop early by their own
tolerance; one tensor is also checked against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import canonical, rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(Xs, R, L, iters, tols, graph=True):
    """Decomposes Xs one by one and as one batch; asserts the batch result of
    every tensor equals its single run bit for bit.  R, L: one value for all
    tensors or one per tensor."""
    torch = _torch()
    import paper_2203_12798_amd as d
    n = len(Xs)
    Rs = R if isinstance(R, (list, tuple)) else [R] * n
    Ls = L if isinstance(L, (list, tuple)) else [L] * n
    print(f"[gpu] batch of {n}: K={[X.K for X in Xs]} J={[X.J for X in Xs]} R={Rs} L={Ls} iters={iters} "
          f"graph={graph}", flush=True)
    Ts = [d.Tensor.from_numpy(X.slab, X.offsets) for X in Xs]
    os_ = [d.Options(rank=r, sketch=l, sketch2=l, max_iter=iters, tol=t, graph=graph)
           for r, l, t in zip(Rs, Ls, tols)]
    oms = [synth.omegas(X.J, l, X.K * r, seed=11 + i) for i, (X, r, l) in enumerate(zip(Xs, Rs, Ls))]
    inits = [synth.init_factors(X.J, X.K, r, seed=21 + i) for i, (X, r) in enumerate(zip(Xs, Rs))]
    om1 = [torch.from_numpy(a).cuda() for a, _ in oms]
    om2 = [torch.from_numpy(b).cuda() for _, b in oms]
    # each tensor alone
    single = []
    for T, o, a, b, (H0, V0, W0) in zip(Ts, os_, om1, om2, inits):
        f = d.Factors.from_numpy(H0, V0, W0)
        ws = d.alloc_workspace(T, o)
        d.decompose(T, o, a, b, f, ws)
        single.append((f.numpy(), d.report_read(T, o, ws)))
    # all at once
    fs = [d.Factors.from_numpy(*ini) for ini in inits]
    wsb = d.alloc_batch_workspace(Ts, os_)
    d.decompose_batch(Ts, os_, om1, om2, fs, wsb)
    reps = d.batch_report_read(Ts, os_, wsb)
    for i, (f, ((H, V, W), rep)) in enumerate(zip(fs, single)):
        Hb, Vb, Wb = f.numpy()
        assert np.array_equal(Hb, H) and np.array_equal(Vb, V) and np.array_equal(Wb, W), i
        for key in ("iters", "converged", "err_last", "fit_true", "xnorm2", "warn_bits"):
            assert reps[i][key] == rep[key], (i, key, reps[i][key], rep[key])
    return fs, reps, oms, inits


def test_batch_equals_single_runs():
    """Three small-parity tensors of 64, 37 and 130 slices (I_k in
    [50, 200], [15, 40] and [15, 300]), R=5, L=15, 40 iterations; the second
    stops early by tol=1.5e-2 (its error decreases slowly)."""
    Xs = [synth.small_parity(seed=1, K=64),
          synth.small_parity(seed=3, K=37, imin=15, imax=40),
          synth.small_parity(seed=5, K=130, imin=15, imax=300)]
    R, L, iters = 5, 15, 40
    fs, reps, oms, inits = _case(Xs, R, L, iters, [-1.0, 1.5e-2, -1.0])
    assert reps[0]["iters"] == iters and reps[2]["iters"] == iters
    assert reps[1]["converged"] and reps[1]["iters"] < iters
    # the first tensor against the oracle (model tensor, within 1e-5)
    X = Xs[0]
    ref = O.dpar2(X.slab, X.offsets, R, oms[0][0], oms[0][1], *inits[0], iters)
    H, V, W = fs[0].numpy()
    Hg, Vg, Wg = canonical(H, V, W)
    Hr, Vr, Wr = canonical(ref.state.H, ref.state.V, ref.state.W)
    assert rel(Vg, Vr) < 1e-5 and rel(Wg, Wr) < 1e-5
    assert abs(reps[0]["fit_true"] - ref.fit) < 1e-7


def test_batch_of_tiny_and_stock_shaped_tensors():
    """Mixed sizes at the stock shape (J=88, R=10, L=20): K = 2, 3, 300 (one
    slice longer than a work item of the slab pass, 20000 rows), 8
    iterations."""
    rows = synth.stock_like_rows(300, 4)
    rows[7] = 20000
    Xs = [synth.parafac2(np.array([120, 60]), 88, 10, 31, noise_rel=0.05),
          synth.parafac2(np.array([300, 25, 900]), 88, 10, 32, noise_rel=0.05),
          synth.parafac2(rows, 88, 10, 33, noise_rel=0.05, col_scale_decades=(-2.0, 3.0))]
    _case(Xs, 10, 20, 8, [-1.0, -1.0, -1.0])


def test_heterogeneous_batch_is_grouped():
    """Tensors of different J and R in one call (J in {32, 64}, R in {5, 10},
    L = R + 10, interleaved so that groups are not contiguous in the batch),
    20 iterations; each equals its single run."""
    spec = [(32, 5, 40, 1), (64, 10, 25, 2), (32, 5, 17, 3), (64, 5, 60, 4), (64, 10, 33, 5)]
    Xs = [synth.parafac2(synth.uniform_rows(K, 32, 400, seed), J, R, seed, noise_rel=0.05)
          for J, R, K, seed in spec]
    Rs = [R for _, R, _, _ in spec]
    _case(Xs, Rs, [R + 10 for R in Rs], 20, [-1.0, 1e-5, -1.0, -1.0, 1e-5])


def test_graph_replays_match_eager():
    """The iterations replayed from a captured HIP graph equal the eager
    launches bit for bit, on every replay, with eager work (another
    decomposition, torch ops) and synchronisations between the replays; also
    for als_step called in pieces of different step counts."""
    torch = _torch()
    import paper_2203_12798_amd as d
    X = synth.small_parity(seed=9, K=50)
    X2 = synth.small_parity(seed=10, K=30)
    R, L, iters = 5, 15, 30
    print(f"[gpu] graph replays: K={X.K} R={R} iters={iters}", flush=True)
    T, T2 = d.Tensor.from_numpy(X.slab, X.offsets), d.Tensor.from_numpy(X2.slab, X2.offsets)
    om1, om2 = (torch.from_numpy(a).cuda() for a in synth.omegas(X.J, L, X.K * R))
    p1, p2 = (torch.from_numpy(a).cuda() for a in synth.omegas(X2.J, L, X2.K * R, seed=3))
    ini = synth.init_factors(X.J, X.K, R)
    ini2 = synth.init_factors(X2.J, X2.K, R)

    def run(graph, ws=None, pieces=None):
        o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, graph=graph)
        ws = d.alloc_workspace(T, o) if ws is None else ws
        f = d.Factors.from_numpy(*ini)
        if pieces is None:
            d.decompose(T, o, om1, om2, f, ws)
        else:
            d.compress(T, o, om1, om2, ws)
            et = torch.zeros(iters, dtype=torch.float64, device="cuda")
            done = 0
            for n in pieces:
                d.als_step(T, o, f, n, ws, err_trace=et[done:])
                done += n
            d.fitness(T, o, f, ws)
        rep = d.report_read(T, o, ws)
        return f.numpy(), rep, ws

    (H, V, W), rep, _ = run(False)
    ws = None
    for replay in range(3):
        (Hg, Vg, Wg), repg, ws = run(True, ws)
        assert np.array_equal(Hg, H) and np.array_equal(Vg, V) and np.array_equal(Wg, W), replay
        assert repg == rep, replay
        # eager work in between: another decomposition and plain torch ops
        o2 = d.Options(rank=R, sketch=L, sketch2=L, max_iter=7, graph=False)
        f2 = d.Factors.from_numpy(*ini2)
        d.decompose(T2, o2, p1, p2, f2, d.alloc_workspace(T2, o2))
        _ = (torch.randn(1000, device="cuda") * 2).sum().item()
        torch.cuda.synchronize()
    for pieces in ((10, 20), (10, 10, 10)):
        (He, Ve, We), repe, _ = run(False, pieces=pieces)
        (Hg, Vg, Wg), repg, _ = run(True, pieces=pieces)
        assert np.array_equal(He, Hg) and np.array_equal(Ve, Vg) and np.array_equal(We, Wg), pieces
        assert repe == repg
        assert repe["iters"] == iters


@pytest.mark.parametrize("shape", ["J600_three", "J4096_R32_pair", "J600_R40_pair"])
def test_long_j_batch_equals_single_runs(shape):
    """Batches at long J (the second stage's J-long steps on one wave per 64
    rows, the wide Y2 partials summed one thread per entry, per tensor):
    three tensors at J = 600 (R = 5, L = 15), two rank-32 tensors at
    J = 4096 whose K R together would call for longer row chunks of the
    second-stage sketch than each alone (the chunk length is the tensor's
    own), and two rank-40 tensors at J = 600 (L = 50: one slice per block
    in the iteration, the block table across both tensors); bit for bit the
    single runs."""
    if shape == "J600_three":
        Xs = [synth.parafac2(synth.uniform_rows(K, 40, 120, 60 + i), 600, 5, 60 + i, noise_abs=0.02)
              for i, K in enumerate([30, 45, 20])]
        _case(Xs, 5, 15, 12, [-1.0] * 3)
    elif shape == "J600_R40_pair":
        Xs = [synth.parafac2(synth.uniform_rows(K, 60, 160, 80 + i), 600, 40, 80 + i, noise_abs=0.02)
              for i, K in enumerate([24, 17])]
        _case(Xs, 40, 50, 6, [-1.0] * 2)
    else:
        Xs = [synth.parafac2(synth.uniform_rows(140, 33, 40, 70 + i), 4096, 32, 70 + i, noise_abs=0.02)
              for i in range(2)]
        _case(Xs, 32, 32, 4, [-1.0] * 2)
