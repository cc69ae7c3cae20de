"""dpar2_decompose_noalloc (the library's static device scratch instead of a
caller workspace) against dpar2_decompose on the same inputs, through the C
ABI: two calls in a row, the second on a smaller tensor, each equal to the
workspace entry point's result bit for bit (factors, U_k, report); a
decomposition too large for the scratch is rejected before anything runs."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(X, R, L, iters, tol=-1.0):
    torch = _torch()
    import paper_2203_12798_amd as d
    print(f"[gpu] noalloc K={X.K} J={X.J} N={X.N} R={R} L={L} iters={iters}", flush=True)
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, tol=tol)
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    o1, o2 = torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda()
    init = synth.init_factors(X.J, X.K, R)
    # the workspace entry point
    fw = d.Factors.from_numpy(*init)
    ws = d.alloc_workspace(T, o)
    Uw = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    rw = d.decompose(T, o, o1, o2, fw, ws, U=Uw, report=True)
    # the allocation-free one
    fn = d.Factors.from_numpy(*init)
    Un = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    rn = d.decompose_noalloc(T, o, o1, o2, fn, U=Un, report=True)
    return (fw.numpy(), Uw.cpu().numpy(), rw), (fn.numpy(), Un.cpu().numpy(), rn)


def _same(a, b):
    (fa, Ua, ra), (fb, Ub, rb) = a, b
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    assert np.array_equal(Ua, Ub)
    for key in ("iters", "converged", "err_last", "fit_true", "xnorm2", "warn_bits", "status"):
        assert ra[key] == rb[key], (key, ra[key], rb[key])


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    """64 slices (I_k in [50, 200], J = 32, R = 5, 40 iterations), then 29
    slices (I_k in [20, 90], J = 24, R = 4, 25 iterations, stopping early by
    tol): the second call reuses the scratch the first one left."""
    X1 = synth.small_parity(seed=1)
    a, b = _both(X1, 5, 15, 40)
    _same(a, b)
    assert b[2]["iters"] == 40 and b[2]["warn_bits"] == 0
    X2 = synth.small_parity(seed=9, K=29, J=24, rank=4, imin=20, imax=90)
    a, b = _both(X2, 4, 10, 25, tol=2e-2)
    _same(a, b)
    assert b[2]["iters"] <= 25


def test_noalloc_rejects_a_decomposition_beyond_the_scratch():
    """A tensor whose workspace exceeds the 64 MiB scratch: DPAR2_EWORKSPACE,
    nothing enqueued (the factors keep their values)."""
    torch = _torch()
    import paper_2203_12798_amd as d
    rows = np.full(3000, 100, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    J, R, L = 256, 10, 30
    slab = torch.zeros((int(off[-1]), J), dtype=torch.float32, device="cuda")
    T = d.Tensor(slab, torch.from_numpy(off).cuda(), off)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=3)
    from paper_2203_12798_amd import binding
    assert d.workspace_size(T, o) > binding.NOALLOC_SCRATCH_BYTES
    om1, om2 = synth.omegas(J, L, 3000 * R)
    H0, V0, W0 = synth.init_factors(J, 3000, R)
    f = d.Factors.from_numpy(H0, V0, W0)
    with pytest.raises(d.Dpar2Error) as ei:
        d.decompose_noalloc(T, o, torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda(), f)
    assert ei.value.status == -6 and "static scratch" in str(ei.value)
    H, V, W = f.numpy()
    assert np.array_equal(H, H0) and np.array_equal(V, V0) and np.array_equal(W, W0)


def test_noalloc_equals_workspace_entry_point_at_rank_40():
    """Rank 40 with L = 50 (one slice per block in the iteration, the chunked
    slab pass with four tiles of Y): 20 slices of 60..160 rows at J = 300,
    8 iterations; bit for bit the workspace entry point."""
    X = synth.parafac2(synth.uniform_rows(20, 60, 160, 40), 300, 40, 40, noise_abs=0.02)
    a, b = _both(X, 40, 50, 8)
    _same(a, b)
