"""Status codes, report and resumable mode of the C ABI, on the GPU: a NaN or
Inf in the slab returns DPAR2_ENUMERIC (single calls and batches, where the
other tensors still come out as when run alone); a tolerance the iteration
does not reach returns DPAR2_ENOCONV with a valid result; the resumable flag
gives 16 + 16 iterations equal to 32 bit for bit; A_k of Eq. 4 matches the
oracle; a released or reused workspace still gives the fresh results."""
import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import rel

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(X, R, L, iters, tol=-1.0, **kw):
    torch = _torch()
    import paper_2203_12798_amd as d
    T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters, tol=tol, **kw)
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    init = synth.init_factors(X.J, X.K, R)
    return d, T, o, torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda(), init


@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_nonfinite_slab_returns_enumeric(bad):
    """One entry of slice 3 set to NaN (or -Inf): the report of the tensor says
    DPAR2_WARN_NONFINITE and the iteration did not run; decompose with a
    report and report_read both return DPAR2_ENUMERIC."""
    X = synth.small_parity(seed=1)
    slab = X.slab.copy()
    slab[X.offsets[3] + 2, 5] = np.float32("nan") if bad == "nan" else np.float32("-inf")
    Xb = synth.IrregularTensor(slab=slab, offsets=X.offsets)
    print(f"[gpu] non-finite slab ({bad})", flush=True)
    d, T, o, o1, o2, (H0, V0, W0) = _setup(Xb, 5, 15, 20)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_workspace(T, o)
    with pytest.raises(d.Dpar2Error) as ei:
        d.decompose(T, o, o1, o2, f, ws, report=True)
    assert ei.value.status == -3
    r = ei.value.report
    assert r["warn_bits"] & 0x4 and r["iters"] == 0 and not r["converged"]
    assert not np.isfinite(r["xnorm2"])
    with pytest.raises(d.Dpar2Error) as ei:
        d.report_read(T, o, ws)
    assert ei.value.status == -3
    # the factors were left as given (no iteration ran); V is written back only
    # after a V update
    H, V, W = f.numpy()
    assert np.array_equal(H, H0) and np.array_equal(W, W0) and np.array_equal(V, V0)


def test_nonfinite_tensor_in_batch_leaves_the_others_intact():
    """A batch of a clean tensor, a tensor with a NaN and another clean one (one
    group): the batch report returns DPAR2_ENUMERIC with every report filled;
    the clean tensors equal their single runs bit for bit."""
    torch = _torch()
    import paper_2203_12798_amd as d
    Xs = [synth.small_parity(seed=s, K=k) for s, k in ((1, 40), (2, 33), (3, 50))]
    slab = Xs[1].slab.copy()
    slab[Xs[1].offsets[7], 0] = np.float32("nan")
    Xs[1] = synth.IrregularTensor(slab=slab, offsets=Xs[1].offsets)
    R, L, iters = 5, 15, 25
    print("[gpu] batch with a NaN tensor", flush=True)
    Ts = [d.Tensor.from_numpy(X.slab, X.offsets) for X in Xs]
    os_ = [d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters) for _ in Xs]
    oms = [synth.omegas(X.J, L, X.K * R, seed=11 + i) for i, X in enumerate(Xs)]
    inits = [synth.init_factors(X.J, X.K, R, seed=21 + i) for i, X in enumerate(Xs)]
    om1 = [torch.from_numpy(a).cuda() for a, _ in oms]
    om2 = [torch.from_numpy(b).cuda() for _, b in oms]
    fs = [d.Factors.from_numpy(*ini) for ini in inits]
    wsb = d.alloc_batch_workspace(Ts, os_)
    d.decompose_batch(Ts, os_, om1, om2, fs, wsb)
    with pytest.raises(d.Dpar2Error) as ei:
        d.batch_report_read(Ts, os_, wsb)
    assert ei.value.status == -3 and b"tensor 1" in str(ei.value).encode()
    reps = ei.value.report
    assert reps[1]["warn_bits"] & 0x4 and reps[1]["iters"] == 0
    for i in (0, 2):
        assert reps[i]["warn_bits"] == 0 and reps[i]["iters"] == iters
        f1 = d.Factors.from_numpy(*inits[i])
        ws = d.alloc_workspace(Ts[i], os_[i])
        d.decompose(Ts[i], os_[i], om1[i], om2[i], f1, ws)
        for a, b in zip(f1.numpy(), fs[i].numpy()):
            assert np.array_equal(a, b), i


def test_tolerance_not_reached_returns_enoconv():
    """tol = 1e-12 within 6 iterations: DPAR2_ENOCONV, the report filled and
    the result equal to the same run without a report; tol = 5e-3 within 200
    iterations stops early and returns DPAR2_OK."""
    X = synth.small_parity(seed=5)
    d, T, o, o1, o2, (H0, V0, W0) = _setup(X, 5, 15, 6, tol=1e-12)
    print("[gpu] ENOCONV", flush=True)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_workspace(T, o)
    r = d.decompose(T, o, o1, o2, f, ws, report=True)
    assert r["status"] == -4 and r["iters"] == 6 and not r["converged"]
    f2 = d.Factors.from_numpy(H0, V0, W0)
    ws2 = d.alloc_workspace(T, o)
    d.decompose(T, o, o1, o2, f2, ws2)
    for a, b in zip(f.numpy(), f2.numpy()):
        assert np.array_equal(a, b)
    d, T, o, o1, o2, _ = _setup(X, 5, 15, 200, tol=5e-3)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_workspace(T, o)
    r = d.decompose(T, o, o1, o2, f, ws, report=True)
    assert r["status"] == 0 and r["converged"] and r["iters"] < 200


@pytest.mark.parametrize("graph", [True, False])
def test_resumable_mode_is_bitwise(graph):
    """DPAR2_FLAG_DETERMINISTIC: 32 iterations in one call, 16 + 16, and
    8 + 8 + 16 give the same bits (factors, error trace, last error); the
    result is the method's (within 1e-9 of the default mode's model)."""
    torch = _torch()
    X = synth.small_parity(seed=6)
    d, T, o, o1, o2, (H0, V0, W0) = _setup(X, 5, 15, 32, deterministic=True, graph=graph)
    print(f"[gpu] resumable mode graph={graph}", flush=True)
    outs = []
    for split in ([32], [16, 16], [8, 8, 16]):
        f = d.Factors.from_numpy(H0, V0, W0)
        ws = d.alloc_workspace(T, o)
        d.compress(T, o, o1, o2, ws)
        trace = []
        for n in split:
            et = torch.zeros(n, dtype=torch.float64, device="cuda")
            d.als_step(T, o, f, n, ws, err_trace=et)
            trace.append(et.cpu().numpy())
        rep = d.report_read(T, o, ws)
        outs.append((f.numpy(), np.concatenate(trace), rep["err_last"], rep["iters"]))
    (Ha, Va, Wa), ta, ea, ia = outs[0]
    assert ia == 32
    for (Hb, Vb, Wb), tb, eb, ib in outs[1:]:
        assert ib == 32 and eb == ea
        assert np.array_equal(tb, ta)
        assert np.array_equal(Ha, Hb) and np.array_equal(Va, Vb) and np.array_equal(Wa, Wb)
    # the default mode: same method, other rounding
    d2, T2, o2_, p1, p2, _ = _setup(X, 5, 15, 32, graph=graph)
    f = d2.Factors.from_numpy(H0, V0, W0)
    ws = d2.alloc_workspace(T2, o2_)
    d2.decompose(T2, o2_, p1, p2, f, ws)
    from tests._helpers import model_tensor
    assert rel(model_tensor(*f.numpy()), model_tensor(Ha, Va, Wa)) < 1e-9


def test_output_A_matches_oracle():
    """A_k of Eq. 4 (first-stage left factor, I_k x R) against the oracle's,
    per slice within 1e-5 relative, and column-orthonormal to 5e-6: the pass
    recomputes the float32 sketch Y_k tile by tile and multiplies it by Phi_k,
    which whitens the 22-bit fixed-point Y_k of the Gram; the two differ by up
    to 2^-22 of a tile column's maximum, which leaves A_k^T A_k - I at a few
    1e-6 (the emulation in tests/golden/derive_parity_bounds.py puts the
    output's relative error at 6.6e-7 on the small parity tensor)."""
    torch = _torch()
    X = synth.small_parity(seed=3, K=48)
    R, L = 5, 15
    d, T, o, o1, o2, _ = _setup(X, R, L, 0)
    print("[gpu] output_A", flush=True)
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    c = O.compress(X.slab, X.offsets, R, om1, om2)
    ws = d.alloc_workspace(T, o)
    d.compress(T, o, o1, o2, ws)
    A = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    d.output_A(T, o, A, ws)
    Ag = A.cpu().numpy()
    for k in range(X.K):
        a = Ag[X.offsets[k]:X.offsets[k + 1]]
        assert rel(a, c.A[k]) < 1e-5, (k, rel(a, c.A[k]))
        assert np.abs(a.T @ a - np.eye(R)).max() < 5e-6


def test_released_and_reused_workspace():
    """One workspace buffer used for a tensor (iterations captured into a
    graph), released, then used for a tensor of another shape (different
    layout offsets) and for the first again: every result equals a run on a
    fresh workspace bit for bit."""
    torch = _torch()
    import paper_2203_12798_amd as d
    Xa = synth.small_parity(seed=1, K=64)
    Xb = synth.small_parity(seed=2, K=41, imin=20, imax=90)
    R, L, iters = 5, 15, 12
    print("[gpu] workspace reuse", flush=True)

    def run(X, ws=None):
        T = d.Tensor.from_numpy(X.slab, X.offsets)
        o = d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters)
        om1, om2 = synth.omegas(X.J, L, X.K * R)
        f = d.Factors.from_numpy(*synth.init_factors(X.J, X.K, R))
        if ws is None:
            ws = d.alloc_workspace(T, o)
        d.decompose(T, o, torch.from_numpy(om1).cuda(), torch.from_numpy(om2).cuda(), f, ws)
        return f.numpy(), d.report_read(T, o, ws)["err_last"]

    fresh_a, fresh_b = run(Xa), run(Xb)
    n = max(d.workspace_size(d.Tensor.from_numpy(X.slab, X.offsets),
                             d.Options(rank=R, sketch=L, sketch2=L, max_iter=iters)) for X in (Xa, Xb))
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    seq = [(Xa, fresh_a), (Xb, fresh_b), (Xa, fresh_a)]
    for i, (X, (fr, er)) in enumerate(seq):
        got, eg = run(X, ws)
        assert eg == er, i
        for a, b in zip(got, fr):
            assert np.array_equal(a, b), i
        if i == 0:
            torch.cuda.synchronize()
            d.release(ws)
    d.release(ws)


@pytest.mark.parametrize("R,L", [(5, 15), (10, 15), (20, 24), (40, 40), (50, 50)])
def test_rank_deficient_q_step_keeps_psi_orthogonal(R, L):
    """A starting W with a zero column makes every T_k of the first Q-step
    (Eq. 8) singular: the polar factor is then not unique, and the Q-step
    completes Z_k so that Psi_k = Z_k P_k^T stays orthogonal.  Checked through
    U_k = A_k Psi_k H: U_k^T U_k = H^T H for every slice (A_k has orthonormal
    columns), with the rank-deficiency warning raised and finite factors;
    R = 5, 10 and 20 (groups of 8, 16 and 32 lanes per slice, one lane per
    column), and R = 40, 50 (one slice per 64-lane block, J = 64)."""
    torch = _torch()
    X = synth.small_parity(seed=2, K=40) if R <= 32 else synth.small_parity(seed=2, K=40, J=64)
    d, T, o, o1, o2, (H0, V0, W0) = _setup(X, R, L, 1)
    W0 = W0.copy()
    W0[:, 2] = 0.0
    print(f"[gpu] rank-deficient Q-step R={R}", flush=True)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_workspace(T, o)
    d.compress(T, o, o1, o2, ws)
    d.als_step(T, o, f, 1, ws)
    U = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    d.output_U(T, o, f, U, ws)
    rep = d.report_read(T, o, ws)
    assert rep["warn_bits"] & 0x2
    H, V, W = f.numpy()
    assert np.all(np.isfinite(H)) and np.all(np.isfinite(V)) and np.all(np.isfinite(W))
    Ug = U.cpu().numpy()
    HtH = H.T @ H
    for k in range(X.K):
        u = Ug[X.offsets[k]:X.offsets[k + 1]]
        assert np.abs(u.T @ u - HtH).max() < 1e-5 * np.abs(HtH).max(), k
