"""PARAFAC2-ALS on the uncompressed slices (Alg. 2) on the GPU, through the C
ABI, against the FP64 oracle's als_plain on the same seeded inputs and
starting factors: the error of every iteration, the stop iteration, the
factors (up to the PARAFAC2 gauges), U_k = Q_k H and the fitness.

Precision: each iteration forms X_k V on the slab pass (float32-level, V
rounded to float32) and the exact Gram and projection of its 22-bit
fixed-point tile representation, then FP64.  The bounds come from a CPU
emulation of exactly that arithmetic against the oracle
(tests/golden/derive_parity_bounds.py, plain cases; 4 x the emulated
deviation, never below 1e-6 relative / 1e-8 in fitness)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dpar2_oracle as O
from tests._helpers import canonical, model_tensor, rel
from tests.golden.derive_parity_bounds import PLAIN_CASES

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(X, R, iters, tol=-1.0, T=None, wide_slab=False):
    torch = _torch()
    import paper_2203_12798_amd as d
    print(f"[gpu] plain ALS K={X.K} J={X.J} N={X.N} R={R} iters={iters} tol={tol}", flush=True)
    if T is None:
        T = d.Tensor.from_numpy(X.slab, X.offsets)
    o = d.Options(rank=R, sketch=R, sketch2=R, max_iter=iters, tol=tol, wide_slab=wide_slab)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    f = d.Factors.from_numpy(H0, V0, W0)
    ws = d.alloc_plain_workspace(T, o)
    et = torch.zeros(max(iters, 1), dtype=torch.float64, device="cuda")
    U = torch.zeros((X.N, R), dtype=torch.float64, device="cuda")
    rep = d.als_plain(T, o, f, ws, err_trace=et, U=U, report=True)
    H, V, W = f.numpy()
    return dict(H=H, V=V, W=W, rep=rep, err=et.cpu().numpy()[:rep["iters"]], U=U.cpu().numpy()), (H0, V0, W0)


BOUNDS = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                     "parity_bounds.json")))["bounds"]


@pytest.mark.parametrize("case", sorted(PLAIN_CASES))
def test_plain_als_matches_oracle(case):
    """The small parity tensor (30 iterations); 60 US-Stock-shaped slices
    (J = 88, feature scales over five decades, R = 10) stopping by
    tol = 1e-2; 12 ragged slices of 7..260 rows at J = 300 (the
    128-column-chunk pass) and J = 40 (that pass forced)."""
    make, R, iters, tol = PLAIN_CASES[case]
    X = make()
    b = BOUNDS[case]
    g, (H0, V0, W0) = _run(X, R, iters, tol=tol, wide_slab=(case == "plain_ragged_J40"))
    ref = O.als_plain(X.slab, X.offsets, R, H0, V0, W0, iters, tol=tol)
    e_ref = np.asarray(ref.errors)
    assert g["rep"]["iters"] == len(e_ref)
    if tol >= 0.0:
        assert len(e_ref) < iters and g["rep"]["converged"] and g["rep"]["status"] == 0
    assert np.max(np.abs(g["err"] - e_ref) / e_ref) < b["errors"]
    mg, mr = model_tensor(g["H"], g["V"], g["W"]), model_tensor(ref.H, ref.V, ref.W)
    assert rel(mg, mr) < b["model"], rel(mg, mr)
    Hg, Vg, Wg = canonical(g["H"], g["V"], g["W"])
    Hr, Vr, Wr = canonical(ref.H, ref.V, ref.W)
    assert rel(Vg, Vr) < b["V"] and rel(Wg, Wr) < b["W"]
    assert rel(Hg.T @ Hg, Hr.T @ Hr) < b["HtH"]
    assert rel(g["U"], np.concatenate(ref.U, axis=0)) < b["U"]
    assert abs(g["rep"]["fit_true"] - ref.fit) < b["fit"], (g["rep"]["fit_true"], ref.fit)
    assert g["rep"]["warn_bits"] == 0
