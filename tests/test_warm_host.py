"""Host logic of the warm-start training (no GPU): the assignment that
orders each target's components like the prediction's before the loss
(WarmNet._match), on CPU tensors.  A prediction that is the target with its
components permuted (plus noise far below the gaps between components) must
get back exactly that permutation of H^T H (rows and columns), of the
columns of V~ and of the columns of every token's W row."""
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_match_recovers_a_permutation_of_the_components():
    from paper_2203_12798_amd.warm import WarmNet
    R, Ks = 4, [5, 7, 3]
    rng = np.random.default_rng(3)
    n = len(Ks)
    off = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int32)
    A = rng.standard_normal((n, R, R))
    tH = torch.from_numpy(np.einsum("bij,bkj->bik", A, A)).float()
    tV = torch.from_numpy(rng.standard_normal((n, R, R))).float()
    tW = torch.from_numpy(rng.standard_normal((int(off[-1]), R))).float()
    perms = [rng.permutation(R) for _ in range(n)]
    pV = torch.stack([tV[i][:, perms[i]] for i in range(n)]) + 1e-4 * torch.randn(n, R, R)
    pW = torch.cat([tW[off[i]:off[i + 1]][:, perms[i]] for i in range(n)]) + 1e-4 * torch.randn(int(off[-1]), R)
    pH = torch.zeros(n, R, R)
    tH2, tV2, tW2 = WarmNet._match(types.SimpleNamespace(R=R), off, pV, pW, tH, tV, tW)
    for i in range(n):
        p = perms[i]
        assert torch.equal(tV2[i], tV[i][:, p])
        assert torch.equal(tH2[i], tH[i][p][:, p])
        assert torch.equal(tW2[off[i]:off[i + 1]], tW[off[i]:off[i + 1]][:, p])
    # the identity order is kept when the prediction already matches
    tH3, tV3, tW3 = WarmNet._match(types.SimpleNamespace(R=R), off, tV.clone(), tW.clone(), tH, tV, tW)
    assert torch.equal(tV3, tV) and torch.equal(tH3, tH) and torch.equal(tW3, tW)
    assert pH.shape == tH2.shape
