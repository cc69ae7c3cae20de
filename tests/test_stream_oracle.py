"""Pins for the streaming oracle (oracle/stream_oracle.py): appending slices
must give exactly what DPar2 gives on the grown tensor in one go, because the
first stage of Sec. III-B factors each slice by itself (Eq. 4) and the
second stage (Eq. 5) is run again over the whole M.  The reference is the
pinned batch oracle (tests/test_oracle_pins.py) on the concatenated tensor;
three broken appends kept here as fixtures (second stage over the new slices
only, Omega_2 rows of the new slices put first, second stage not run again)
must each fail the same comparison.  CPU only."""
import numpy as np

import synth
from oracle import dpar2_oracle as O
from oracle import stream_oracle as S


def _tensor(K=14, J=11, R=3, seed=5):
    rows = synth.uniform_rows(K, 12, 30, seed)
    return synth.parafac2(rows, J, R, seed, noise_abs=0.05)


def _same(a: O.Compressed, b: O.Compressed):
    return (len(a.A) == len(b.A) and all(np.array_equal(x, y) for x, y in zip(a.A, b.A))
            and all(np.array_equal(x, y) for x, y in zip(a.C, b.C))
            and np.array_equal(a.Bdiag, b.Bdiag) and np.array_equal(a.M, b.M)
            and np.array_equal(a.xnorm2, b.xnorm2) and np.array_equal(a.D, b.D)
            and np.array_equal(a.E, b.E) and np.array_equal(a.F, b.F))


def _split(X, k):
    off = np.asarray(X.offsets, dtype=np.int64)
    return X.slab[:off[k]], off[:k + 1], X.slab[off[k]:], off[k:] - off[k]


# broken appends (fixtures): each makes one plausible mistake
def _stage2_new_only(prev, slab_new, off_new, R, om1, om2, q=0):
    A, Bd, C, xn = O.first_stage(slab_new, off_new, R, om1, q)
    c = O.second_stage(A, Bd, C, xn, om2[-len(A) * R:])
    return O.Compressed(A=prev.A + c.A, Bdiag=np.concatenate([prev.Bdiag, Bd]), C=prev.C + c.C,
                        M=np.concatenate([prev.M, c.M], axis=1), D=c.D, E=c.E,
                        F=np.concatenate([prev.F, c.F]), xnorm2=np.concatenate([prev.xnorm2, xn]))


def _omega2_new_first(prev, slab_new, off_new, R, om1, om2, q=0):
    kn = len(off_new) - 1
    rolled = np.concatenate([om2[-kn * R:], om2[:-kn * R]])
    return S.append_compress(prev, slab_new, off_new, R, om1, rolled, q)


def _no_second_stage(prev, slab_new, off_new, R, om1, om2, q=0):
    A, Bd, C, xn = O.first_stage(slab_new, off_new, R, om1, q)
    M = np.concatenate([prev.M] + [C[k] * Bd[k][None, :] for k in range(len(A))], axis=1)
    F = np.concatenate([prev.F, np.zeros((len(A) * R, R))])
    return O.Compressed(A=prev.A + A, Bdiag=np.concatenate([prev.Bdiag, Bd]), C=prev.C + C, M=M,
                        D=prev.D, E=prev.E, F=F, xnorm2=np.concatenate([prev.xnorm2, xn]))


def test_append_equals_compressing_the_grown_tensor():
    """10 + 4 slices, q = 0 and q = 1: every field of the compressed data
    (A_k, B_k, C_k, M, ||X_k||^2, D, E, F) equals the batch oracle's on all
    14 slices exactly; each broken append differs."""
    X = _tensor()
    R, L = 3, 6
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    for q in (0, 1):
        full = O.compress(X.slab, X.offsets, R, om1, om2, q=q)
        s0, o0, s1, o1 = _split(X, 10)
        prev = O.compress(s0, o0, R, om1, om2[:10 * R], q=q)
        assert _same(S.append_compress(prev, s1, o1, R, om1, om2, q), full)
        for broken in (_stage2_new_only, _omega2_new_first, _no_second_stage):
            assert not _same(broken(prev, s1, o1, R, om1, om2, q), full), broken.__name__


def test_three_appends_equal_one_compress():
    """5 + 4 + 1 + 4 slices (one append of a single slice): the result of
    the last append equals the batch oracle on the 14 slices."""
    X = _tensor(seed=8)
    R, L = 3, 5
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    off = np.asarray(X.offsets, dtype=np.int64)
    c = O.compress(X.slab[:off[5]], off[:6], R, om1, om2[:5 * R])
    for a, b in ((5, 9), (9, 10), (10, 14)):
        c = S.append_compress(c, X.slab[off[a]:off[b]], off[a:b + 1] - off[a], R, om1, om2[:b * R])
    assert _same(c, O.compress(X.slab, X.offsets, R, om1, om2))


def test_dpar2_append_equals_dpar2_on_the_grown_tensor():
    """The iteration, U_k and the fitness after an append: identical to
    DPar2 on the grown tensor from the same initial factors; the earlier
    columns of M are the previous ones, unchanged."""
    X = _tensor(seed=9)
    R, L, iters = 3, 6, 12
    om1, om2 = synth.omegas(X.J, L, X.K * R)
    H0, V0, W0 = synth.init_factors(X.J, X.K, R)
    s0, o0, _, _ = _split(X, 9)
    prev = O.compress(s0, o0, R, om1, om2[:9 * R])
    got = S.dpar2_append(prev, X.slab, X.offsets, 9, R, om1, om2, H0, V0, W0, iters)
    ref = O.dpar2(X.slab, X.offsets, R, om1, om2, H0, V0, W0, iters)
    assert np.array_equal(got.comp.M[:, :9 * R], prev.M)
    assert np.array_equal(got.state.H, ref.state.H) and np.array_equal(got.state.V, ref.state.V)
    assert np.array_equal(got.state.W, ref.state.W)
    assert all(np.array_equal(a, b) for a, b in zip(got.U, ref.U))
    assert got.fit == ref.fit and got.state.errors == ref.state.errors
