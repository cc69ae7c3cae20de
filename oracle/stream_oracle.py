"""FP64 CPU oracle of DPar2 on a tensor that grows by appended slices (the
streaming setting that Sec. VI names as future work).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path never calls it and
shares no code with it.

The paper defines no streaming algorithm; this follows the structure of
Sec. III-B.  Reading (listed with the others in the design notes):

  * the first stage factors each slice by itself (Eq. 4: the randomized SVD of
    X_k reads X_k and the shared Omega_1 only), so an append runs the first
    stage on the new slices alone and keeps A_k, B_k, C_k and ||X_k||^2 of
    the earlier slices as they were;
  * M = ||_k C_k B_k grows by the new slices' columns, and the second stage
    (Eq. 5) runs again on the whole M with an Omega_2 of (K R) x L2 rows for
    the K slices after the append (rows kR..kR+R-1 belong to slice k);
  * the iteration of Alg. 3 then starts from factors that the caller supplies
    (for instance the previous H and V, and W with a row per new slice).

  append_compress   first stage of the new slices, second stage of all
  dpar2_append      append_compress, the iteration, U_k and the fitness
"""
from __future__ import annotations

import numpy as np

from oracle import dpar2_oracle as O


def append_compress(prev: O.Compressed, slab_new, offsets_new, R: int, omega1, omega2,
                    q: int = 0) -> O.Compressed:
    """Compressed data after appending the slices of (slab_new, offsets_new)
    to those of `prev`: the first stage on the new slices only, the second
    stage over the concatenated M with omega2 ((K_prev + K_new) R x L2)."""
    A, Bd, C, xn = O.first_stage(slab_new, offsets_new, R, omega1, q)
    return O.second_stage(prev.A + A, np.concatenate([prev.Bdiag, Bd]), prev.C + C,
                          np.concatenate([prev.xnorm2, xn]), omega2)


def dpar2_append(prev: O.Compressed, slab, offsets, k_prev: int, R: int, omega1, omega2, H0, V0, W0,
                 max_iter: int, tol: float = -1.0, q: int = 0) -> O.Result:
    """DPar2 after an append: `prev` holds the compressed data of slices
    0..k_prev-1 of (slab, offsets); slices k_prev.. are the new ones.  The
    iteration starts from (H0, V0, W0) (W0 with a row for every slice); U_k
    and the fitness cover every slice."""
    off = np.asarray(offsets, dtype=np.int64)
    base = int(off[k_prev])
    c = append_compress(prev, slab[base:], off[k_prev:] - base, R, omega1, omega2, q)
    st = O.als_compressed(c, H0, V0, W0, max_iter, tol)
    U = O.output_U(c, st)
    return O.Result(comp=c, state=st, U=U, fit=O.fitness(slab, off, U, st.W, st.V))
