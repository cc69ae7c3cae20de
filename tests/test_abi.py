"""The C ABI loads, exports every symbol the header declares, and rejects bad
arguments on the host before touching the GPU.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpar2.h")


def _lib():
    from paper_2203_12798_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libdpar2.so not built (run __graft_entry__.build())")
    return binding, binding.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpar2_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dpar2_compress", "dpar2_als_step", "dpar2_decompose", "dpar2_workspace_bytes",
              "dpar2_workspace_size", "dpar2_fitness", "dpar2_output_U", "dpar2_output_A",
              "dpar2_report_read", "dpar2_compressed_view", "dpar2_release", "dpar2_release_all"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    binding, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) == set(declared_functions())


def _tensor(binding, offsets, J=8):
    off = np.asarray(offsets, dtype=np.int64)
    t = binding.c_tensor(len(off) - 1, J, 0x1000, off.ctypes.data_as(ctypes.c_void_p).value, 0x2000, 0)
    return t, off


def _status(lib, binding, t, o, ws=0x10000, nbytes=1 << 40):
    return lib.dpar2_compress(ctypes.byref(t), ctypes.byref(o), 0x3000, 0x4000, ws, nbytes, None)


@pytest.mark.parametrize("offsets,opts,status", [
    ([0, 10, 5], (2, 3, 3, 5), -1),        # decreasing offsets
    ([1, 10, 20], (2, 3, 3, 5), -1),       # offsets[0] != 0
    ([0, 10, 12], (2, 3, 3, 5), -2),       # slice shorter than L
    ([0, 10, 20], (2, 9, 3, 5), -2),       # L > J
    ([0, 10, 20], (4, 3, 4, 5), -2),       # L < R
    ([0, 10, 20], (2, 3, 5, 5), -2),       # L2 > K R
    ([0, 10, 20], (0, 3, 3, 5), -2),       # R = 0
    ([0, 10, 20], (2, 3, 3, -1), -1),      # max_iter < 0
])
def test_invalid_arguments_are_rejected_on_host(offsets, opts, status):
    binding, lib = _lib()
    t, _keep = _tensor(binding, offsets)
    o = binding.c_opts(opts[0], opts[1], opts[2], opts[3], -1.0, 0)
    assert _status(lib, binding, t, o) == status
    assert lib.dpar2_last_error().decode()
    assert lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o)) == 0


def test_rank_and_sketch_width_sets():
    """Ranks 1..32 and, above, 40 and 50; sketch widths 1..32 and 40, 50, 60
    (every other value is a shape error before anything is enqueued)."""
    binding, lib = _lib()
    off = np.array([0, 80, 160], dtype=np.int64)
    hp = off.ctypes.data_as(ctypes.c_void_p).value
    t = binding.c_tensor(2, 600, 0x1000, hp, 0x2000, binding.DPAR2_F32, None)
    for R, L, L2, ok in [(40, 50, 50, True), (50, 60, 60, True), (40, 40, 40, True), (32, 60, 40, True),
                         (33, 40, 40, False), (48, 50, 50, False), (40, 45, 50, False), (40, 50, 64, False),
                         (64, 64, 64, False), (50, 60, 70, False)]:
        o = binding.c_opts(R, L, L2, 5, -1.0, 0)
        need = lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o))
        assert (need > 0) == ok, (R, L, L2)
        if not ok:
            assert _status(lib, binding, t, o) == -2, (R, L, L2)


def test_workspace_checks():
    binding, lib = _lib()
    t, _keep = _tensor(binding, [0, 10, 25, 40])
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0)
    need = lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o))
    assert need > 0
    assert _status(lib, binding, t, o, ws=0, nbytes=need) == -6          # NULL
    assert _status(lib, binding, t, o, ws=0x10010, nbytes=need) == -6    # misaligned
    assert _status(lib, binding, t, o, ws=0x10000, nbytes=need - 1) == -6  # too small
    assert b"too small" in lib.dpar2_last_error()


def test_null_pointers_rejected():
    binding, lib = _lib()
    off = np.array([0, 10, 20], dtype=np.int64)
    t = binding.c_tensor(2, 8, 0, off.ctypes.data_as(ctypes.c_void_p).value, 0x2000, 0)
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0)
    assert _status(lib, binding, t, o) == -1
    t2, _k = _tensor(binding, [0, 10, 20])
    assert lib.dpar2_compress(ctypes.byref(t2), ctypes.byref(o), None, 0x4000, 0x10000, 1 << 40, None) == -1


def test_status_strings():
    _, lib = _lib()
    seen = set()
    for st in (0, -1, -2, -3, -4, -5, -6):
        s = lib.dpar2_status_string(st)
        assert s and s != b"unknown status"
        seen.add(s)
    assert len(seen) == 7
    assert lib.dpar2_status_string(7) == b"unknown status"
    assert b"NaN" in lib.dpar2_status_string(-3)


def test_dtype_and_power_options_validated_on_host():
    """fp8 slabs need per-slice scales; power_iters in [0, 4]; J up to
    16384 for every dtype."""
    binding, lib = _lib()
    off = np.array([0, 10, 20], dtype=np.int64)
    hp = off.ctypes.data_as(ctypes.c_void_p).value
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0, 0)
    t = binding.c_tensor(2, 8, 0x1000, hp, 0x2000, binding.DPAR2_FP8_E4M3, None)
    assert _status(lib, binding, t, o) == -1
    assert b"scale" in lib.dpar2_last_error()
    t = binding.c_tensor(2, 8, 0x1000, hp, 0x2000, 7, None)
    assert _status(lib, binding, t, o) == -1
    for q, st in ((-1, -1), (5, -1)):
        oq = binding.c_opts(2, 3, 3, 5, -1.0, 0, q)
        t = binding.c_tensor(2, 8, 0x1000, hp, 0x2000, binding.DPAR2_F32, None)
        assert _status(lib, binding, t, oq) == st
    offw = np.array([0, 200, 400], dtype=np.int64)
    hw = offw.ctypes.data_as(ctypes.c_void_p).value
    tb = binding.c_tensor(2, 16385, 0x1000, hw, 0x2000, binding.DPAR2_BF16, None)
    assert _status(lib, binding, tb, o) == -2
    for J in (160, 2049, 16384):
        for dt in (binding.DPAR2_F32, binding.DPAR2_BF16):
            tf = binding.c_tensor(2, J, 0x1000, hw, 0x2000, dt, None)
            assert lib.dpar2_workspace_size(ctypes.byref(tf), ctypes.byref(o)) > 0
    # the wide pass (J above 256 for float32) keeps the digit planes of Y:
    # (3 * 16 * 64 + 16 * 4) bytes per 64-row tile slot at L <= 16, with
    # ceil(N / 64) + n_items slots
    t256 = binding.c_tensor(2, 256, 0x1000, hw, 0x2000, binding.DPAR2_F32, None)
    t257 = binding.c_tensor(2, 257, 0x1000, hw, 0x2000, binding.DPAR2_F32, None)
    ws256 = lib.dpar2_workspace_size(ctypes.byref(t256), ctypes.byref(o))
    ws257 = lib.dpar2_workspace_size(ctypes.byref(t257), ctypes.byref(o))
    ybuf = (3 * 16 * 64 + 16 * 4) * ((400 + 63) // 64 + 2)
    assert ws257 - ws256 >= ybuf
    # a power step needs one sketch matrix per slice in the workspace
    o1 = binding.c_opts(2, 3, 3, 5, -1.0, 0, 1)
    t8 = binding.c_tensor(2, 8, 0x1000, hp, 0x2000, binding.DPAR2_F32, None)
    assert (lib.dpar2_workspace_size(ctypes.byref(t8), ctypes.byref(o1))
            >= lib.dpar2_workspace_size(ctypes.byref(t8), ctypes.byref(o)) + 2 * 8 * 3 * 4)
    # the 128-column-chunk pass asked for below the limit keeps Y as well;
    # unknown flag bits are rejected
    ow = binding.c_opts(2, 3, 3, 5, -1.0, binding.DPAR2_FLAG_WIDE_SLAB, 0)
    assert (lib.dpar2_workspace_size(ctypes.byref(t256), ctypes.byref(ow))
            >= ws256 + ybuf)
    assert lib.dpar2_workspace_size(ctypes.byref(t257), ctypes.byref(ow)) == ws257
    ox = binding.c_opts(2, 3, 3, 5, -1.0, 0x8, 0)
    assert _status(lib, binding, t8, ox) == -1
    assert b"flags" in lib.dpar2_last_error()


def test_batch_arguments_validated_on_host():
    """A batch is split into groups of tensors sharing J, dtype, rank, sketch
    widths, power_iters, max_iter and flags; K, the row offsets and tol may
    differ inside a group.  The workspace is the groups' layouts end to end;
    an invalid tensor is rejected before anything is enqueued, and the error
    names it by its index in the batch."""
    binding, lib = _lib()
    offa = np.array([0, 10, 20], dtype=np.int64)
    offb = np.array([0, 7, 30, 33], dtype=np.int64)
    ha = offa.ctypes.data_as(ctypes.c_void_p).value
    hb = offb.ctypes.data_as(ctypes.c_void_p).value
    T = binding.c_tensor * 3
    O = binding.c_opts * 3
    ta = binding.c_tensor(2, 8, 0x1000, ha, 0x2000, binding.DPAR2_F32, None)
    tb = binding.c_tensor(3, 8, 0x3000, hb, 0x4000, binding.DPAR2_F32, None)
    tc = binding.c_tensor(3, 9, 0x3000, hb, 0x4000, binding.DPAR2_F32, None)
    oa = binding.c_opts(2, 3, 3, 5, -1.0, 0, 0)
    ob = binding.c_opts(2, 3, 3, 5, 1e-6, 0, 0)

    def size(ts, os_):
        return lib.dpar2_batch_workspace_size(len(ts), T(*ts), O(*os_))

    def single(t, o):
        return lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o))

    assert size([ta], [oa]) == single(ta, oa) > 0
    # one group (tol may differ): one layout over both tensors
    both = size([ta, tb], [oa, ob])
    assert both > single(ta, oa)
    # J differs: two groups, laid out end to end (256-byte aligned)
    al = lambda n: (n + 255) // 256 * 256
    assert size([ta, tc], [oa, oa]) == al(single(ta, oa)) + al(single(tc, oa))
    # grouping is by first appearance; members need not be adjacent
    assert size([ta, tc, tb], [oa, oa, ob]) == al(both) + al(single(tc, oa))
    for o2 in (binding.c_opts(3, 3, 3, 5, -1.0, 0, 0), binding.c_opts(2, 3, 3, 6, -1.0, 0, 0),
               binding.c_opts(2, 3, 3, 5, -1.0, binding.DPAR2_FLAG_NO_GRAPH, 0)):
        assert size([ta, tb], [oa, o2]) == al(single(ta, oa)) + al(single(tb, o2))
    assert lib.dpar2_batch_workspace_size(0, T(ta, tb, tc), O(oa, ob, oa)) == 0
    # an invalid tensor is named by its batch index
    bad = binding.c_tensor(3, 9, 0x3000, hb, 0, binding.DPAR2_F32, None)
    assert size([ta, tc, bad], [oa, oa, oa]) == 0
    assert lib.dpar2_last_error().startswith(b"tensor 2")
    assert size([ta, bad], [oa, oa]) == 0          # alone in its group
    assert lib.dpar2_last_error().startswith(b"tensor 1")
    # unknown flag bits are rejected
    assert size([ta], [binding.c_opts(2, 3, 3, 5, -1.0, 0x80, 0)]) == 0


def test_item_rows_option():
    """opts.item_rows: 0 (default size) or 64..65536; smaller items mean more
    work items (more partials in the workspace); it is part of the group key."""
    binding, lib = _lib()
    off = np.array([0, 5000, 5100, 12000], dtype=np.int64)
    h = off.ctypes.data_as(ctypes.c_void_p).value
    t = binding.c_tensor(3, 8, 0x1000, h, 0x2000, binding.DPAR2_F32, None)
    size = lambda ir: lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, ir)))
    assert size(0) > 0 and size(64) > size(1024) > size(0) == size(16384)
    for bad in (1, 63, 65537, -5):
        assert size(bad) == 0
        assert b"item_rows" in lib.dpar2_last_error()
    T = binding.c_tensor * 2
    O = binding.c_opts * 2
    one = lib.dpar2_batch_workspace_size(2, T(t, t), O(binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, 0),
                                                        binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, 0)))
    two = lib.dpar2_batch_workspace_size(2, T(t, t), O(binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, 0),
                                                        binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, 512)))
    al = lambda n: (n + 255) // 256 * 256
    assert two == al(size(0)) + al(size(512)) and one < two


def test_wide_slab_flag_and_autotuner_arguments():
    """DPAR2_FLAG_WIDE_SLAB is part of the group key (a batch mixing it forms
    two groups); the slab autotuner rejects missing candidate arrays before
    touching the device."""
    binding, lib = _lib()
    off = np.array([0, 500, 900], dtype=np.int64)
    h = off.ctypes.data_as(ctypes.c_void_p).value
    t = binding.c_tensor(2, 24, 0x1000, h, 0x2000, binding.DPAR2_F32, None)
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0, 0, 0)
    ow = binding.c_opts(2, 3, 3, 5, -1.0, binding.DPAR2_FLAG_WIDE_SLAB, 0, 0)
    one = lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o))
    wide = lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(ow))
    assert wide >= one + (3 * 16 * 64 + 16 * 4) * ((900 + 63) // 64 + 2)
    T = binding.c_tensor * 2
    O = binding.c_opts * 2
    al = lambda n: (n + 255) // 256 * 256
    assert lib.dpar2_batch_workspace_size(2, T(t, t), O(o, ow)) == al(one) + al(wide)
    rows = (ctypes.c_int32 * 2)(0, 0)
    best = ctypes.c_int32()
    st = lib.dpar2_autotune_slab(ctypes.byref(t), ctypes.byref(o), ctypes.c_void_p(0x3000), rows, None, 2,
                                 ctypes.c_void_p(0x4000), 1 << 30, ctypes.byref(best), None, None)
    assert st == -1
    assert b"wide" in lib.dpar2_last_error()
    st = lib.dpar2_autotune_slab(ctypes.byref(t), ctypes.byref(o), ctypes.c_void_p(0x3000), None, rows, 2,
                                 ctypes.c_void_p(0x4000), 1 << 30, ctypes.byref(best), None, None)
    assert st == -1


def test_workspace_bytes_and_new_entry_points_validate_on_host():
    """dpar2_workspace_bytes (and its earlier name) agree; the resumable flag
    is accepted and is part of the group key; decompose, output_A and
    release reject bad arguments before touching the device; release of a
    workspace the library never saw is a no-op."""
    binding, lib = _lib()
    t, _keep = _tensor(binding, [0, 10, 25, 40])
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0)
    od = binding.c_opts(2, 3, 3, 5, -1.0, binding.DPAR2_FLAG_DETERMINISTIC)
    n = lib.dpar2_workspace_bytes(ctypes.byref(t), ctypes.byref(o))
    assert n > 0 and n == lib.dpar2_workspace_size(ctypes.byref(t), ctypes.byref(o))
    assert lib.dpar2_workspace_bytes(ctypes.byref(t), ctypes.byref(od)) == n
    T = binding.c_tensor * 2
    O = binding.c_opts * 2
    al = lambda x: (x + 255) // 256 * 256
    assert lib.dpar2_batch_workspace_size(2, T(t, t), O(o, od)) == 2 * al(n)
    f = binding.c_factors(0x5000, 0x6000, 0x7000)
    rep = binding.c_report()
    # NULL omega, NULL factor pointer, workspace too small: no device work
    assert lib.dpar2_decompose(ctypes.byref(t), ctypes.byref(o), None, 0x4000, ctypes.byref(f), None,
                               ctypes.byref(rep), 0x10000, n, None) == -1
    fz = binding.c_factors(0x5000, None, 0x7000)
    assert lib.dpar2_decompose(ctypes.byref(t), ctypes.byref(o), 0x3000, 0x4000, ctypes.byref(fz), None,
                               ctypes.byref(rep), 0x10000, n, None) == -1
    assert lib.dpar2_decompose(ctypes.byref(t), ctypes.byref(o), 0x3000, 0x4000, ctypes.byref(f), None,
                               ctypes.byref(rep), 0x10000, n - 1, None) == -6
    assert lib.dpar2_output_A(ctypes.byref(t), ctypes.byref(o), None, 0x10000, n, None) == -1
    assert lib.dpar2_output_A(ctypes.byref(t), ctypes.byref(o), 0x8000, 0x10000, n - 1, None) == -6
    assert lib.dpar2_release(ctypes.c_void_p(0x123400)) == 0
    assert lib.dpar2_release(None) == 0


def test_append_validates_on_host():
    """dpar2_append_workspace_bytes: the grown tensor's layout plus the
    appended slices' own (larger than a plain workspace, zero for a bad
    k_prev); dpar2_append rejects k_prev out of range, NULL factors or
    omegas, a ws_prev or ws that is too small, and overlapping workspaces,
    all before touching the device.  An append of one slice with R = 2 and
    L2 = 3 > 1 * R is accepted (the new slices run no second stage of their
    own)."""
    binding, lib = _lib()
    t, _keep = _tensor(binding, [0, 10, 25, 40, 52])
    o = binding.c_opts(2, 3, 3, 5, -1.0, 0)
    tp, _kp = _tensor(binding, [0, 10, 25, 40])
    n_all = lib.dpar2_workspace_bytes(ctypes.byref(t), ctypes.byref(o))
    n_prev = lib.dpar2_workspace_bytes(ctypes.byref(tp), ctypes.byref(o))
    n = lib.dpar2_append_workspace_bytes(ctypes.byref(t), 3, ctypes.byref(o))
    assert n > n_all > n_prev > 0
    for bad in (0, 4, -1):
        assert lib.dpar2_append_workspace_bytes(ctypes.byref(t), bad, ctypes.byref(o)) == 0
    f = binding.c_factors(0x5000, 0x6000, 0x7000)
    fz = binding.c_factors(0x5000, None, 0x7000)
    prev, ws = 0x100000000, 0x200000000

    def call(k=3, om1=0x3000, om2=0x4000, wp=prev, nwp=n_prev, fac=f, w=ws, nw=n):
        return lib.dpar2_append(ctypes.byref(t), k, ctypes.byref(o), om1, om2, wp, nwp, ctypes.byref(fac),
                                None, None, w, nw, None)
    assert call(k=0) == -1 and call(k=4) == -1
    assert call(om1=None) == -1 and call(om2=None) == -1
    assert call(fac=fz) == -1
    assert call(nwp=n_prev - 1) == -6 and b"ws_prev" in lib.dpar2_last_error()
    assert call(nw=n - 1) == -6
    assert call(w=0) == -6 and call(w=ws + 16) == -6
    assert call(w=prev + 256 * (n_prev // 512)) == -1           # overlaps ws_prev
    assert b"overlap" in lib.dpar2_last_error()
