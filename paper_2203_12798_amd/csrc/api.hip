// C ABI of libdpar2: argument validation, the first-stage work schedule (the
// GPU form of Alg. 4), workspace carving and the launch sequence of Alg. 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dpar2.h"
#include "internal.h"

using namespace dpar2;

namespace {

thread_local std::string g_last_error;

dpar2_status fail(dpar2_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// A group of tensors sharing J, R, L, L2, the dtype and the iteration options
// (a single-tensor call is a group of one).
struct Group {
  int nt = 0;
  std::vector<dpar2_tensor> Xv;        // nt tensors (copies of the caller's structs)
  std::vector<dpar2_opts> ov;          // nt options
  std::vector<int> orig;               // index of each tensor in the caller's batch
  const dpar2_tensor* X = nullptr;     // = Xv.data()
  const dpar2_opts* o = nullptr;       // = ov.data()
  std::vector<int64_t> k0;             // first global slice of each tensor (nt + 1)
  bool noalloc = false;                // dpar2_decompose_noalloc: tables as kernel arguments,
                                       // no pinned staging, no graphs, no profiling events
};

// Host-side tables of a group: the slab-pass schedule and the block / chunk
// maps of the per-slice and second-stage kernels.
struct Schedule {
  std::vector<Item> items;          // longest first; Item::pad = tensor
  std::vector<int32_t> slice_ptr;   // K+1
  std::vector<int32_t> slice_list;  // item indices of each slice
  std::vector<Blk> blk, blk0;
  std::vector<Chunk> chunks, ychunks;
  std::vector<int64_t> seg_blk, seg_blk0, seg_chunk, seg_ychunk, seg_slice;
  std::vector<int32_t> slice_t;
};

dpar2_status validate(const dpar2_tensor* X, const dpar2_opts* o) {
  if (!X || !o) return fail(DPAR2_EINVAL, "tensor or options pointer is NULL");
  if (X->K < 1 || X->J < 1) return fail(DPAR2_EINVAL, "K and J must be >= 1");
  if (X->K > (int64_t)1 << 30) return fail(DPAR2_EINVAL, "K too large");
  if (X->J > (int64_t)1 << 30) return fail(DPAR2_EINVAL, "J too large");
  if (!X->row_offsets || !X->row_offsets_host || !X->slab)
    return fail(DPAR2_EINVAL, "row_offsets, row_offsets_host and slab must be non-NULL");
  if (X->dtype != DPAR2_F32 && X->dtype != DPAR2_BF16 && X->dtype != DPAR2_FP8_E4M3)
    return fail(DPAR2_EINVAL, "unsupported slab dtype");
  if (X->dtype == DPAR2_FP8_E4M3 && !X->slice_scale)
    return fail(DPAR2_EINVAL, "fp8 slabs need slice_scale");
  if (o->flags & ~(DPAR2_FLAG_NO_GRAPH | DPAR2_FLAG_WIDE_SLAB | DPAR2_FLAG_DETERMINISTIC))
    return fail(DPAR2_EINVAL, "unknown bits in opts.flags");
  if (o->item_rows != 0 && (o->item_rows < 64 || o->item_rows > 65536))
    return fail(DPAR2_EINVAL, "opts.item_rows must be 0 or in 64..65536");
  if (o->power_iters < 0 || o->power_iters > 4) return fail(DPAR2_EINVAL, "power_iters must be in [0, 4]");
  const int R = o->rank, L = o->sketch, L2 = o->sketch2;
  if (!rank_supported(R)) return fail(DPAR2_ESHAPE, "rank must be in [1, 32] or one of 40, 50");
  if (L < R || !width_supported(L))
    return fail(DPAR2_ESHAPE, "sketch width L must satisfy R <= L and be in [1, 32] or one of 40, 50, 60");
  if (L2 < R || !width_supported(L2))
    return fail(DPAR2_ESHAPE, "sketch width L2 must satisfy R <= L2 and be in [1, 32] or one of 40, 50, 60");
  if (o->max_iter < 0) return fail(DPAR2_EINVAL, "max_iter must be >= 0");
  const int64_t K = X->K, J = X->J;
  if (L > J) return fail(DPAR2_ESHAPE, "sketch width L exceeds J");
  if (L2 > J) return fail(DPAR2_ESHAPE, "sketch width L2 exceeds J");
  if ((int64_t)L2 > K * R) return fail(DPAR2_ESHAPE, "sketch width L2 exceeds K*R");
  if (!sketch_supported((int)J, L, X->dtype))
    return fail(DPAR2_ESHAPE, "J exceeds the slab pass limit of 16384 columns");
  const int64_t* off = X->row_offsets_host;
  if (off[0] != 0) return fail(DPAR2_EINVAL, "row_offsets[0] must be 0");
  for (int64_t k = 0; k < K; ++k) {
    if (off[k + 1] < off[k]) return fail(DPAR2_EINVAL, "row_offsets must be non-decreasing");
    if (off[k + 1] - off[k] < L)
      return fail(DPAR2_ESHAPE, "slice " + std::to_string(k) + " has fewer rows than the sketch width L");
  }
  return DPAR2_OK;
}

// Options that tensors of one group share (everything but tol).
bool same_group(const dpar2_tensor& a, const dpar2_opts& oa, const dpar2_tensor& b, const dpar2_opts& ob) {
  return a.J == b.J && a.dtype == b.dtype && oa.rank == ob.rank && oa.sketch == ob.sketch &&
         oa.sketch2 == ob.sketch2 && oa.power_iters == ob.power_iters && oa.max_iter == ob.max_iter &&
         oa.flags == ob.flags && oa.item_rows == ob.item_rows;
}

dpar2_status make_group(int32_t n, const dpar2_tensor* X, const dpar2_opts* o, Group* g) {
  if (n < 1) return fail(DPAR2_EINVAL, "a group needs at least one tensor");
  if (!X || !o) return fail(DPAR2_EINVAL, "tensor or options pointer is NULL");
  g->nt = n;
  g->Xv.assign(X, X + n);
  g->ov.assign(o, o + n);
  g->X = g->Xv.data();
  g->o = g->ov.data();
  if (g->orig.size() != (size_t)n) {
    g->orig.resize((size_t)n);
    std::iota(g->orig.begin(), g->orig.end(), 0);
  }
  g->k0.assign((size_t)n + 1, 0);
  for (int32_t t = 0; t < n; ++t) {
    dpar2_status st = validate(&X[t], &o[t]);
    if (st != DPAR2_OK) {
      if (n > 1) g_last_error = "tensor " + std::to_string(g->orig[(size_t)t]) + ": " + g_last_error;
      return st;
    }
    if (!same_group(X[t], o[t], X[0], o[0]))
      return fail(DPAR2_EINVAL, "tensors of one group must share J, dtype, rank, sketch widths, "
                                "power_iters, max_iter and flags (tensor " + std::to_string(t) + " differs)");
    g->k0[(size_t)t + 1] = g->k0[(size_t)t] + X[t].K;
  }
  if (g->k0[(size_t)n] > ((int64_t)1 << 30)) return fail(DPAR2_EINVAL, "too many slices in one batch");
  return DPAR2_OK;
}

// Alg. 4 on the GPU: slices longer than the item size (opts.item_rows, default
// MAX_CHUNK_ROWS) are cut into near-equal
// row ranges; all items are sorted by length, longest first (stable), and
// block b of the slab pass takes item b.  The hardware dispatcher starts each
// next block on the first compute unit that frees up, i.e. greedy list
// scheduling of the longest remaining item on the least-loaded unit.
int64_t item_cap(const Group& g) { return g.o[0].item_rows > 0 ? g.o[0].item_rows : MAX_CHUNK_ROWS; }
int64_t items_of(int64_t rows, int64_t cap) { return std::max<int64_t>(1, (rows + cap - 1) / cap); }

void build_schedule(const Group& g, Schedule* s) {
  const int nt = g.nt;
  const int64_t K = g.k0[(size_t)nt];
  const int64_t J = g.X[0].J;
  const int R = g.o[0].rank;
  const int64_t cap = item_cap(g);
  std::vector<Item> raw;
  raw.reserve((size_t)K);
  int64_t rbase = 0;   // first row of tensor t in the group's row space
  for (int t = 0; t < nt; ++t) {
    const int64_t* off = g.X[t].row_offsets_host;
    for (int64_t k = 0; k < g.X[t].K; ++k) {
      const int64_t n = off[k + 1] - off[k], nc = items_of(n, cap);
      for (int64_t c = 0; c < nc; ++c) {
        Item it;
        it.row0 = off[k] + n * c / nc;
        it.row1 = off[k] + n * (c + 1) / nc;
        it.slice = (int32_t)(g.k0[(size_t)t] + k);
        it.pad = t;
        // items in row order: the slot ranges [floor(row / 64) + i, + tiles)
        // of consecutive items never overlap, and the last one ends below
        // ceil(N / 64) + n_items
        it.tslot = (rbase + it.row0) / SKETCH_TM + (int64_t)raw.size();
        raw.push_back(it);
      }
    }
    rbase += off[g.X[t].K];
  }
  std::vector<size_t> idx(raw.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    return (raw[a].row1 - raw[a].row0) > (raw[b].row1 - raw[b].row0);
  });
  s->items.resize(raw.size());
  for (size_t i = 0; i < idx.size(); ++i) s->items[i] = raw[idx[i]];
  s->slice_ptr.assign((size_t)K + 1, 0);
  for (const Item& it : s->items) s->slice_ptr[(size_t)it.slice + 1]++;
  for (int64_t k = 0; k < K; ++k) s->slice_ptr[(size_t)k + 1] += s->slice_ptr[(size_t)k];
  s->slice_list.assign(s->items.size(), 0);
  std::vector<int32_t> fill(s->slice_ptr.begin(), s->slice_ptr.end() - 1);
  for (size_t i = 0; i < s->items.size(); ++i) s->slice_list[(size_t)fill[s->items[i].slice]++] = (int32_t)i;
  // per-slice kernel blocks (never straddling tensors), begin blocks (local
  // rows 0 .. max(K_t, J)), second-stage chunks of M^T, slice -> tensor
  const int gpb = als_slices_per_block(R);
  s->blk.clear();
  s->blk0.clear();
  s->chunks.clear();
  s->ychunks.clear();
  s->seg_blk.assign(1, 0);
  s->seg_blk0.assign(1, 0);
  s->seg_chunk.assign(1, 0);
  s->seg_ychunk.assign(1, 0);
  s->seg_slice.assign(g.k0.begin(), g.k0.end());
  s->slice_t.assign((size_t)K, 0);
  for (int t = 0; t < nt; ++t) {
    const int64_t k0 = g.k0[(size_t)t], Kt = g.X[t].K;
    for (int64_t b = 0; b < Kt; b += gpb)
      s->blk.push_back(Blk{t, (int32_t)(k0 + b), (int32_t)(k0 + std::min<int64_t>(Kt, b + gpb)), 0});
    const int64_t rows = std::max<int64_t>(Kt, J);
    for (int64_t b = 0; b < rows; b += gpb)
      s->blk0.push_back(Blk{t, (int32_t)b, (int32_t)std::min<int64_t>(rows, b + gpb), 0});
    for (int64_t r = k0 * R; r < (k0 + Kt) * R; r += STAGE2_CHUNK)
      s->chunks.push_back(Chunk{r, std::min<int64_t>((k0 + Kt) * R, r + STAGE2_CHUNK), t, 0});
    // the tensor's own chunk length, so that its partial sums are blocked as
    // in a decomposition of that tensor alone
    const int64_t ych = stage2_ychunk(Kt * R, J);
    for (int64_t r = k0 * R; r < (k0 + Kt) * R; r += ych)
      s->ychunks.push_back(Chunk{r, std::min<int64_t>((k0 + Kt) * R, r + ych), t, 0});
    s->seg_blk.push_back((int64_t)s->blk.size());
    s->seg_blk0.push_back((int64_t)s->blk0.size());
    s->seg_chunk.push_back((int64_t)s->chunks.size());
    s->seg_ychunk.push_back((int64_t)s->ychunks.size());
    for (int64_t k = 0; k < Kt; ++k) s->slice_t[(size_t)(k0 + k)] = t;
  }
}

Layout make_layout(const Group& g) {
  Layout y;
  std::memset(&y, 0, sizeof(y));
  const dpar2_opts* o = g.o;
  y.nt = g.nt;
  y.K = g.k0[(size_t)g.nt];
  y.J = g.X[0].J;
  y.R = o->rank;
  y.L = o->sketch;
  y.L2 = o->sketch2;
  y.max_iter = o->max_iter;
  y.q = o->power_iters;
  y.N = 0;
  y.n_items = 0;
  y.n2 = 0;
  y.n2y = 0;
  y.nblk = 0;
  y.nblk0 = 0;
  const int gpb = als_slices_per_block(y.R);
  for (int t = 0; t < g.nt; ++t) {
    const int64_t* off = g.X[t].row_offsets_host;
    const int64_t Kt = g.X[t].K;
    y.N += off[Kt];
    for (int64_t k = 0; k < Kt; ++k) y.n_items += items_of(off[k + 1] - off[k], item_cap(g));
    y.n2 += (Kt * y.R + STAGE2_CHUNK - 1) / STAGE2_CHUNK;
    const int64_t ych = stage2_ychunk(Kt * y.R, y.J);
    y.n2y += (Kt * y.R + ych - 1) / ych;
    y.nblk += (int)((Kt + gpb - 1) / gpb);
    y.nblk0 += (int)((std::max<int64_t>(Kt, y.J) + gpb - 1) / gpb);
  }
  const int64_t nt = y.nt, K = y.K, J = y.J, R = y.R, L = y.L, L2 = y.L2, KR = K * R, RR = R * R;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align256(p + bytes);
    return at;
  };
  y.tdesc = take(sizeof(TDesc) * (size_t)nt);
  y.blk = take(sizeof(Blk) * (size_t)y.nblk);
  y.blk0 = take(sizeof(Blk) * (size_t)y.nblk0);
  y.chunks = take(sizeof(Chunk) * (size_t)y.n2);
  y.ychunks = take(sizeof(Chunk) * (size_t)y.n2y);
  y.seg_blk = take(sizeof(int64_t) * (size_t)(nt + 1));
  y.seg_blk0 = take(sizeof(int64_t) * (size_t)(nt + 1));
  y.seg_chunk = take(sizeof(int64_t) * (size_t)(nt + 1));
  y.seg_ychunk = take(sizeof(int64_t) * (size_t)(nt + 1));
  y.seg_slice = take(sizeof(int64_t) * (size_t)(nt + 1));
  y.slice_t = take(sizeof(int32_t) * (size_t)K);
  y.items = take(sizeof(Item) * (size_t)y.n_items);
  y.slice_ptr = take(sizeof(int32_t) * (size_t)(K + 1));
  y.slice_list = take(sizeof(int32_t) * (size_t)y.n_items);
  y.tables_end = p;   // [tdesc, tables_end): host-built tables, one upload
  y.ctl = take(sizeof(Ctl) * (size_t)nt);
  y.partG = take(sizeof(double) * (size_t)(y.n_items * L * L));
  y.partP = take(sizeof(double) * (size_t)(y.n_items * L * J));
  y.partS = take(sizeof(double) * (size_t)y.n_items);
  y.xnorm2 = take(sizeof(double) * (size_t)K);
  y.Mt = take(sizeof(double) * (size_t)(KR * J));
  y.Phi = take(sizeof(double) * (size_t)(K * L * R));
  y.sig1 = take(sizeof(double) * (size_t)KR);
  y.msgn = take(sizeof(float) * (size_t)KR);
  y.Y2p = take(sizeof(double) * (size_t)(y.n2y * L2 * J));
  y.Y2 = take(sizeof(double) * (size_t)(nt * J * L2));
  y.B2t = take(sizeof(double) * (size_t)(KR * L2));
  y.S2p = take(sizeof(double) * (size_t)(y.n2 * L2 * (L2 + 1) / 2));
  y.S2 = take(sizeof(double) * (size_t)(nt * L2 * (L2 + 1) / 2));
  y.U2 = take(sizeof(double) * (size_t)(nt * L2 * R));
  y.s2s = take(sizeof(double) * (size_t)s2_scratch_doubles(nt, J, L2, R));
  y.D = take(sizeof(double) * (size_t)(nt * J * R));
  y.E = take(sizeof(double) * (size_t)(nt * R));
  y.F = take(sizeof(double) * (size_t)(KR * R));
  y.FtFp = take(sizeof(double) * (size_t)(y.n2 * RR));
  y.Psi = take(sizeof(double) * (size_t)(K * RR));
  y.Pw = take(sizeof(double) * (size_t)(K * RR));
  y.Mk = take(sizeof(double) * (size_t)(K * RR));
  y.small = take(sizeof(double) * (size_t)(nt * SM_COUNT * RR));
  y.partA = take(sizeof(double) * (size_t)(y.nblk * RR));
  y.partB = take(sizeof(double) * (size_t)(y.nblk * RR));
  y.partC = take(sizeof(double) * (size_t)(y.nblk * (RR + 2)));
  y.partBegin = take(sizeof(double) * (size_t)(y.nblk0 * 3 * RR));
  y.red = take(sizeof(double) * (size_t)(nt * (RED_WIDTH * RR + 2)));
  y.fitp = take(sizeof(double) * (size_t)(2 * K + 2 * nt));
  y.trace = take(sizeof(double) * (size_t)(K * L * R));   // Theta for the U output
  y.om1 = take(sizeof(float) * (size_t)(nt * J * L));      // copy of each Omega_1 for the U pass
  y.omq = take(y.q > 0 ? sizeof(float) * (size_t)(K * J * L) : 0);   // power-step sketches
  // the wide slab pass keeps Y (16 LT floats per row) between its two kernels
  y.wide = J > narrow_j_limit(g.X[0].dtype) || y.L > 32 || (o->flags & DPAR2_FLAG_WIDE_SLAB) != 0;
  y.ybuf = take(y.wide ? wide_tile_bytes(y.L) * (size_t)((y.N + SKETCH_TM - 1) / SKETCH_TM + y.n_items) : 0);
  y.det = (o->flags & DPAR2_FLAG_DETERMINISTIC) != 0;
  y.total = p;
  return y;
}

// Every field of a layout, in declaration order (the graph cache key).
std::vector<int64_t> layout_key(const Layout& y) {
  return {y.nt, y.K, y.J, y.N, y.n_items, y.R, y.L, y.L2, y.max_iter, y.q, y.n2, y.n2y, y.nblk, y.nblk0,
          (int64_t)y.tdesc, (int64_t)y.blk, (int64_t)y.blk0, (int64_t)y.chunks, (int64_t)y.ychunks, (int64_t)y.seg_blk,
          (int64_t)y.seg_blk0, (int64_t)y.seg_chunk, (int64_t)y.seg_ychunk, (int64_t)y.seg_slice, (int64_t)y.slice_t, (int64_t)y.ctl,
          (int64_t)y.items, (int64_t)y.slice_ptr, (int64_t)y.slice_list, (int64_t)y.partG, (int64_t)y.partP,
          (int64_t)y.partS, (int64_t)y.xnorm2, (int64_t)y.Mt, (int64_t)y.Phi, (int64_t)y.sig1, (int64_t)y.msgn, (int64_t)y.Y2p,
          (int64_t)y.Y2, (int64_t)y.B2t, (int64_t)y.S2p, (int64_t)y.S2, (int64_t)y.U2, (int64_t)y.s2s, (int64_t)y.D,
          (int64_t)y.E, (int64_t)y.F, (int64_t)y.FtFp, (int64_t)y.Psi, (int64_t)y.Pw, (int64_t)y.Mk,
          (int64_t)y.small, (int64_t)y.partA, (int64_t)y.partB, (int64_t)y.partC, (int64_t)y.partBegin,
          (int64_t)y.red, (int64_t)y.fitp, (int64_t)y.trace, (int64_t)y.om1, (int64_t)y.omq, (int64_t)y.ybuf,
          (int64_t)y.wide, (int64_t)y.det, (int64_t)y.tables_end, (int64_t)y.total};
}

dpar2_status check_ws(const Layout& y, const void* ws, size_t bytes) {
  if (!ws) return fail(DPAR2_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(DPAR2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < y.total)
    return fail(DPAR2_EWORKSPACE, "workspace too small: need " + std::to_string(y.total) + " bytes");
  return DPAR2_OK;
}

// A batch: its tensors partitioned into groups (same J, dtype, rank, sketch
// widths, power_iters, max_iter and flags; in order of first appearance),
// each group with its own layout in consecutive 256-byte aligned parts of
// one workspace.
struct Batch {
  std::vector<Group> groups;
  std::vector<Layout> lay;
  std::vector<size_t> base;
  size_t total = 0;
};

dpar2_status make_batch(int32_t n, const dpar2_tensor* X, const dpar2_opts* o, Batch* b) {
  if (n < 1) return fail(DPAR2_EINVAL, "a batch needs at least one tensor");
  if (!X || !o) return fail(DPAR2_EINVAL, "tensor or options pointer is NULL");
  std::vector<std::vector<int>> members;
  for (int32_t t = 0; t < n; ++t) {
    const dpar2_status st = validate(&X[t], &o[t]);
    if (st != DPAR2_OK) {
      g_last_error = "tensor " + std::to_string(t) + ": " + g_last_error;
      return st;
    }
    size_t gi = 0;
    while (gi < members.size() && !same_group(X[t], o[t], X[members[gi][0]], o[members[gi][0]])) ++gi;
    if (gi == members.size()) members.emplace_back();
    members[gi].push_back(t);
  }
  b->groups.resize(members.size());
  b->lay.clear();
  b->base.clear();
  b->total = 0;
  for (size_t gi = 0; gi < members.size(); ++gi) {
    std::vector<dpar2_tensor> xs;
    std::vector<dpar2_opts> os;
    for (int t : members[gi]) {
      xs.push_back(X[t]);
      os.push_back(o[t]);
    }
    Group& g = b->groups[gi];
    g.orig = members[gi];
    dpar2_status st = make_group((int32_t)xs.size(), xs.data(), os.data(), &g);
    if (st != DPAR2_OK) return st;
    b->lay.push_back(make_layout(g));
    b->base.push_back(b->total);
    b->total = align256(b->total + b->lay.back().total);
  }
  return DPAR2_OK;
}

dpar2_status hip_fail(hipError_t e, const char* where) {
  return fail(DPAR2_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Pinned staging buffers for the table uploads: a ring of STAGE_SLOTS per
// workspace, each guarded by an event until the copy out of it has completed
// (so the host waits only on an upload STAGE_SLOTS calls back).  Each upload
// is ONE copy of a contiguous image of the table region of the workspace.
constexpr int STAGE_SLOTS = 4;
struct Staging {
  void* host[STAGE_SLOTS] = {};
  size_t bytes[STAGE_SLOTS] = {};
  hipEvent_t done[STAGE_SLOTS] = {};
  int next = 0;
  // host image of the schedule tables of the last compress on this
  // workspace, and what it was built from (reused when that is unchanged)
  std::vector<int64_t> key;
  std::vector<char> image;
};
std::mutex g_stage_mu;
std::unordered_map<const void*, Staging> g_stage;

__global__ __launch_bounds__(256) void k_upload(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

// Copies bytes [0, n) of `img` to the workspace at offset `at`, through the
// staging ring, asynchronously on s.  Caller holds g_stage_mu.
dpar2_status upload_locked(Staging& sg, char* w, const char* img, size_t n, size_t at, hipStream_t s) {
  const int i = sg.next;
  sg.next = (i + 1) % STAGE_SLOTS;
  hipError_t e;
  if (sg.done[i]) {
    if ((e = hipEventSynchronize(sg.done[i])) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  } else if ((e = hipEventCreateWithFlags(&sg.done[i], hipEventDisableTiming)) != hipSuccess) {
    return hip_fail(e, "hipEventCreate");
  }
  const size_t cap = (n + 15) / 16 * 16;
  if (sg.bytes[i] < cap) {
    if (sg.host[i]) (void)hipHostFree(sg.host[i]);
    sg.host[i] = nullptr;
    sg.bytes[i] = 0;
    if ((e = hipHostMalloc(&sg.host[i], cap, hipHostMallocDefault)) != hipSuccess)
      return hip_fail(e, "hipHostMalloc");
    sg.bytes[i] = cap;
  }
  std::memcpy(sg.host[i], img, n);
  // a kernel reads the pinned buffer over the bus: stream-ordered like a
  // copy, without the host waiting for the stream
  const int64_t n16 = (int64_t)(n + 15) / 16;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (n16 + 255) / 256);
  hipLaunchKernelGGL(k_upload, dim3(blocks), dim3(256), 0, s, static_cast<const uint4*>(sg.host[i]),
                     reinterpret_cast<uint4*>(w + at), n16);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "table upload");
  if ((e = hipEventRecord(sg.done[i], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return DPAR2_OK;
}

// Upload without any allocation (dpar2_decompose_noalloc): the bytes travel
// as the by-value argument of a copy kernel, PUT_BYTES per launch, so no
// pinned buffer and no copy from pageable host memory is involved.
constexpr int PUT_BYTES = 3072;
struct PutArg {
  unsigned char b[PUT_BYTES];
};
__global__ __launch_bounds__(256) void k_put(PutArg a, unsigned char* __restrict__ dst, int n) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = a.b[i];
}
dpar2_status upload_args(char* w, const char* img, size_t n, size_t at, hipStream_t s) {
  PutArg a;
  for (size_t o = 0; o < n; o += PUT_BYTES) {
    const int m = (int)std::min<size_t>(PUT_BYTES, n - o);
    std::memcpy(a.b, img + o, (size_t)m);
    hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, s, a, reinterpret_cast<unsigned char*>(w + at + o), m);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "table upload (kernel arguments)");
}

// Per-tensor descriptors; factor and trace pointers come from the call that
// uses them (NULL where a call has none).
std::vector<TDesc> descriptors(const Group& g, const float* const* om1, const float* const* om2,
                               const dpar2_factors* f, double* const* trace) {
  std::vector<TDesc> td((size_t)g.nt);
  int64_t rbase = 0;
  for (int t = 0; t < g.nt; ++t) {
    TDesc& d = td[(size_t)t];
    std::memset(&d, 0, sizeof(d));
    d.rbase = rbase;
    rbase += g.X[t].row_offsets_host[g.X[t].K];
    d.K = g.X[t].K;
    d.k0 = g.k0[(size_t)t];
    d.slab = g.X[t].slab;
    d.scale = g.X[t].dtype == DPAR2_FP8_E4M3 ? g.X[t].slice_scale : nullptr;
    d.om1 = om1 ? om1[t] : nullptr;
    d.om2 = om2 ? om2[t] : nullptr;
    if (f) {
      d.H = f[t].H;
      d.V = f[t].V;
      d.W = f[t].W;
    }
    d.trace = trace ? trace[t] : nullptr;
    d.tol = g.o[t].tol;
  }
  return td;
}

// Slab-pass timing (dpar2_profile_*).
struct Profile {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
};
std::mutex g_prof_mu;
Profile g_prof;

// Start of a compress: clears each tensor's control block and keeps a copy
// of its Omega_1 in the workspace (for a later U pass); one block per tensor.
__global__ __launch_bounds__(256) void k_prep(const TDesc* __restrict__ td, int JL, Ctl* __restrict__ ctl,
                                              float* __restrict__ om1_copy) {
  const int t = blockIdx.x;
  if (threadIdx.x == 0) {
    Ctl z;
    std::memset(&z, 0, sizeof(z));
    ctl[t] = z;
  }
  const float* __restrict__ src = td[t].om1;
  float* __restrict__ dst = om1_copy + (size_t)t * JL;
  for (int e = threadIdx.x; e < JL; e += 256) dst[e] = src[e];
}

// Puts the schedule tables of g (the part of [tdesc, tables_end) after the
// descriptors) into sg.image, rebuilding them only when what they depend on
// (J, R and every tensor's row offsets) changed since the last compress on
// this workspace.
void stage_tables(const Group& g, const Layout& y, Staging& sg) {
  std::vector<int64_t> key = {g.nt, y.J, y.R, item_cap(g)};
  for (int t = 0; t < g.nt; ++t) {
    key.push_back(g.X[t].K);
    key.insert(key.end(), g.X[t].row_offsets_host, g.X[t].row_offsets_host + g.X[t].K + 1);
  }
  const size_t n = y.tables_end - y.tdesc;
  if (key == sg.key && sg.image.size() == n) return;
  Schedule sch;
  build_schedule(g, &sch);
  sg.image.assign(n, 0);
  auto put = [&](const void* src, size_t bytes, size_t at) {
    if (bytes) std::memcpy(sg.image.data() + (at - y.tdesc), src, bytes);
  };
  put(sch.blk.data(), sizeof(Blk) * sch.blk.size(), y.blk);
  put(sch.blk0.data(), sizeof(Blk) * sch.blk0.size(), y.blk0);
  put(sch.chunks.data(), sizeof(Chunk) * sch.chunks.size(), y.chunks);
  put(sch.ychunks.data(), sizeof(Chunk) * sch.ychunks.size(), y.ychunks);
  put(sch.seg_blk.data(), sizeof(int64_t) * sch.seg_blk.size(), y.seg_blk);
  put(sch.seg_blk0.data(), sizeof(int64_t) * sch.seg_blk0.size(), y.seg_blk0);
  put(sch.seg_chunk.data(), sizeof(int64_t) * sch.seg_chunk.size(), y.seg_chunk);
  put(sch.seg_ychunk.data(), sizeof(int64_t) * sch.seg_ychunk.size(), y.seg_ychunk);
  put(sch.seg_slice.data(), sizeof(int64_t) * sch.seg_slice.size(), y.seg_slice);
  put(sch.slice_t.data(), sizeof(int32_t) * sch.slice_t.size(), y.slice_t);
  put(sch.items.data(), sizeof(Item) * sch.items.size(), y.items);
  put(sch.slice_ptr.data(), sizeof(int32_t) * sch.slice_ptr.size(), y.slice_ptr);
  put(sch.slice_list.data(), sizeof(int32_t) * sch.slice_list.size(), y.slice_list);
  sg.key = std::move(key);
}

// Uploads the descriptors alone (factor and trace pointers of a call).
dpar2_status upload_descriptors(char* w, const Layout& y, const std::vector<TDesc>& td, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  return upload_locked(g_stage[w], w, reinterpret_cast<const char*>(td.data()), sizeof(TDesc) * td.size(),
                       y.tdesc, s);
}

// --- group steps -------------------------------------------------------------

dpar2_status group_first_stage(const Group& g, char* w, const Layout& y, hipStream_t s);

// Parts of a compress: the first stage (slab passes and per-slice
// completion), the second stage (and the iteration state).  The tables,
// descriptors and control blocks are set up in every case.
enum : int { CP_FIRST = 1, CP_SECOND = 2, CP_ALL = 3 };

dpar2_status group_compress(const Group& g, const float* const* om1, const float* const* om2,
                            const dpar2_factors* f, char* w, const Layout& y, hipStream_t s,
                            int parts = CP_ALL) {
  for (int t = 0; t < g.nt; ++t)
    if (!om1[t] || !om2[t]) return fail(DPAR2_EINVAL, "omega1 and omega2 must be non-NULL");
  const std::vector<TDesc> td = descriptors(g, om1, om2, f, nullptr);
  {
    // descriptors + schedule tables: one copy
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging& sg = g_stage[w];
    stage_tables(g, y, sg);
    std::memcpy(sg.image.data(), td.data(), sizeof(TDesc) * td.size());
    dpar2_status st = g.noalloc ? upload_args(w, sg.image.data(), sg.image.size(), y.tdesc, s)
                                : upload_locked(sg, w, sg.image.data(), sg.image.size(), y.tdesc, s);
    if (st != DPAR2_OK) return st;
  }
  hipError_t e;
  Ctl* ctl = reinterpret_cast<Ctl*>(w + y.ctl);
  hipLaunchKernelGGL(k_prep, dim3((unsigned)g.nt), dim3(256), 0, s, reinterpret_cast<const TDesc*>(w + y.tdesc),
                     (int)(y.J * y.L), ctl, reinterpret_cast<float*>(w + y.om1));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "compress set-up");

  if (parts & CP_FIRST) {
    const dpar2_status st = group_first_stage(g, w, y, s);
    if (st != DPAR2_OK) return st;
  }
  if (!(parts & CP_SECOND)) return DPAR2_OK;
  e = launch_stage2(y, w, s);
  if (e != hipSuccess) return hip_fail(e, "second stage");
  e = launch_pw_identity(y, w, s);
  if (e != hipSuccess) return hip_fail(e, "iteration state init");
  return DPAR2_OK;
}

// The first stage of every slice of g (Sec. III-B, Eq. 4): power_iters + 1
// slab passes, each followed by the per-slice completion.
dpar2_status group_first_stage(const Group& g, char* w, const Layout& y, hipStream_t s) {
  hipError_t e;
  Ctl* ctl = reinterpret_cast<Ctl*>(w + y.ctl);
  const Item* items = reinterpret_cast<const Item*>(w + y.items);
  double* partG = reinterpret_cast<double*>(w + y.partG);
  double* partP = reinterpret_cast<double*>(w + y.partP);
  double* partS = reinterpret_cast<double*>(w + y.partS);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.on && !g.noalloc) {
      if (g_prof.used == g_prof.pool.size()) {
        hipEvent_t a0, a1;
        if ((e = hipEventCreate(&a0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        if ((e = hipEventCreate(&a1)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        g_prof.pool.emplace_back(a0, a1);
      }
      ev0 = g_prof.pool[g_prof.used].first;
      ev1 = g_prof.pool[g_prof.used].second;
      g_prof.used++;
    }
  }
  const int dtype = g.X[0].dtype;
  const int esize = dtype == DPAR2_F32 ? 4 : (dtype == DPAR2_BF16 ? 2 : 1);
  bool vec = y.J % 4 == 0;
  for (int t = 0; t < g.nt; ++t) vec = vec && ((uintptr_t)g.X[t].slab % (4 * esize) == 0);
  SlabArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.td = reinterpret_cast<const TDesc*>(w + y.tdesc);
  sa.J = (int)y.J;
  sa.L = y.L;
  sa.R = y.R;
  sa.items = items;
  sa.partG = partG;
  sa.partP = partP;
  sa.partS = partS;
  sa.ybuf = reinterpret_cast<float*>(w + y.ybuf);
  float* omq = reinterpret_cast<float*>(w + y.omq);
  for (int pass = 0; pass <= y.q; ++pass) {
    // pass 0 sketches with each tensor's Omega_1; a power step with each
    // slice's own matrix
    sa.omega = pass == 0 ? nullptr : omq;
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = launch_slab(sa, dtype, y.n_items, vec, false, y.wide, s);
    if (e != hipSuccess) return hip_fail(e, "slab pass");
    if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    ev0 = ev1 = nullptr;   // the timing hooks cover the first pass
    e = launch_slice_finish(y.K, (int)y.J, y.L, y.R, reinterpret_cast<const int32_t*>(w + y.slice_ptr),
                            reinterpret_cast<const int32_t*>(w + y.slice_list), partG, partP, partS,
                            reinterpret_cast<double*>(w + y.xnorm2), reinterpret_cast<double*>(w + y.Mt),
                            reinterpret_cast<double*>(w + y.Phi), reinterpret_cast<double*>(w + y.sig1),
                            pass < y.q ? omq : nullptr, reinterpret_cast<float*>(w + y.msgn), ctl,
                            reinterpret_cast<const int32_t*>(w + y.slice_t), s);
    if (e != hipSuccess) return hip_fail(e, "slice finish");
  }
  return DPAR2_OK;
}

dpar2_status group_factors(const Group& g, const dpar2_factors* f, double* const* trace, char* w, const Layout& y,
                           hipStream_t s) {
  for (int t = 0; t < g.nt; ++t)
    if (!f[t].H || !f[t].V || !f[t].W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  // the Omega pointers are needed by the slab pass only: the iteration and
  // fitness kernels read factors, trace and tolerance
  return upload_descriptors(w, y, descriptors(g, nullptr, nullptr, f, trace), s);
}

// Streams on which the groups of a batch run side by side (their kernels are
// small and latency-bound), forked from and joined back into the caller's
// stream with events; created once, default priority.
constexpr int BATCH_STREAMS = 8;
struct StreamPool {
  std::mutex mu;
  bool ready = false;
  hipStream_t s[BATCH_STREAMS] = {};
  hipEvent_t done[BATCH_STREAMS] = {};
  hipEvent_t fork = nullptr;
};
StreamPool g_spool;

dpar2_status pool_ready_locked() {
  if (g_spool.ready) return DPAR2_OK;
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&g_spool.fork, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "hipEventCreate");
  for (int i = 0; i < BATCH_STREAMS; ++i) {
    if ((e = hipStreamCreateWithFlags(&g_spool.s[i], hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "hipStreamCreate");
    if ((e = hipEventCreateWithFlags(&g_spool.done[i], hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  }
  g_spool.ready = true;
  return DPAR2_OK;
}

hipError_t enqueue_als(int32_t n_steps, char* w, const Layout& y, hipStream_t s) {
  hipError_t e = launch_als_begin(y, w, s);
  for (int32_t i = 0; e == hipSuccess && i < n_steps; ++i) e = launch_als_iteration(y, w, s);
  if (e == hipSuccess) e = launch_als_end(y, w, s);
  return e;
}

// Captured iteration sequences, per workspace (a few step counts each).
struct GraphEntry {
  std::vector<int64_t> key;
  hipGraphExec_t exec = nullptr;
};
struct GraphCache {
  hipStream_t cap = nullptr;   // capture stream (never runs work)
  std::vector<GraphEntry> entries;
};
constexpr size_t GRAPHS_PER_WS = 4;
std::mutex g_graph_mu;
std::unordered_map<const void*, GraphCache> g_graphs;

dpar2_status group_als(const Group& g, int32_t n_steps, char* w, const Layout& y, hipStream_t s) {
  hipError_t e;
  if (n_steps < 2 || g.noalloc || (g.o[0].flags & DPAR2_FLAG_NO_GRAPH)) {
    if ((e = enqueue_als(n_steps, w, y, s)) != hipSuccess) return hip_fail(e, "iteration");
    return DPAR2_OK;
  }
  // every kernel argument is a workspace address or a layout field: the graph
  // of one (workspace, layout, step count) replays for any factors.  The key
  // holds every field of the layout, so a workspace reused for another shape
  // whose offsets differ never replays a stale graph.
  std::vector<int64_t> key = layout_key(y);
  key.push_back(n_steps);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  GraphCache& gc = g_graphs[w];
  GraphEntry* hit = nullptr;
  for (GraphEntry& ge : gc.entries)
    if (ge.key == key) hit = &ge;
  if (!hit) {
    if (!gc.cap && (e = hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "hipStreamCreate");
    if ((e = hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "hipStreamBeginCapture");
    const hipError_t el = enqueue_als(n_steps, w, y, gc.cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(gc.cap, &graph);
    if (el != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(el, "iteration (capture)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (gc.entries.size() >= GRAPHS_PER_WS) {
      (void)hipGraphExecDestroy(gc.entries.front().exec);
      gc.entries.erase(gc.entries.begin());
    }
    gc.entries.push_back(GraphEntry{key, exec});
    hit = &gc.entries.back();
  }
  if ((e = hipGraphLaunch(hit->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return DPAR2_OK;
}

// U_k = A_k Z_k P_k^T H (Alg. 3 output) by re-running the tiles of the last
// slab pass (same Y bit for bit) against Theta_k = Phi_k Psi_k H; with H ==
// NULL, A_k = Y_k Phi_k itself (Theta_k = Phi_k).  The descriptors on the
// device must hold the Omega_1 of that pass.
dpar2_status group_output_U(const Group& g, const Layout& y, char* w, const double* H, double* U, hipStream_t s) {
  const double* theta = reinterpret_cast<const double*>(w + y.Phi);
  hipError_t e;
  if (H) {
    double* th = reinterpret_cast<double*>(w + y.trace);
    if ((e = launch_theta(y, w, H, th, s)) != hipSuccess) return hip_fail(e, "theta");
    theta = th;
  }
  const int dtype = g.X[0].dtype;
  const int esize = dtype == DPAR2_F32 ? 4 : (dtype == DPAR2_BF16 ? 2 : 1);
  SlabArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.td = reinterpret_cast<const TDesc*>(w + y.tdesc);
  sa.J = (int)y.J;
  sa.L = y.L;
  sa.R = y.R;
  sa.omega = y.q > 0 ? reinterpret_cast<const float*>(w + y.omq) : nullptr;
  sa.items = reinterpret_cast<const Item*>(w + y.items);
  sa.theta = theta;
  sa.U = U;
  sa.ybuf = reinterpret_cast<float*>(w + y.ybuf);
  const bool vec = (y.J % 4 == 0) && ((uintptr_t)g.X[0].slab % (4 * esize) == 0);
  e = launch_slab(sa, dtype, y.n_items, vec, true, y.wide, s);
  if (e != hipSuccess) return hip_fail(e, "U pass");
  return DPAR2_OK;
}

dpar2_status group_report(const Group& g, const void* ws, const Layout& y, dpar2_report* rep, hipStream_t s) {
  std::vector<Ctl> c((size_t)g.nt);
  hipError_t e = hipMemcpyAsync(c.data(), static_cast<const char*>(ws) + y.ctl, sizeof(Ctl) * c.size(),
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int t = 0; t < g.nt; ++t) {
    const Ctl& ct = c[(size_t)t];
    dpar2_report& r = rep[t];
    r.iters = ct.iters;
    r.converged = ct.done && !ct.bad;
    r.err_last = ct.e_prev;
    r.xnorm2 = ct.xnorm2;
    r.fit_compressed = ct.xnorm2 > 0 ? 1.0 - ct.e_prev / ct.xnorm2 : 0.0;
    r.fit_true = ct.fit_true;
    r.warn_bits = ct.warn;
  }
  for (int t = 0; t < g.nt; ++t)
    if (c[(size_t)t].bad)
      return fail(DPAR2_ENUMERIC, "the slab of tensor " + std::to_string(g.orig[(size_t)t]) + " holds NaN or Inf");
  return DPAR2_OK;
}

}  // namespace

namespace {
// Device scratch of dpar2_decompose_noalloc: the workspace of its
// decomposition, one copy per GPU, held until the process ends.  Host code
// never uses the array's name as an address: g_scratch_dev[d] is its device
// address on device d, looked up once with that device current.
constexpr size_t NOALLOC_BYTES = DPAR2_NOALLOC_SCRATCH_BYTES;
constexpr size_t NOALLOC_TABLE_BYTES = size_t(1) << 20;   // schedule tables, sent as kernel arguments
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
dpar2_status scratch_address(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DPAR2_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
    if (!p || (uintptr_t)p % 256 != 0) return fail(DPAR2_EHIP, "scratch symbol address missing or misaligned");
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_dev[dev]);
  return DPAR2_OK;
}

// the compressed representation of a single-tensor workspace
struct Comp {
  Group g;
  Layout y;
};
dpar2_status comp_of(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes, Comp* c) {
  dpar2_status st = make_group(1, X, o, &c->g);
  if (st != DPAR2_OK) return st;
  c->y = make_layout(c->g);
  return check_ws(c->y, ws, ws_bytes);
}

// PARAFAC2-ALS on the uncompressed slices (Alg. 2): a single-tensor group
// whose slab pass sketches with V (L = R), and the buffers of the iteration.
struct PlainLayout {
  Layout y;                 // tables, control block, item partials (L = R), xnorm2, small, red, ybuf
  size_t Y, theta, g1p, g2p, wp, g2, om_next, om_cur;
  size_t total;
};

dpar2_opts plain_opts(const dpar2_opts* o) {
  dpar2_opts q = *o;
  q.sketch = q.sketch2 = o->rank;
  q.power_iters = 0;
  q.flags = o->flags & DPAR2_FLAG_WIDE_SLAB;
  return q;
}

dpar2_status plain_group(const dpar2_tensor* X, const dpar2_opts* o, Group* g, dpar2_opts* q) {
  if (!X || !o) return fail(DPAR2_EINVAL, "tensor or options pointer is NULL");
  if (o->flags & ~(DPAR2_FLAG_NO_GRAPH | DPAR2_FLAG_WIDE_SLAB | DPAR2_FLAG_DETERMINISTIC))
    return fail(DPAR2_EINVAL, "unknown bits in opts.flags");
  *q = plain_opts(o);
  return make_group(1, X, q, g);
}

PlainLayout make_plain_layout(const Group& g) {
  PlainLayout p;
  p.y = make_layout(g);
  const int64_t K = p.y.K, J = p.y.J, R = p.y.R;
  const int64_t nvb = (K + PL_VSLICES - 1) / PL_VSLICES;
  size_t at = p.y.total;
  auto take = [&](size_t bytes) {
    const size_t r = at;
    at = align256(at + bytes);
    return r;
  };
  p.Y = take(sizeof(double) * (size_t)(K * R * J));
  p.theta = take(sizeof(double) * (size_t)(K * R * R));
  p.g1p = take(sizeof(double) * (size_t)(K * R * R));
  p.g2p = take(sizeof(double) * (size_t)(nvb * J * R));
  p.wp = take(sizeof(double) * (size_t)(K * (R * R + 2)));
  p.g2 = take(sizeof(double) * (size_t)(J * R));
  p.om_next = take(sizeof(float) * (size_t)(J * R));
  p.om_cur = take(sizeof(float) * (size_t)(J * R));
  p.total = at;
  return p;
}

PlainArgs plain_args(const PlainLayout& p, char* w, const dpar2_factors* f, double* trace, double tol) {
  const Layout& y = p.y;
  PlainArgs a;
  std::memset(&a, 0, sizeof(a));
  a.K = y.K;
  a.J = (int)y.J;
  a.slice_ptr = reinterpret_cast<const int32_t*>(w + y.slice_ptr);
  a.slice_list = reinterpret_cast<const int32_t*>(w + y.slice_list);
  a.partG = reinterpret_cast<const double*>(w + y.partG);
  a.partP = reinterpret_cast<const double*>(w + y.partP);
  a.partS = reinterpret_cast<const double*>(w + y.partS);
  a.xnorm2 = reinterpret_cast<double*>(w + y.xnorm2);
  a.H = f->H;
  a.V = f->V;
  a.W = f->W;
  a.trace = trace;
  a.tol = tol;
  a.Y = reinterpret_cast<double*>(w + p.Y);
  a.theta = reinterpret_cast<double*>(w + p.theta);
  a.g1p = reinterpret_cast<double*>(w + p.g1p);
  a.g2p = reinterpret_cast<double*>(w + p.g2p);
  a.wp = reinterpret_cast<double*>(w + p.wp);
  a.small = reinterpret_cast<double*>(w + y.small);
  a.red = reinterpret_cast<double*>(w + y.red);
  a.g2 = reinterpret_cast<double*>(w + p.g2);
  a.om_next = reinterpret_cast<float*>(w + p.om_next);
  a.om_cur = reinterpret_cast<float*>(w + p.om_cur);
  a.ctl = reinterpret_cast<Ctl*>(w + y.ctl);
  return a;
}

dpar2_status check_tokens(int32_t rank, int32_t n, const int32_t* off_dev, const int32_t* off_host) {
  if (rank < 1 || rank > 32) return fail(DPAR2_EINVAL, "rank must be in 1..32");
  if (n < 1) return fail(DPAR2_EINVAL, "n must be >= 1");
  if (!off_dev || !off_host) return fail(DPAR2_EINVAL, "token offsets must be non-NULL");
  if (off_host[0] != 0) return fail(DPAR2_EINVAL, "token offsets must start at 0");
  for (int32_t b = 0; b < n; ++b)
    if (off_host[b + 1] <= off_host[b]) return fail(DPAR2_EINVAL, "every tensor needs at least one token");
  return DPAR2_OK;
}
}  // namespace

extern "C" {

size_t dpar2_workspace_bytes(const dpar2_tensor* X, const dpar2_opts* o) {
  Group g;
  if (make_group(1, X, o, &g) != DPAR2_OK) return 0;
  return make_layout(g).total;
}

size_t dpar2_workspace_size(const dpar2_tensor* X, const dpar2_opts* o) { return dpar2_workspace_bytes(X, o); }

size_t dpar2_batch_workspace_size(int32_t n, const dpar2_tensor* X, const dpar2_opts* o) {
  Batch b;
  if (make_batch(n, X, o, &b) != DPAR2_OK) return 0;
  return b.total;
}

dpar2_status dpar2_compress(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                            const float* omega2, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  return group_compress(g, &omega1, &omega2, nullptr, static_cast<char*>(ws), y,
                        reinterpret_cast<hipStream_t>(stream));
}

dpar2_status dpar2_als_step(const dpar2_tensor* X, const dpar2_opts* o, dpar2_factors* f, int32_t n_steps,
                            double* err_trace, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!f) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  if (n_steps < 0) return fail(DPAR2_EINVAL, "n_steps must be >= 0");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if ((st = group_factors(g, f, &err_trace, w, y, s)) != DPAR2_OK) return st;
  return group_als(g, n_steps, w, y, s);
}

dpar2_status dpar2_fitness(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f, double* fit,
                           void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!f) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  double* none = nullptr;
  if ((st = group_factors(g, f, &none, w, y, s)) != DPAR2_OK) return st;
  hipError_t e = launch_fitness(y, w, fit, s);
  if (e != hipSuccess) return hip_fail(e, "fitness");
  return DPAR2_OK;
}

dpar2_status dpar2_output_U(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f, double* U,
                            void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !U) return fail(DPAR2_EINVAL, "H and U must be non-NULL");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  // the descriptor's Omega_1 is the workspace copy taken by dpar2_compress
  const float* om1 = reinterpret_cast<const float*>(w + y.om1);
  if ((st = upload_descriptors(w, y, descriptors(g, &om1, &om1, f, nullptr), s)) != DPAR2_OK) return st;
  return group_output_U(g, y, w, f->H, U, s);
}

dpar2_status dpar2_output_A(const dpar2_tensor* X, const dpar2_opts* o, double* A, void* ws, size_t ws_bytes,
                            dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!A) return fail(DPAR2_EINVAL, "A must be non-NULL");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const float* om1 = reinterpret_cast<const float*>(w + y.om1);
  if ((st = upload_descriptors(w, y, descriptors(g, &om1, &om1, nullptr, nullptr), s)) != DPAR2_OK) return st;
  return group_output_U(g, y, w, nullptr, A, s);
}

namespace {
// Alg. 3 after the compression: the iteration, the true fitness, U_k (when U
// is given) and the report (when rep is given; ENOCONV when a tolerance was
// set and the stop rule never fired).
dpar2_status decompose_tail(const Group& g, const dpar2_opts* o, const dpar2_factors* f, double* U,
                            dpar2_report* rep, char* w, const Layout& y, hipStream_t s) {
  dpar2_status st;
  if ((st = group_als(g, o->max_iter, w, y, s)) != DPAR2_OK) return st;
  hipError_t e = launch_fitness(y, w, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "fitness");
  if (U && (st = group_output_U(g, y, w, f->H, U, s)) != DPAR2_OK) return st;
  if (!rep) return DPAR2_OK;
  if ((st = group_report(g, w, y, rep, s)) != DPAR2_OK) return st;
  if (o->tol >= 0.0 && !rep->converged)
    return fail(DPAR2_ENOCONV, "the stop rule did not fire within " + std::to_string(o->max_iter) + " iterations");
  return DPAR2_OK;
}
}  // namespace

dpar2_status dpar2_decompose(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                             const float* omega2, dpar2_factors* f, double* U, dpar2_report* rep, void* ws,
                             size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  // one upload: the descriptors carry Omega, the factors and (NULL) trace
  if ((st = group_compress(g, &omega1, &omega2, f, w, y, s)) != DPAR2_OK) return st;
  return decompose_tail(g, o, f, U, rep, w, y, s);
}

dpar2_status dpar2_decompose_noalloc(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                     const float* omega2, dpar2_factors* f, double* U, dpar2_report* rep,
                                     dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  g.noalloc = true;
  const Layout y = make_layout(g);
  if (y.total > NOALLOC_BYTES)
    return fail(DPAR2_EWORKSPACE, "dpar2_decompose_noalloc: this decomposition needs " + std::to_string(y.total) +
                                      " bytes of workspace; the static scratch holds " +
                                      std::to_string(NOALLOC_BYTES));
  if (y.tables_end - y.tdesc > NOALLOC_TABLE_BYTES)
    return fail(DPAR2_EWORKSPACE, "dpar2_decompose_noalloc: the schedule tables need " +
                                      std::to_string(y.tables_end - y.tdesc) + " bytes, above the limit of " +
                                      std::to_string(NOALLOC_TABLE_BYTES));
  char* w = nullptr;
  if ((st = scratch_address(&w)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((st = group_compress(g, &omega1, &omega2, f, w, y, s)) != DPAR2_OK) return st;
  return decompose_tail(g, o, f, U, rep, w, y, s);
}

// --- streaming: slices appended to a decomposed tensor ----------------------

namespace {
// The tensor of an append in three views: all K slices, its first k_prev
// slices (decomposed by an earlier call), and the appended slices as a tensor
// of their own (host row offsets rebased to 0, slab and fp8 scales advanced to
// its first row and slice).
struct AppendPlan {
  std::vector<int64_t> off_add;
  dpar2_tensor Xp, Xa;
  dpar2_opts oa;
  Group all, prev, add;
  Layout y_all, y_prev, y_add;
  size_t total = 0;   // y_all.total + y_add.total
};

dpar2_status append_plan(const dpar2_tensor* X, int64_t k_prev, const dpar2_opts* o, AppendPlan* p) {
  dpar2_status st = make_group(1, X, o, &p->all);
  if (st != DPAR2_OK) return st;
  if (k_prev < 1 || k_prev >= X->K) return fail(DPAR2_EINVAL, "k_prev must be in [1, K - 1]");
  const int64_t* off = X->row_offsets_host;
  const int esize = X->dtype == DPAR2_F32 ? 4 : (X->dtype == DPAR2_BF16 ? 2 : 1);
  p->Xp = *X;
  p->Xp.K = k_prev;
  p->off_add.assign(off + k_prev, off + X->K + 1);
  for (int64_t& v : p->off_add) v -= off[k_prev];
  p->Xa = *X;
  p->Xa.K = X->K - k_prev;
  p->Xa.row_offsets_host = p->off_add.data();
  // the device offsets are not rebased: the first stage reads the host table
  // only (row ranges of the work items)
  p->Xa.row_offsets = X->row_offsets + k_prev;
  p->Xa.slab = static_cast<const char*>(X->slab) + (size_t)off[k_prev] * (size_t)X->J * (size_t)esize;
  p->Xa.slice_scale = X->slice_scale ? X->slice_scale + k_prev : nullptr;
  if ((st = make_group(1, &p->Xp, o, &p->prev)) != DPAR2_OK) return st;
  // the appended slices never run a second stage of their own: L2 <= K R
  // need not hold for them alone
  p->oa = *o;
  p->oa.sketch2 = (int32_t)std::min<int64_t>(o->sketch2, p->Xa.K * o->rank);
  if ((st = make_group(1, &p->Xa, &p->oa, &p->add)) != DPAR2_OK) return st;
  p->y_all = make_layout(p->all);
  p->y_prev = make_layout(p->prev);
  p->y_add = make_layout(p->add);
  p->total = p->y_all.total + p->y_add.total;
  return DPAR2_OK;
}

// Per-slice results of the first stage (||X_k||^2, the rows of M^T, the A_k
// recipe Phi_k, the singular values, the power step's sketch matrices) of n
// slices from src (layout ys, from its slice 0) to dst (layout yd, from slice
// k_dst).
hipError_t copy_first_stage(const char* src, const Layout& ys, char* dst, const Layout& yd, int64_t k_dst, int64_t n,
                            hipStream_t s) {
  const size_t J = (size_t)yd.J, R = (size_t)yd.R, L = (size_t)yd.L;
  const size_t per[5] = {sizeof(double), sizeof(double) * R * J, sizeof(double) * L * R, sizeof(double) * R,
                         yd.q > 0 ? sizeof(float) * J * L : 0};
  const size_t from[5] = {ys.xnorm2, ys.Mt, ys.Phi, ys.sig1, ys.omq};
  const size_t to[5] = {yd.xnorm2, yd.Mt, yd.Phi, yd.sig1, yd.omq};
  for (int i = 0; i < 5; ++i) {
    if (!per[i]) continue;
    const hipError_t e = hipMemcpyAsync(dst + to[i] + (size_t)k_dst * per[i], src + from[i], (size_t)n * per[i],
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Warning bits of the earlier decomposition and of the appended slices' first
// stage into the grown tensor's control block.
__global__ void k_merge_warn(Ctl* __restrict__ dst, const Ctl* __restrict__ a, const Ctl* __restrict__ b) {
  if (threadIdx.x == 0) dst->warn |= a->warn | b->warn;
}

std::mutex g_sub_mu;
std::unordered_map<const void*, const void*> g_sub;   // append workspace -> its second part
}  // namespace

size_t dpar2_append_workspace_bytes(const dpar2_tensor* X, int64_t k_prev, const dpar2_opts* o) {
  AppendPlan p;
  if (append_plan(X, k_prev, o, &p) != DPAR2_OK) return 0;
  return p.total;
}

dpar2_status dpar2_append(const dpar2_tensor* X, int64_t k_prev, const dpar2_opts* o, const float* omega1,
                          const float* omega2, const void* ws_prev, size_t ws_prev_bytes, dpar2_factors* f,
                          double* U, dpar2_report* rep, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  AppendPlan p;
  dpar2_status st = append_plan(X, k_prev, o, &p);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  if (!omega1 || !omega2) return fail(DPAR2_EINVAL, "omega1 and omega2 must be non-NULL");
  if ((st = check_ws(p.y_prev, ws_prev, ws_prev_bytes)) != DPAR2_OK) {
    g_last_error = "ws_prev: " + g_last_error;
    return st;
  }
  if (!ws) return fail(DPAR2_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(DPAR2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < p.total)
    return fail(DPAR2_EWORKSPACE, "workspace too small: need " + std::to_string(p.total) + " bytes");
  const uintptr_t a0 = (uintptr_t)ws, a1 = a0 + p.total, b0 = (uintptr_t)ws_prev, b1 = b0 + p.y_prev.total;
  if (a0 < b1 && b0 < a1) return fail(DPAR2_EINVAL, "ws and ws_prev overlap");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  char* wa = w + p.y_all.total;
  {
    std::lock_guard<std::mutex> lk(g_sub_mu);
    g_sub[ws] = wa;
  }
  // first stage of the appended slices, in the second part of the workspace
  if ((st = group_compress(p.add, &omega1, &omega2, nullptr, wa, p.y_add, s, CP_FIRST)) != DPAR2_OK) return st;
  // tables, descriptors and control block of the grown tensor, then the
  // per-slice results of both parts in slice order
  if ((st = group_compress(p.all, &omega1, &omega2, f, w, p.y_all, s, 0)) != DPAR2_OK) return st;
  hipError_t e = copy_first_stage(static_cast<const char*>(ws_prev), p.y_prev, w, p.y_all, 0, k_prev, s);
  if (e == hipSuccess) e = copy_first_stage(wa, p.y_add, w, p.y_all, k_prev, X->K - k_prev, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  hipLaunchKernelGGL(k_merge_warn, dim3(1), dim3(64), 0, s, reinterpret_cast<Ctl*>(w + p.y_all.ctl),
                     reinterpret_cast<const Ctl*>(static_cast<const char*>(ws_prev) + p.y_prev.ctl),
                     reinterpret_cast<const Ctl*>(wa + p.y_add.ctl));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "append set-up");
  // second stage over the whole M, then Alg. 3 as in dpar2_decompose
  if ((e = launch_stage2(p.y_all, w, s)) != hipSuccess) return hip_fail(e, "second stage");
  if ((e = launch_pw_identity(p.y_all, w, s)) != hipSuccess) return hip_fail(e, "iteration state init");
  return decompose_tail(p.all, o, f, U, rep, w, p.y_all, s);
}

dpar2_status dpar2_decompose_batch(int32_t n, const dpar2_tensor* X, const dpar2_opts* o,
                                   const float* const* omega1, const float* const* omega2, dpar2_factors* f,
                                   void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Batch b;
  dpar2_status st = make_batch(n, X, o, &b);
  if (st != DPAR2_OK) return st;
  if (!omega1 || !omega2 || !f) return fail(DPAR2_EINVAL, "omega and factor arrays must be non-NULL");
  for (int32_t t = 0; t < n; ++t)
    if (!f[t].H || !f[t].V || !f[t].W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  if (!ws) return fail(DPAR2_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(DPAR2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < b.total)
    return fail(DPAR2_EWORKSPACE, "workspace too small: need " + std::to_string(b.total) + " bytes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto run_group = [&](size_t gi, hipStream_t gs) -> dpar2_status {
    const Group& g = b.groups[gi];
    const Layout& y = b.lay[gi];
    char* w = static_cast<char*>(ws) + b.base[gi];
    std::vector<const float*> o1, o2;
    std::vector<dpar2_factors> fg;
    for (int t : g.orig) {
      o1.push_back(omega1[t]);
      o2.push_back(omega2[t]);
      fg.push_back(f[t]);
    }
    dpar2_status r = group_compress(g, o1.data(), o2.data(), fg.data(), w, y, gs);
    if (r == DPAR2_OK) r = group_als(g, g.o[0].max_iter, w, y, gs);
    if (r == DPAR2_OK) {
      const hipError_t e = launch_fitness(y, w, nullptr, gs);
      if (e != hipSuccess) r = hip_fail(e, "fitness");
    }
    return r;
  };
  if (b.groups.size() == 1) return run_group(0, s);
  // several groups: each on a stream of the pool, forked from and joined
  // back into the caller's stream
  std::lock_guard<std::mutex> lk(g_spool.mu);
  if ((st = pool_ready_locked()) != DPAR2_OK) return st;
  const int used = (int)std::min<size_t>(b.groups.size(), BATCH_STREAMS);
  hipError_t e;
  if ((e = hipEventRecord(g_spool.fork, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  for (int i = 0; i < used; ++i)
    if ((e = hipStreamWaitEvent(g_spool.s[i], g_spool.fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  for (size_t gi = 0; gi < b.groups.size() && st == DPAR2_OK; ++gi) st = run_group(gi, g_spool.s[gi % BATCH_STREAMS]);
  for (int i = 0; i < used; ++i) {
    if ((e = hipEventRecord(g_spool.done[i], g_spool.s[i])) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(s, g_spool.done[i], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  return st;
}

dpar2_status dpar2_batch_report_read(int32_t n, const dpar2_tensor* X, const dpar2_opts* o, const void* ws,
                                     dpar2_report* rep, dpar2_stream_t stream) {
  Batch b;
  dpar2_status st = make_batch(n, X, o, &b);
  if (st != DPAR2_OK) return st;
  if (!rep || !ws) return fail(DPAR2_EINVAL, "report and workspace must be non-NULL");
  dpar2_status worst = DPAR2_OK;
  std::string msg;
  for (size_t gi = 0; gi < b.groups.size(); ++gi) {
    const Group& g = b.groups[gi];
    std::vector<dpar2_report> r((size_t)g.nt);
    st = group_report(g, static_cast<const char*>(ws) + b.base[gi], b.lay[gi], r.data(),
                      reinterpret_cast<hipStream_t>(stream));
    if (st == DPAR2_ENUMERIC) {   // reports filled; keep going
      if (worst == DPAR2_OK) msg = g_last_error;
      worst = st;
    } else if (st != DPAR2_OK) {
      return st;
    }
    for (int t = 0; t < g.nt; ++t) rep[g.orig[(size_t)t]] = r[(size_t)t];
  }
  if (worst != DPAR2_OK) return fail(worst, msg);
  return DPAR2_OK;
}

dpar2_status dpar2_report_read(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, dpar2_report* rep,
                               dpar2_stream_t stream) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!rep || !ws) return fail(DPAR2_EINVAL, "report and workspace must be non-NULL");
  return group_report(g, ws, make_layout(g), rep, reinterpret_cast<hipStream_t>(stream));
}

dpar2_status dpar2_compressed_view(const dpar2_tensor* X, const dpar2_opts* o, const void* ws,
                                   size_t ws_bytes, dpar2_compressed* out) {
  Group g;
  dpar2_status st = make_group(1, X, o, &g);
  if (st != DPAR2_OK) return st;
  if (!out) return fail(DPAR2_EINVAL, "out is NULL");
  const Layout y = make_layout(g);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  const char* w = static_cast<const char*>(ws);
  out->Mt = reinterpret_cast<const double*>(w + y.Mt);
  out->D = reinterpret_cast<const double*>(w + y.D);
  out->E = reinterpret_cast<const double*>(w + y.E);
  out->F = reinterpret_cast<const double*>(w + y.F);
  out->Phi = reinterpret_cast<const double*>(w + y.Phi);
  out->sigma = reinterpret_cast<const double*>(w + y.sig1);
  out->xnorm2 = reinterpret_cast<const double*>(w + y.xnorm2);
  return DPAR2_OK;
}

// --- PARAFAC2-ALS on the uncompressed slices (Alg. 2) ----------------------

size_t dpar2_plain_workspace_bytes(const dpar2_tensor* X, const dpar2_opts* o) {
  Group g;
  dpar2_opts q;
  if (plain_group(X, o, &g, &q) != DPAR2_OK) return 0;
  return make_plain_layout(g).total;
}

dpar2_status dpar2_als_plain(const dpar2_tensor* X, const dpar2_opts* o, dpar2_factors* f, double* err_trace,
                             double* U, dpar2_report* rep, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  Group g;
  dpar2_opts q;
  dpar2_status st = plain_group(X, o, &g, &q);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  const PlainLayout p = make_plain_layout(g);
  if (!ws) return fail(DPAR2_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(DPAR2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < p.total) return fail(DPAR2_EWORKSPACE, "workspace too small: need " + std::to_string(p.total) + " bytes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const Layout& y = p.y;
  // descriptor (the slab pass sketches with the float32 copy of V) and the
  // schedule tables: one upload
  float* om_cur = reinterpret_cast<float*>(w + p.om_cur);
  const float* om = om_cur;
  {
    const std::vector<TDesc> td = descriptors(g, &om, &om, f, &err_trace);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging& sg = g_stage[w];
    stage_tables(g, y, sg);
    std::memcpy(sg.image.data(), td.data(), sizeof(TDesc) * td.size());
    if ((st = upload_locked(sg, w, sg.image.data(), sg.image.size(), y.tdesc, s)) != DPAR2_OK) return st;
  }
  const PlainArgs a = plain_args(p, w, f, err_trace, o->tol);
  const int dtype = X->dtype;
  const int esize = dtype == DPAR2_F32 ? 4 : (dtype == DPAR2_BF16 ? 2 : 1);
  PlainLaunch pl;
  std::memset(&pl, 0, sizeof(pl));
  pl.slab.td = reinterpret_cast<const TDesc*>(w + y.tdesc);
  pl.slab.J = (int)y.J;
  pl.slab.L = y.R;
  pl.slab.R = y.R;
  pl.slab.items = reinterpret_cast<const Item*>(w + y.items);
  pl.slab.partG = reinterpret_cast<double*>(w + y.partG);
  pl.slab.partP = reinterpret_cast<double*>(w + y.partP);
  pl.slab.partS = reinterpret_cast<double*>(w + y.partS);
  pl.slab.ybuf = reinterpret_cast<float*>(w + y.ybuf);
  pl.slab.skip = &reinterpret_cast<const Ctl*>(w + y.ctl)->done;
  pl.dtype = dtype;
  pl.n_items = y.n_items;
  pl.vec = (y.J % 4 == 0) && ((uintptr_t)X->slab % (4 * esize) == 0);
  pl.wide = y.wide;
  hipError_t e = launch_plain(0, y.R, a, pl, s);
  for (int32_t i = 0; e == hipSuccess && i < o->max_iter; ++i) e = launch_plain(1, y.R, a, pl, s);
  if (e != hipSuccess) return hip_fail(e, "plain ALS iteration");
  if (U) {
    // U_k = Q_k H = (X_k V) Theta_k H, V of the last slab pass that ran
    if ((e = launch_plain(2, y.R, a, pl, s)) != hipSuccess) return hip_fail(e, "plain ALS theta");
    SlabArgs sa = pl.slab;
    sa.skip = nullptr;
    sa.partG = sa.partP = sa.partS = nullptr;
    sa.theta = reinterpret_cast<const double*>(w + p.theta);
    sa.U = U;
    if ((e = launch_slab(sa, dtype, y.n_items, pl.vec, true, y.wide, s)) != hipSuccess) return hip_fail(e, "U pass");
  }
  if (!rep) return DPAR2_OK;
  if ((st = group_report(g, w, y, rep, s)) != DPAR2_OK) return st;
  rep->fit_compressed = rep->fit_true;
  if (o->tol >= 0.0 && !rep->converged)
    return fail(DPAR2_ENOCONV, "the stop rule did not fire within " + std::to_string(o->max_iter) + " iterations");
  return DPAR2_OK;
}

// --- post-processing of the factors (Sec. IV-E) -----------------------------

dpar2_status dpar2_feature_pcc(int64_t J, int32_t R, const double* V, double* C, dpar2_stream_t stream) {
  if (J < 1 || J > ((int64_t)1 << 20)) return fail(DPAR2_EINVAL, "J must be in 1..2^20");
  if (!rank_supported(R)) return fail(DPAR2_EINVAL, "R must be in 1..32 or one of 40, 50");
  if (!V || !C) return fail(DPAR2_EINVAL, "V and C must be non-NULL");
  const hipError_t e = launch_pcc(J, R, V, C, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "feature pcc");
}

dpar2_status dpar2_slice_similarity(const dpar2_tensor* X, int32_t R, const double* U, int32_t n, const int32_t* idx,
                                    const int32_t* idx_host, double gamma, double* S, dpar2_stream_t stream) {
  if (!X || !X->row_offsets || !X->row_offsets_host) return fail(DPAR2_EINVAL, "tensor and row offsets must be non-NULL");
  if (!rank_supported(R)) return fail(DPAR2_EINVAL, "R must be in 1..32 or one of 40, 50");
  if (n < 1 || n > (1 << 20)) return fail(DPAR2_EINVAL, "n must be in 1..2^20");
  if (!U || !idx || !idx_host || !S) return fail(DPAR2_EINVAL, "U, idx and S must be non-NULL");
  if (!(gamma >= 0.0)) return fail(DPAR2_EINVAL, "gamma must be >= 0");
  const int64_t* off = X->row_offsets_host;
  int64_t rows = -1;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t k = idx_host[i];
    if (k < 0 || k >= X->K) return fail(DPAR2_EINVAL, "slice index " + std::to_string(k) + " out of range");
    const int64_t r = off[k + 1] - off[k];
    if (rows < 0) rows = r;
    if (r != rows)
      return fail(DPAR2_ESHAPE, "the similarity of Eq. 9 needs slices of one length (slice " + std::to_string(k) +
                                    " has " + std::to_string(r) + " rows, not " + std::to_string(rows) + ")");
  }
  const hipError_t e = launch_similarity(n, rows * R, R, X->row_offsets, idx, U, gamma, S,
                                         reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "slice similarity");
}

dpar2_status dpar2_top_k(const double* v, int32_t n, int32_t exclude, int32_t k, int32_t* out,
                         dpar2_stream_t stream) {
  if (!v || !out) return fail(DPAR2_EINVAL, "v and out must be non-NULL");
  if (n < 1) return fail(DPAR2_EINVAL, "n must be >= 1");
  const int32_t avail = n - ((exclude >= 0 && exclude < n) ? 1 : 0);
  if (k < 1 || k > avail) return fail(DPAR2_EINVAL, "k must be in 1.." + std::to_string(avail));
  const hipError_t e = launch_topk(v, n, exclude, k, out, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "top k");
}

dpar2_status dpar2_rwr(const double* S, int32_t n, int32_t target, double c, int32_t iters, double* r, double* work,
                       dpar2_stream_t stream) {
  if (!S || !r || !work) return fail(DPAR2_EINVAL, "S, r and work must be non-NULL");
  if (n < 1 || n > (1 << 20)) return fail(DPAR2_EINVAL, "n must be in 1..2^20");
  if (target < 0 || target >= n) return fail(DPAR2_EINVAL, "target out of range");
  if (!(c > 0.0 && c <= 1.0)) return fail(DPAR2_EINVAL, "the restart probability c must be in (0, 1]");
  if (iters < 0) return fail(DPAR2_EINVAL, "iters must be >= 0");
  const hipError_t e = launch_rwr(S, n, target, c, iters, r, work, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "rwr");
}

// --- learned warm start ------------------------------------------------------

int64_t dpar2_warm_param_count(int32_t rank) {
  if (rank < 1 || rank > 32) return 0;
  return warm_layout(rank).P;
}


dpar2_status dpar2_warm_features(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                                 float* tok, dpar2_stream_t stream) {
  Comp c;
  if (o && o->rank > 32) return fail(DPAR2_EINVAL, "the warm start takes ranks up to 32");
  dpar2_status st = comp_of(X, o, ws, ws_bytes, &c);
  if (st != DPAR2_OK) return st;
  if (!tok) return fail(DPAR2_EINVAL, "tok is NULL");
  const char* w = static_cast<const char*>(ws);
  hipError_t e = launch_warm_feat(c.y.K, (int)c.y.J, c.y.R, reinterpret_cast<const double*>(w + c.y.F),
                                  reinterpret_cast<const double*>(w + c.y.E),
                                  reinterpret_cast<const double*>(w + c.y.D), tok,
                                  reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm features");
}

dpar2_status dpar2_warm_targets(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                                const dpar2_factors* f, float* tH, float* tV, float* tW, dpar2_stream_t stream) {
  Comp c;
  if (o && o->rank > 32) return fail(DPAR2_EINVAL, "the warm start takes ranks up to 32");
  dpar2_status st = comp_of(X, o, ws, ws_bytes, &c);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W || !tH || !tV || !tW) return fail(DPAR2_EINVAL, "NULL factor or target");
  const char* w = static_cast<const char*>(ws);
  hipError_t e = launch_warm_targets(c.y.K, (int)c.y.J, c.y.R, reinterpret_cast<const double*>(w + c.y.D),
                                     reinterpret_cast<const double*>(w + c.y.E), f->H, f->V, f->W, tH, tV, tW,
                                     reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm targets");
}

dpar2_status dpar2_warm_apply(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                              const float* pH, const float* pV, const float* pW, dpar2_factors* f,
                              dpar2_stream_t stream) {
  Comp c;
  if (o && o->rank > 32) return fail(DPAR2_EINVAL, "the warm start takes ranks up to 32");
  dpar2_status st = comp_of(X, o, ws, ws_bytes, &c);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W || !pH || !pV || !pW) return fail(DPAR2_EINVAL, "NULL factor or prediction");
  const char* w = static_cast<const char*>(ws);
  hipError_t e = launch_warm_apply(c.y.K, (int)c.y.J, c.y.R, reinterpret_cast<const double*>(w + c.y.D),
                                   reinterpret_cast<const double*>(w + c.y.E), pH, pV, pW, f->H, f->V, f->W,
                                   reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm apply");
}

dpar2_status dpar2_warm_forward(int32_t rank, int32_t n, const int32_t* tok_off, const int32_t* tok_off_host,
                                const float* tok, const float* theta, float* act, float* pH, float* pV, float* pW,
                                dpar2_stream_t stream) {
  dpar2_status st = check_tokens(rank, n, tok_off, tok_off_host);
  if (st != DPAR2_OK) return st;
  if (!tok || !theta || !act || !pH || !pV || !pW) return fail(DPAR2_EINVAL, "NULL buffer");
  hipError_t e = launch_warm_forward(rank, n, tok_off, tok, theta, act, pH, pV, pW,
                                     reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm forward");
}

dpar2_status dpar2_warm_backward(int32_t rank, int32_t n, const int32_t* tok_off, const int32_t* tok_off_host,
                                 const float* tok, const float* theta, float* act, const float* pH, const float* pV,
                                 const float* pW, const float* tH, const float* tV, const float* tW,
                                 float* grad_part, float* grad, float* loss, dpar2_stream_t stream) {
  dpar2_status st = check_tokens(rank, n, tok_off, tok_off_host);
  if (st != DPAR2_OK) return st;
  if (!tok || !theta || !act || !pH || !pV || !pW || !tH || !tV || !tW || !grad_part || !grad || !loss)
    return fail(DPAR2_EINVAL, "NULL buffer");
  hipError_t e = launch_warm_backward(rank, n, tok_off, tok, theta, act, pH, pV, pW, tH, tV, tW, grad_part, grad,
                                      loss, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm backward");
}

dpar2_status dpar2_warm_adam(int32_t rank, float* theta, const float* grad, float* m, float* v, int32_t step,
                             float lr, float beta1, float beta2, float eps, float grad_scale,
                             dpar2_stream_t stream) {
  if (rank < 1 || rank > 32) return fail(DPAR2_EINVAL, "rank must be in 1..32");
  if (!theta || !grad || !m || !v) return fail(DPAR2_EINVAL, "NULL buffer");
  if (step < 1) return fail(DPAR2_EINVAL, "step counts from 1");
  hipError_t e = launch_warm_adam(rank, theta, grad, m, v, step, lr, beta1, beta2, eps, grad_scale,
                                  reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DPAR2_OK : hip_fail(e, "warm adam");
}

// Times the first stage's slab pass for each candidate (work-item size,
// whole-row or 128-column-chunk pass); *best = index of the fastest.
static dpar2_status autotune_slab_impl(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                       const int32_t* cands, const int32_t* wide, int32_t n_cands, void* ws,
                                       size_t ws_bytes, int32_t* best, float* times_ms, dpar2_stream_t stream) {
  if (!o || !cands || n_cands < 1 || !best || !omega1) return fail(DPAR2_EINVAL, "NULL argument or no candidates");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  dpar2_status st = DPAR2_OK;
  float best_ms = 0.f;
  for (int32_t c = 0; c < n_cands && st == DPAR2_OK; ++c) {
    dpar2_opts oc = *o;
    oc.item_rows = cands[c];
    oc.power_iters = 0;
    oc.flags = (o->flags & ~DPAR2_FLAG_WIDE_SLAB) | ((wide && wide[c]) ? DPAR2_FLAG_WIDE_SLAB : 0u);
    Group g;
    if ((st = make_group(1, X, &oc, &g)) != DPAR2_OK) break;
    const Layout y = make_layout(g);
    if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) break;
    // the first stage's set-up and slab pass, as in group_compress
    const std::vector<TDesc> td = descriptors(g, &omega1, &omega1, nullptr, nullptr);
    {
      std::lock_guard<std::mutex> lk(g_stage_mu);
      Staging& sg = g_stage[w];
      stage_tables(g, y, sg);
      std::memcpy(sg.image.data(), td.data(), sizeof(TDesc) * td.size());
      if ((st = upload_locked(sg, w, sg.image.data(), sg.image.size(), y.tdesc, s)) != DPAR2_OK) break;
    }
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(256), 0, s, reinterpret_cast<const TDesc*>(w + y.tdesc),
                       (int)(y.J * y.L), reinterpret_cast<Ctl*>(w + y.ctl), reinterpret_cast<float*>(w + y.om1));
    const int esize = X->dtype == DPAR2_F32 ? 4 : (X->dtype == DPAR2_BF16 ? 2 : 1);
    SlabArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.td = reinterpret_cast<const TDesc*>(w + y.tdesc);
    sa.J = (int)y.J;
    sa.L = y.L;
    sa.R = y.R;
    sa.items = reinterpret_cast<const Item*>(w + y.items);
    sa.partG = reinterpret_cast<double*>(w + y.partG);
    sa.partP = reinterpret_cast<double*>(w + y.partP);
    sa.partS = reinterpret_cast<double*>(w + y.partS);
    sa.ybuf = reinterpret_cast<float*>(w + y.ybuf);
    const bool vec = (y.J % 4 == 0) && ((uintptr_t)X->slab % (4 * esize) == 0);
    float t[4];
    for (int r = 0; r < 4 && st == DPAR2_OK; ++r) {   // one warm-up launch, three timed
      if ((e = hipEventRecord(e0, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
      else if ((e = launch_slab(sa, X->dtype, y.n_items, vec, false, y.wide, s)) != hipSuccess) st = hip_fail(e, "slab pass");
      else if ((e = hipEventRecord(e1, s)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
      else if ((e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
      else if ((e = hipEventElapsedTime(&t[r], e0, e1)) != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
    }
    if (st != DPAR2_OK) break;
    std::sort(t + 1, t + 4);
    if (times_ms) times_ms[c] = t[2];
    if (c == 0 || t[2] < best_ms) {
      best_ms = t[2];
      *best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

dpar2_status dpar2_autotune_item_rows(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                      const int32_t* cands, int32_t n_cands, void* ws, size_t ws_bytes,
                                      int32_t* best, float* times_ms, dpar2_stream_t stream) {
  int32_t idx = 0;
  const dpar2_status st =
      autotune_slab_impl(X, o, omega1, cands, nullptr, n_cands, ws, ws_bytes, &idx, times_ms, stream);
  if (st == DPAR2_OK) *best = cands[idx];
  return st;
}

dpar2_status dpar2_autotune_slab(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                 const int32_t* item_rows, const int32_t* wide, int32_t n_cands, void* ws,
                                 size_t ws_bytes, int32_t* best, float* times_ms, dpar2_stream_t stream) {
  if (!wide) return fail(DPAR2_EINVAL, "wide must be non-NULL");
  return autotune_slab_impl(X, o, omega1, item_rows, wide, n_cands, ws, ws_bytes, best, times_ms, stream);
}

dpar2_status dpar2_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.on = on != 0;
  return DPAR2_OK;
}

dpar2_status dpar2_profile_read(int32_t* launches, double* total_ms) {
  if (!launches || !total_ms) return fail(DPAR2_EINVAL, "launches and total_ms must be non-NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  for (size_t i = 0; i < g_prof.used; ++i) {
    hipError_t e = hipEventSynchronize(g_prof.pool[i].second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, g_prof.pool[i].first, g_prof.pool[i].second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    tot += ms;
  }
  *launches = (int32_t)g_prof.used;
  *total_ms = tot;
  g_prof.used = 0;
  return DPAR2_OK;
}

namespace {
dpar2_status release_one(const void* ws);
}

dpar2_status dpar2_release(const void* ws) {
  const void* sub = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_sub_mu);
    auto it = g_sub.find(ws);
    if (it != g_sub.end()) {
      sub = it->second;
      g_sub.erase(it);
    }
  }
  const dpar2_status st = release_one(ws);
  const dpar2_status st2 = sub ? release_one(sub) : DPAR2_OK;
  return st != DPAR2_OK ? st : st2;
}

namespace {
dpar2_status release_one(const void* ws) {
  hipError_t first = hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    auto it = g_stage.find(ws);
    if (it != g_stage.end()) {
      Staging& sg = it->second;
      for (int i = 0; i < STAGE_SLOTS; ++i) {
        if (sg.done[i]) {
          const hipError_t e = hipEventSynchronize(sg.done[i]);
          if (first == hipSuccess) first = e;
          (void)hipEventDestroy(sg.done[i]);
        }
        if (sg.host[i]) (void)hipHostFree(sg.host[i]);
      }
      g_stage.erase(it);
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(ws);
    if (it != g_graphs.end()) {
      for (GraphEntry& ge : it->second.entries) (void)hipGraphExecDestroy(ge.exec);
      if (it->second.cap) (void)hipStreamDestroy(it->second.cap);
      g_graphs.erase(it);
    }
  }
  if (first != hipSuccess) return hip_fail(first, "dpar2_release");
  return DPAR2_OK;
}
}  // namespace

dpar2_status dpar2_release_all(void) {
  std::vector<const void*> keys;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto& kv : g_stage) keys.push_back(kv.first);
  }
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& kv : g_graphs) keys.push_back(kv.first);
  }
  dpar2_status st = DPAR2_OK;
  for (const void* k : keys) {
    const dpar2_status r = dpar2_release(k);
    if (st == DPAR2_OK) st = r;
  }
  std::lock_guard<std::mutex> lk(g_spool.mu);
  if (g_spool.ready) {
    for (int i = 0; i < BATCH_STREAMS; ++i) {
      (void)hipStreamSynchronize(g_spool.s[i]);
      (void)hipStreamDestroy(g_spool.s[i]);
      (void)hipEventDestroy(g_spool.done[i]);
    }
    (void)hipEventDestroy(g_spool.fork);
    g_spool.ready = false;
  }
  return st;
}

const char* dpar2_status_string(int32_t status) {
  switch (status) {
    case DPAR2_OK: return "ok";
    case DPAR2_EINVAL: return "invalid argument";
    case DPAR2_ESHAPE: return "shape not supported";
    case DPAR2_ENUMERIC: return "the slab holds NaN or Inf";
    case DPAR2_ENOCONV: return "the stop rule did not fire within max_iter";
    case DPAR2_EHIP: return "HIP runtime error";
    case DPAR2_EWORKSPACE: return "workspace missing, misaligned or too small";
    default: return "unknown status";
  }
}

const char* dpar2_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
