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

// Host-side schedule of the slab pass.
struct Schedule {
  std::vector<Item> items;          // longest first
  std::vector<int32_t> slice_ptr;   // K+1
  std::vector<int32_t> slice_list;  // item indices of each slice
};

// Alg. 4 on the GPU: slices longer than MAX_CHUNK_ROWS are cut into near-equal
// row ranges; all items are sorted by length, longest first (stable), and
// block b of the slab pass takes item b.  The hardware dispatcher starts each
// next block on the first compute unit that frees up, i.e. greedy list
// scheduling of the longest remaining item on the least-loaded unit.
void build_schedule(const int64_t* off, int64_t K, Schedule* s) {
  std::vector<Item> raw;
  raw.reserve((size_t)K);
  for (int64_t k = 0; k < K; ++k) {
    const int64_t n = off[k + 1] - off[k];
    const int64_t nc = std::max<int64_t>(1, (n + MAX_CHUNK_ROWS - 1) / MAX_CHUNK_ROWS);
    for (int64_t c = 0; c < nc; ++c) {
      Item it;
      it.row0 = off[k] + n * c / nc;
      it.row1 = off[k] + n * (c + 1) / nc;
      it.slice = (int32_t)k;
      it.pad = 0;
      raw.push_back(it);
    }
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
}

int64_t count_items(const int64_t* off, int64_t K) {
  int64_t n = 0;
  for (int64_t k = 0; k < K; ++k) {
    const int64_t r = off[k + 1] - off[k];
    n += std::max<int64_t>(1, (r + MAX_CHUNK_ROWS - 1) / MAX_CHUNK_ROWS);
  }
  return n;
}

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
  if (o->flags != 0) return fail(DPAR2_EINVAL, "opts.flags must be 0");
  if (o->power_iters < 0 || o->power_iters > 4) return fail(DPAR2_EINVAL, "power_iters must be in [0, 4]");
  const int R = o->rank, L = o->sketch, L2 = o->sketch2;
  if (R < 1 || R > 32) return fail(DPAR2_ESHAPE, "rank must be in [1, 32]");
  if (L < R || L > 32) return fail(DPAR2_ESHAPE, "sketch width L must satisfy R <= L <= 32");
  if (L2 < R || L2 > 32) return fail(DPAR2_ESHAPE, "sketch width L2 must satisfy R <= L2 <= 32");
  if (o->max_iter < 0) return fail(DPAR2_EINVAL, "max_iter must be >= 0");
  const int64_t K = X->K, J = X->J;
  if (L > J) return fail(DPAR2_ESHAPE, "sketch width L exceeds J");
  if (L2 > J) return fail(DPAR2_ESHAPE, "sketch width L2 exceeds J");
  if ((int64_t)L2 > K * R) return fail(DPAR2_ESHAPE, "sketch width L2 exceeds K*R");
  if (!sketch_supported((int)J, L, X->dtype))
    return fail(DPAR2_ESHAPE, "J exceeds the slab pass limit (256 for float32, 128 for bf16 / fp8)");
  const int64_t* off = X->row_offsets_host;
  if (off[0] != 0) return fail(DPAR2_EINVAL, "row_offsets[0] must be 0");
  for (int64_t k = 0; k < K; ++k) {
    if (off[k + 1] < off[k]) return fail(DPAR2_EINVAL, "row_offsets must be non-decreasing");
    if (off[k + 1] - off[k] < L)
      return fail(DPAR2_ESHAPE, "slice " + std::to_string(k) + " has fewer rows than the sketch width L");
  }
  return DPAR2_OK;
}

Layout make_layout(const dpar2_tensor* X, const dpar2_opts* o) {
  Layout y;
  std::memset(&y, 0, sizeof(y));
  y.K = X->K;
  y.J = X->J;
  y.N = X->row_offsets_host[X->K];
  y.R = o->rank;
  y.L = o->sketch;
  y.L2 = o->sketch2;
  y.max_iter = o->max_iter;
  y.n_items = count_items(X->row_offsets_host, X->K);
  const int64_t K = y.K, J = y.J, R = y.R, L = y.L, L2 = y.L2, KR = K * R, RR = R * R;
  y.n2 = (KR + STAGE2_CHUNK - 1) / STAGE2_CHUNK;
  y.nblkA = y.nblkB = y.nblkC = als_blocks(K > J ? K : J, (int)R);
  y.nblkF = (int)std::min<int64_t>(K, 1024);
  const int64_t nbf = (KR + 255) / 256;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align256(p + bytes);
    return at;
  };
  y.ctl = take(sizeof(Ctl));
  y.items = take(sizeof(Item) * (size_t)y.n_items);
  y.slice_ptr = take(sizeof(int32_t) * (size_t)(K + 1));
  y.slice_list = take(sizeof(int32_t) * (size_t)y.n_items);
  y.partG = take(sizeof(double) * (size_t)(y.n_items * L * L));
  y.partP = take(sizeof(double) * (size_t)(y.n_items * L * J));
  y.partS = take(sizeof(double) * (size_t)y.n_items);
  y.xnorm2 = take(sizeof(double) * (size_t)K);
  y.Mt = take(sizeof(double) * (size_t)(KR * J));
  y.Phi = take(sizeof(double) * (size_t)(K * L * R));
  y.sig1 = take(sizeof(double) * (size_t)KR);
  y.Y2p = take(sizeof(double) * (size_t)(y.n2 * L2 * J));
  y.Y2 = take(sizeof(double) * (size_t)(J * L2));
  y.B2t = take(sizeof(double) * (size_t)(KR * L2));
  y.S2p = take(sizeof(double) * (size_t)(y.n2 * L2 * (L2 + 1) / 2));
  y.U2 = take(sizeof(double) * (size_t)(L2 * R));
  y.D = take(sizeof(double) * (size_t)(J * R));
  y.E = take(sizeof(double) * (size_t)R);
  y.F = take(sizeof(double) * (size_t)(KR * R));
  y.FtFp = take(sizeof(double) * (size_t)(nbf * RR));
  y.Psi = take(sizeof(double) * (size_t)(K * RR));
  y.Pw = take(sizeof(double) * (size_t)(K * RR));
  y.Mk = take(sizeof(double) * (size_t)(K * RR));
  y.small = take(sizeof(double) * (size_t)(SM_COUNT * RR));
  y.partA = take(sizeof(double) * (size_t)(y.nblkA * RR));
  y.partB = take(sizeof(double) * (size_t)(y.nblkB * RR));
  y.partC = take(sizeof(double) * (size_t)(y.nblkC * (RR + 2)));
  y.partBegin = take(sizeof(double) * (size_t)(y.nblkC * 3 * RR));
  y.red = take(sizeof(double) * (size_t)(6 * RR + 2));

  y.fitp = take(sizeof(double) * (size_t)(2 * y.nblkF));
  y.trace = take(sizeof(double) * (size_t)(K * L * R));   // Theta for the U output
  y.om1 = take(sizeof(float) * (size_t)(J * L));           // copy of Omega_1 for the U pass
  y.omq = take(o->power_iters > 0 ? sizeof(float) * (size_t)(K * J * L) : 0);   // power-step sketches
  y.total = p;
  return y;
}

dpar2_status check_ws(const Layout& y, const void* ws, size_t bytes) {
  if (!ws) return fail(DPAR2_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(DPAR2_EWORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < y.total)
    return fail(DPAR2_EWORKSPACE, "workspace too small: need " + std::to_string(y.total) + " bytes");
  return DPAR2_OK;
}

dpar2_status hip_fail(hipError_t e, const char* where) {
  return fail(DPAR2_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Pinned staging buffer for the schedule upload, one per workspace; an event
// guards reuse until the previous copy from it has completed.
struct Staging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
std::mutex g_stage_mu;
std::unordered_map<const void*, Staging> g_stage;

// Slab-pass timing (dpar2_profile_*).
struct Profile {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
};
std::mutex g_prof_mu;
Profile g_prof;

__global__ void k_ctl_reset(Ctl* ctl) {
  Ctl z;
  std::memset(&z, 0, sizeof(z));
  *ctl = z;
}

}  // namespace

extern "C" {

size_t dpar2_workspace_size(const dpar2_tensor* X, const dpar2_opts* o) {
  if (validate(X, o) != DPAR2_OK) return 0;
  return make_layout(X, o).total;
}

dpar2_status dpar2_compress(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                            const float* omega2, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!omega1 || !omega2) return fail(DPAR2_EINVAL, "omega1 and omega2 must be non-NULL");
  const Layout y = make_layout(X, o);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);

  Schedule sch;
  build_schedule(X->row_offsets_host, X->K, &sch);
  const size_t b_items = sizeof(Item) * sch.items.size();
  const size_t b_ptr = sizeof(int32_t) * sch.slice_ptr.size();
  const size_t b_list = sizeof(int32_t) * sch.slice_list.size();
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging& sg = g_stage[ws];
    const size_t need = b_items + b_ptr + b_list;
    hipError_t e;
    if (sg.done) {
      if ((e = hipEventSynchronize(sg.done)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else if ((e = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming)) != hipSuccess) {
      return hip_fail(e, "hipEventCreate");
    }
    if (sg.bytes < need) {
      if (sg.host) (void)hipHostFree(sg.host);
      sg.host = nullptr;
      sg.bytes = 0;
      if ((e = hipHostMalloc(&sg.host, need, hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "hipHostMalloc");
      sg.bytes = need;
    }
    char* h = static_cast<char*>(sg.host);
    std::memcpy(h, sch.items.data(), b_items);
    std::memcpy(h + b_items, sch.slice_ptr.data(), b_ptr);
    std::memcpy(h + b_items + b_ptr, sch.slice_list.data(), b_list);
    if ((e = hipMemcpyAsync(w + y.items, h, b_items, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(w + y.slice_ptr, h + b_items, b_ptr, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(w + y.slice_list, h + b_items + b_ptr, b_list, hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipEventRecord(sg.done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  {
    hipError_t e = hipMemcpyAsync(w + y.om1, omega1, sizeof(float) * (size_t)(y.J * y.L),
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  Ctl* ctl = reinterpret_cast<Ctl*>(w + y.ctl);
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(1), 0, s, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ctl reset");

  const Item* items = reinterpret_cast<const Item*>(w + y.items);
  double* partG = reinterpret_cast<double*>(w + y.partG);
  double* partP = reinterpret_cast<double*>(w + y.partP);
  double* partS = reinterpret_cast<double*>(w + y.partS);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.on) {
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
  SlabArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.slab = X->slab;
  sa.scale = X->slice_scale;
  sa.J = (int)y.J;
  sa.L = y.L;
  sa.R = y.R;
  sa.items = items;
  sa.partG = partG;
  sa.partP = partP;
  sa.partS = partS;
  float* omq = reinterpret_cast<float*>(w + y.omq);
  for (int pass = 0; pass <= o->power_iters; ++pass) {
    // pass 0 sketches with Omega_1; a power step with each slice's own matrix
    sa.omega = pass == 0 ? omega1 : omq;
    sa.om_stride = pass == 0 ? 0 : y.J * y.L;
    if (ev0 && (e = hipEventRecord(ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = launch_slab(sa, X->dtype, y.n_items, false, s);
    if (e != hipSuccess) return hip_fail(e, "slab pass");
    if (ev1 && (e = hipEventRecord(ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    ev0 = ev1 = nullptr;   // the timing hooks cover the first pass
    e = launch_slice_finish(y.K, (int)y.J, y.L, y.R, reinterpret_cast<const int32_t*>(w + y.slice_ptr),
                            reinterpret_cast<const int32_t*>(w + y.slice_list), partG, partP, partS,
                            reinterpret_cast<double*>(w + y.xnorm2), reinterpret_cast<double*>(w + y.Mt),
                            reinterpret_cast<double*>(w + y.Phi), reinterpret_cast<double*>(w + y.sig1),
                            pass < o->power_iters ? omq : nullptr, ctl, s);
    if (e != hipSuccess) return hip_fail(e, "slice finish");
  }
  e = launch_stage2(y, w, omega2, s);
  if (e != hipSuccess) return hip_fail(e, "second stage");
  e = launch_pw_identity(y, w, s);
  if (e != hipSuccess) return hip_fail(e, "iteration state init");
  return DPAR2_OK;
}

dpar2_status dpar2_als_step(const dpar2_tensor* X, const dpar2_opts* o, dpar2_factors* f, int32_t n_steps,
                            double* err_trace, void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  if (n_steps < 0) return fail(DPAR2_EINVAL, "n_steps must be >= 0");
  const Layout y = make_layout(X, o);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  hipError_t e = launch_als_begin(y, w, f->H, f->V, f->W, s);
  if (e != hipSuccess) return hip_fail(e, "iteration begin");
  for (int32_t t = 0; t < n_steps; ++t) {
    e = launch_als_iteration(y, w, f->H, f->V, f->W, err_trace, o->tol, s);
    if (e != hipSuccess) return hip_fail(e, "iteration");
  }
  e = launch_als_end(y, w, f->V, s);
  if (e != hipSuccess) return hip_fail(e, "iteration end");
  return DPAR2_OK;
}

dpar2_status dpar2_fitness(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f, double* fit,
                           void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !f->V || !f->W) return fail(DPAR2_EINVAL, "factors must be non-NULL");
  const Layout y = make_layout(X, o);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipError_t e = launch_fitness(y, static_cast<char*>(ws), f->H, f->V, f->W, fit,
                                reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "fitness");
  return DPAR2_OK;
}

dpar2_status dpar2_output_U(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f, double* U,
                            void* ws, size_t ws_bytes, dpar2_stream_t stream) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!f || !f->H || !U) return fail(DPAR2_EINVAL, "H and U must be non-NULL");
  const Layout y = make_layout(X, o);
  if ((st = check_ws(y, ws, ws_bytes)) != DPAR2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  double* theta = reinterpret_cast<double*>(w + y.trace);
  hipError_t e = launch_theta(y, w, f->H, theta, s);
  if (e != hipSuccess) return hip_fail(e, "theta");
  // the tiles of the U pass are those of the (last) slab pass: same Y bit for bit
  SlabArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.slab = X->slab;
  sa.scale = X->slice_scale;
  sa.J = (int)y.J;
  sa.L = y.L;
  sa.R = y.R;
  sa.omega = o->power_iters > 0 ? reinterpret_cast<const float*>(w + y.omq)
                                : reinterpret_cast<const float*>(w + y.om1);
  sa.om_stride = o->power_iters > 0 ? y.J * y.L : 0;
  sa.items = reinterpret_cast<const Item*>(w + y.items);
  sa.theta = theta;
  sa.U = U;
  e = launch_slab(sa, X->dtype, y.n_items, true, s);
  if (e != hipSuccess) return hip_fail(e, "U pass");
  return DPAR2_OK;
}

dpar2_status dpar2_decompose(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                             const float* omega2, dpar2_factors* f, double* U, void* ws, size_t ws_bytes,
                             dpar2_stream_t stream) {
  dpar2_status st = dpar2_compress(X, o, omega1, omega2, ws, ws_bytes, stream);
  if (st != DPAR2_OK) return st;
  st = dpar2_als_step(X, o, f, o->max_iter, nullptr, ws, ws_bytes, stream);
  if (st != DPAR2_OK) return st;
  st = dpar2_fitness(X, o, f, nullptr, ws, ws_bytes, stream);
  if (st != DPAR2_OK) return st;
  if (U) {
    st = dpar2_output_U(X, o, f, U, ws, ws_bytes, stream);
    if (st != DPAR2_OK) return st;
  }
  return DPAR2_OK;
}

dpar2_status dpar2_report_read(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, dpar2_report* rep,
                               dpar2_stream_t stream) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!rep || !ws) return fail(DPAR2_EINVAL, "report and workspace must be non-NULL");
  const Layout y = make_layout(X, o);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Ctl c;
  hipError_t e = hipMemcpyAsync(&c, static_cast<const char*>(ws) + y.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  rep->iters = c.iters;
  rep->converged = c.done;
  rep->err_last = c.e_prev;
  rep->xnorm2 = c.xnorm2;
  rep->fit_compressed = c.xnorm2 > 0 ? 1.0 - c.e_prev / c.xnorm2 : 0.0;
  rep->fit_true = c.fit_true;
  rep->warn_bits = c.warn;
  return DPAR2_OK;
}

dpar2_status dpar2_compressed_view(const dpar2_tensor* X, const dpar2_opts* o, const void* ws,
                                   size_t ws_bytes, dpar2_compressed* out) {
  dpar2_status st = validate(X, o);
  if (st != DPAR2_OK) return st;
  if (!out) return fail(DPAR2_EINVAL, "out is NULL");
  const Layout y = make_layout(X, o);
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

const char* dpar2_status_string(int32_t status) {
  switch (status) {
    case DPAR2_OK: return "ok";
    case DPAR2_EINVAL: return "invalid argument";
    case DPAR2_ESHAPE: return "shape not supported";
    case DPAR2_ENUMERIC: return "numerical failure";
    case DPAR2_EHIP: return "HIP runtime error";
    case DPAR2_EWORKSPACE: return "workspace missing, misaligned or too small";
    default: return "unknown status";
  }
}

const char* dpar2_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
