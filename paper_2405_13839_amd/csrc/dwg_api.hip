// C ABI entry points of libdwg: argument validation (always before the first HIP call),
// workspace carving and the host-side iteration loop of Algorithm 1.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "dwg_internal.h"

namespace dwg {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

}  // namespace dwg

using namespace dwg;

namespace {

#define DWG_CHECK(cond, ...)        \
  do {                              \
    if (!(cond)) {                  \
      ::dwg::set_error(__VA_ARGS__); \
      return DWG_E_INVALID;         \
    }                               \
  } while (0)

#define DWG_PROPAGATE(expr)         \
  do {                              \
    dwg_status s_ = (expr);         \
    if (s_ != DWG_OK) return s_;    \
  } while (0)

const dwg_kernel_params kDefaultKp = {0.0f, 0.0f, 1, 0, 0.0f, 0, {0, 0}};
constexpr int kDefaultLeaf = 32;

bool tree_mode(const dwg_kernel_params& kp) { return kp.tree_beta > 0.0f; }
int tree_leaf(const dwg_kernel_params& kp) { return kp.tree_leaf > 0 ? kp.tree_leaf : kDefaultLeaf; }

dwg_status check_kp(const dwg_kernel_params* kp) {
  if (!kp) return DWG_OK;
  DWG_CHECK(std::isfinite(kp->lambda) && kp->lambda >= 0.0f, "lambda must be finite and >= 0");
  DWG_CHECK(std::isfinite(kp->eps) && kp->eps >= 0.0f, "eps must be finite and >= 0");
  DWG_CHECK(kp->compensated == 0 || kp->compensated == 1, "compensated must be 0 or 1");
  DWG_CHECK(kp->split >= 0 && kp->split <= kMaxSplit, "split must be in [0, 64]");
  DWG_CHECK(std::isfinite(kp->tree_beta) && (kp->tree_beta == 0.0f || kp->tree_beta >= 1.0f),
            "tree_beta must be 0 (all pairs) or a finite value >= 1");
  DWG_CHECK(kp->tree_leaf >= 0 && kp->tree_leaf <= 1024, "tree_leaf must be in [0, 1024]");
  for (int i = 0; i < 2; ++i) DWG_CHECK(kp->reserved[i] == 0, "reserved fields must be zero");
  return DWG_OK;
}

// The current device must be a gfx950 (asked on every call: no state is kept).
dwg_status check_device() {
  int dev = 0;
  DWG_TRY_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  DWG_TRY_HIP(hipGetDeviceProperties(&prop, dev));
  const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  if (!ok) {
    set_error("device %d is %s; libdwg is built for gfx950 only", dev, prop.gcnArchName);
    return DWG_E_UNSUPPORTED;
  }
  return DWG_OK;
}

// kNN-based stages (delta radius, anchor features): neighbour lists of n queries with up to
// 16 neighbours, the anchor copy and the grid.
int64_t feat_chunk(int64_t n) { return std::min<int64_t>(n, int64_t(1) << 20); }

size_t aux_bytes(int64_t n) {
  Carver c(nullptr);
  c.take<float>(3 * (size_t)n);
  c.take<int32_t>((size_t)n * kMaxK);
  c.take<float>((size_t)n * kMaxK);
  const size_t knn = c.used + knn_ws_bytes(n, n);
  Carver a(nullptr);
  carve_anchor(a, n, n, DWG_FEAT_ANCHORS, nullptr);
  return std::max(knn, a.used);
}

// Two HIP events, destroyed with the object.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  dwg_status create() {
    DWG_TRY_HIP(hipEventCreate(&a));
    DWG_TRY_HIP(hipEventCreate(&b));
    return DWG_OK;
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

size_t gwn_bytes(int64_t n_src, int64_t n_qry, const dwg_kernel_params& kp) {
  Carver c(nullptr);
  if (tree_mode(kp)) {
    carve_gwn(c, n_src, n_qry, 1, false, nullptr);
    carve_tree(c, n_src, tree_leaf(kp), kp.tree_beta, nullptr);
  } else {
    carve_gwn(c, n_src, n_qry, choose_split(n_src, n_qry, kp.split), false, nullptr);
  }
  return c.used;
}

// Carves the evaluation state, orders sources and queries and stages the sources: the
// all-pairs tiles, or the octree with its node summaries.
struct EvalState {
  GwnWork wk;
  TreeWork tw;
  bool tree = false;
};

dwg_status eval_prepare(const float* P, const float* N, const float* area, const float* delta, int64_t n,
                        const float* Q, int64_t m, const dwg_kernel_params& kp, bool same, void* ws,
                        hipStream_t st, EvalState* es) {
  Carver c(ws);
  es->tree = tree_mode(kp);
  if (!es->tree) {
    carve_gwn(c, n, m, choose_split(n, m, kp.split), same, &es->wk);
    DWG_PROPAGATE(launch_order(P, n, delta, kp.eps, position_scale(kp), Q, m, same, es->wk, st));
    return launch_stage(P, N, area, delta, n, kp.eps, position_scale(kp), es->wk, st);
  }
  carve_gwn(c, n, m, 1, same, &es->wk);
  carve_tree(c, n, tree_leaf(kp), kp.tree_beta, &es->tw);
  DWG_PROPAGATE(tree_build(P, area, delta, n, kp.eps, es->tw, es->wk.perm_s, st));
  if (!same) DWG_PROPAGATE(spatial_sort(Q, m, nullptr, 0.0f, es->wk.sort, es->wk.perm_q, st));
  DWG_PROPAGATE(launch_stage(P, N, area, delta, n, kp.eps, position_scale(kp), es->wk, st));
  return tree_stage_leaves(es->wk, es->tw, position_scale(kp), st);
}

// w (and grad) at the sorted queries into the per-query partials.
dwg_status eval_run(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad, const EvalState& es,
                    hipStream_t st) {
  if (!es.tree) return launch_gwn(Q, m, kp, grad, es.wk, st);
  DWG_PROPAGATE(tree_moments(es.wk, es.tw, st));
  return tree_eval(Q, m, kp, grad, es.wk, es.tw, st);
}

dwg_status gwn_common(const float* P, const float* N, const float* area, const float* delta,
                      int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kpp,
                      bool grad, float* w, float* g, double* wmean, void* ws, size_t ws_bytes,
                      void* stream) {
  DWG_CHECK(P && N && area && Q, "P, N, area and Q must not be NULL");
  DWG_CHECK(n >= 1 && m >= 1, "n and m must be >= 1 (got n=%lld, m=%lld)", (long long)n, (long long)m);
  DWG_CHECK(n < (int64_t(1) << 31) && m < (int64_t(1) << 31), "n and m must be < 2^31 (int32 point indices)");
  DWG_CHECK(grad ? (g != nullptr) : (w != nullptr), grad ? "grad must not be NULL" : "w must not be NULL");
  DWG_PROPAGATE(check_kp(kpp));
  const dwg_kernel_params kp = kpp ? *kpp : kDefaultKp;
  DWG_CHECK(!tree_mode(kp) || n < (int64_t(1) << 30), "octree mode needs n < 2^30");
  const size_t need = gwn_bytes(n, m, kp);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  EvalState es;
  const bool same = (Q == P && m == n);
  DWG_PROPAGATE(eval_prepare(P, N, area, delta, n, Q, m, kp, same, ws, st, &es));
  DWG_PROPAGATE(eval_run(Q, m, kp, grad, es, st));
  DWG_PROPAGATE(launch_combine(m, kp, grad, w, g, wmean, es.wk, st));
  return DWG_OK;
}

dwg_status check_mcp(const dwg_mc_params* mcp, int64_t n, McParams* out) {
  DWG_CHECK(mcp, "mcp must not be NULL");
  DWG_CHECK(mcp->depth >= 1 && mcp->depth <= 16, "depth must be in [1, 16]");
  DWG_CHECK(mcp->dilate >= 0 && mcp->dilate <= 2, "dilate must be in [0, 2]");
  DWG_CHECK(mcp->k >= 1 && mcp->k <= kMaxK, "k must be in [1, %d]", kMaxK);
  DWG_CHECK(mcp->iso == 0 || mcp->iso == 1, "iso must be 0 (points) or 1 (grid corners)");
  DWG_CHECK(mcp->surface == 0 || mcp->surface == 1, "surface must be 0 (Marching Cubes) or 1 (marching tetrahedra)");
  const int64_t w = 2 * mcp->dilate + 1;
  DWG_CHECK(n > mcp->k && n * w * w * w < (int64_t(1) << 31), "need k < n < 2^31 / (2 dilate + 1)^3");
  *out = McParams{mcp->depth, mcp->dilate, mcp->k, mcp->iso == 0 ? 1 : 0, mcp->surface};
  return DWG_OK;
}

size_t mc_bytes(int64_t n, const dwg_kernel_params& kp, const McParams& mp, int64_t cells) {
  Carver c(nullptr);
  carve_mc_grid(c, n, mp, nullptr);
  if (cells > 0) {
    carve_mc_faces(c, n, cells, mp, nullptr);
    c.used = align256(c.used + gwn_bytes(n, 8 * cells + (mp.iso_points ? n : 0), kp));
  }
  return c.used;
}

// Grid, corners and the evaluation state of the level-set update; checks the workspace
// against the actual cell count.
dwg_status mc_prepare(const float* P, const float* N, const float* area, const float* delta, int64_t n,
                      const dwg_kernel_params& kp, const McParams& mp, void* ws, size_t ws_bytes, hipStream_t st,
                      McWork* w, EvalState* es) {
  Carver c(ws);
  carve_mc_grid(c, n, mp, w);
  int64_t C = 0;
  DWG_PROPAGATE(mc_cells(P, n, mp, *w, &C, st));
  const size_t need = mc_bytes(n, kp, mp, C);
  if (ws_bytes < need) {
    set_error("workspace too small for %lld grid cells: %zu bytes given, %zu needed", (long long)C, ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_CHECK(mc_faces_per_cell(mp) * C < (int64_t(1) << 31), "too many grid cells (%lld)", (long long)C);
  carve_mc_faces(c, n, C, mp, w);
  int64_t m = 0;
  DWG_PROPAGATE(mc_corners(mp, *w, &m, st));
  if (mp.iso_points) DWG_PROPAGATE(mc_append_points(P, n, *w, st));
  DWG_PROPAGATE(knn_grid(P, n, w->knn, st));
  DWG_PROPAGATE(mc_clear(*w, st));
  return eval_prepare(P, N, area, delta, n, w->pos, w->ld, kp, false, static_cast<char*>(ws) + c.used, st, es);
}

// w at the corners (and at the points when w_bar is taken over them) and w_bar.
dwg_status mc_field(const dwg_kernel_params& kp, const McParams& mp, const McWork& w, const EvalState& es,
                    hipStream_t st) {
  DWG_PROPAGATE(eval_run(w.pos, w.ld, kp, false, es, st));
  if (!mp.iso_points) return launch_combine(w.ld, kp, false, w.wc, nullptr, w.iso, es.wk, st);
  DWG_PROPAGATE(launch_combine(w.ld, kp, false, w.wc, nullptr, nullptr, es.wk, st));
  return mc_point_iso(w, w.wc + w.m, w.n, st);
}

// ---- Scratch of dwg_gwn_grad_static: a device array instead of a caller workspace ----
// `scratch` is a device symbol: on the host its name stands for a host-side shadow, so its
// device address is asked from the runtime once per device (with that device current) and
// kept; kernels and copies only ever get that address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device ordinal

dwg_status static_scratch(void** out) {
  int dev = 0;
  DWG_TRY_HIP(hipGetDevice(&dev));
  DWG_CHECK(dev >= 0 && dev < kMaxDevices, "device ordinal %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return DWG_E_DEVICE;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return DWG_OK;
}

// The kernel parameters dwg_gwn_grad_static runs with: an automatic source split is halved
// until the evaluation fits the static scratch (the split only groups the partial sums).
dwg_kernel_params static_params(int64_t n, int64_t m, const dwg_kernel_params& kp) {
  dwg_kernel_params k = kp;
  if (!tree_mode(k) && k.split == 0) {
    k.split = choose_split(n, m, 0);
    while (k.split > 1 && gwn_bytes(n, m, k) > kStaticScratchBytes) k.split = (k.split + 1) / 2;
  }
  return k;
}

}  // namespace

extern "C" {

const char* dwg_version(void) { return "dwg-mi355x 0.1.0 (gfx950)"; }

const char* dwg_status_string(int s) {
  switch (s) {
    case DWG_OK: return "DWG_OK";
    case DWG_NOT_CONVERGED: return "DWG_NOT_CONVERGED";
    case DWG_E_INVALID: return "DWG_E_INVALID";
    case DWG_E_WORKSPACE: return "DWG_E_WORKSPACE";
    case DWG_E_DEVICE: return "DWG_E_DEVICE";
    case DWG_E_NONFINITE: return "DWG_E_NONFINITE";
    case DWG_E_UNSUPPORTED: return "DWG_E_UNSUPPORTED";
    default: return "DWG_UNKNOWN_STATUS";
  }
}

const char* dwg_last_error(void) { return g_err; }

size_t dwg_workspace_bytes(int64_t n_src, int64_t n_qry, const dwg_kernel_params* kp) {
  if (n_src < 1 || n_qry < 1 || n_src >= (int64_t(1) << 31) || n_qry >= (int64_t(1) << 31)) return 0;
  if (check_kp(kp) != DWG_OK) return 0;
  const dwg_kernel_params k = kp ? *kp : kDefaultKp;
  size_t a = gwn_bytes(n_src, n_qry, k);
  size_t b = aux_bytes(std::max(n_src, n_qry));
  size_t c = mlp_ws_bytes(std::max(n_src, n_qry));
  return align256(std::max(a, std::max(b, c)));
}

dwg_status dwg_gwn_eval(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kp,
                        float* w, double* wmean, void* ws, size_t ws_bytes, void* stream) {
  return gwn_common(P, N, area, delta, n, Q, m, kp, false, w, nullptr, wmean, ws, ws_bytes, stream);
}

dwg_status dwg_gwn_grad(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kp,
                        float* w, float* grad, double* wmean, void* ws, size_t ws_bytes,
                        void* stream) {
  return gwn_common(P, N, area, delta, n, Q, m, kp, true, w, grad, wmean, ws, ws_bytes, stream);
}

dwg_status dwg_gwn_grad_static(const float* P, const float* N, const float* area, const float* delta,
                               int64_t n, const float* Q, int64_t m, const dwg_kernel_params* kpp,
                               float* w, float* grad, double* wmean, void* stream) {
  DWG_CHECK(P && N && area && Q, "P, N, area and Q must not be NULL");
  DWG_CHECK(n >= 1 && m >= 1, "n and m must be >= 1 (got n=%lld, m=%lld)", (long long)n, (long long)m);
  DWG_CHECK(n < (int64_t(1) << 31) && m < (int64_t(1) << 31), "n and m must be < 2^31 (int32 point indices)");
  DWG_CHECK(grad != nullptr, "grad must not be NULL");
  DWG_PROPAGATE(check_kp(kpp));
  const dwg_kernel_params kp = static_params(n, m, kpp ? *kpp : kDefaultKp);
  DWG_CHECK(!tree_mode(kp) || n < (int64_t(1) << 30), "octree mode needs n < 2^30");
  const size_t need = gwn_bytes(n, m, kp);
  DWG_CHECK(need <= kStaticScratchBytes,
            "n = %lld sources and m = %lld queries need %zu bytes of scratch; the static scratch holds %zu "
            "(use dwg_gwn_grad with a workspace)",
            (long long)n, (long long)m, need, kStaticScratchBytes);
  DWG_PROPAGATE(check_device());
  void* ws = nullptr;
  DWG_PROPAGATE(static_scratch(&ws));
  return gwn_common(P, N, area, delta, n, Q, m, &kp, true, w, grad, wmean, ws, kStaticScratchBytes, stream);
}

dwg_status dwg_octree_work(const float* P, const float* area, const float* delta, int64_t n, const float* Q,
                           int64_t m, const dwg_kernel_params* kpp, int64_t* work, void* ws, size_t ws_bytes,
                           void* stream) {
  if (work)
    for (int k = 0; k < kTreeWorkCounts; ++k) work[k] = 0;
  DWG_CHECK(P && area && Q && work, "P, area, Q and work must not be NULL");
  DWG_CHECK(n >= 1 && m >= 1, "n and m must be >= 1 (got n=%lld, m=%lld)", (long long)n, (long long)m);
  DWG_CHECK(n < (int64_t(1) << 30) && m < (int64_t(1) << 31), "need n < 2^30 and m < 2^31");
  DWG_PROPAGATE(check_kp(kpp));
  DWG_CHECK(kpp && tree_mode(*kpp), "kp->tree_beta must be > 0 (octree mode)");
  const dwg_kernel_params kp = *kpp;
  Carver need(nullptr);
  carve_gwn(need, n, m, 1, false, nullptr);
  carve_tree(need, n, tree_leaf(kp), kp.tree_beta, nullptr);
  need.take<unsigned long long>(kTreeWorkCounts);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need.used) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need.used);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool same = (Q == P && m == n);
  Carver c(ws);
  GwnWork wk;
  TreeWork tw;
  carve_gwn(c, n, m, 1, same, &wk);
  carve_tree(c, n, tree_leaf(kp), kp.tree_beta, &tw);
  unsigned long long* cnt = c.take<unsigned long long>(kTreeWorkCounts);
  DWG_PROPAGATE(tree_build(P, area, delta, n, kp.eps, tw, wk.perm_s, st));
  if (!same) DWG_PROPAGATE(spatial_sort(Q, m, nullptr, 0.0f, wk.sort, wk.perm_q, st));
  DWG_PROPAGATE(tree_work(Q, m, wk.perm_q, tw, cnt, st));
  unsigned long long h[kTreeWorkCounts] = {};
  DWG_TRY_HIP(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < kTreeWorkCounts; ++k) work[k] = (int64_t)h[k];
  return DWG_OK;
}

dwg_status dwg_iterate(const float* P, const float* area, const float* delta, int64_t n,
                       float* N_inout, const dwg_kernel_params* kpp, const dwg_iterate_params* ip,
                       dwg_iter_stat* stats_host, int* iters_done, void* ws, size_t ws_bytes,
                       void* stream) {
  if (iters_done) *iters_done = 0;
  DWG_CHECK(P && area && N_inout && ip, "P, area, N_inout and ip must not be NULL");
  DWG_CHECK(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31) (got %lld)", (long long)n);
  DWG_CHECK(ip->max_iters >= 1, "max_iters must be >= 1");
  DWG_CHECK(ip->fixed_iters == 0 || ip->fixed_iters == 1, "fixed_iters must be 0 or 1");
  DWG_CHECK(std::isfinite(ip->eps_deg) && ip->eps_deg >= 0.0, "eps_deg must be finite and >= 0");
  DWG_CHECK(ip->top_frac > 0.0 && ip->top_frac <= 1.0, "top_frac must be in (0, 1]");
  DWG_PROPAGATE(check_kp(kpp));
  const dwg_kernel_params kp = kpp ? *kpp : kDefaultKp;
  DWG_CHECK(!tree_mode(kp) || n < (int64_t(1) << 30), "octree mode needs n < 2^30");
  const size_t need = gwn_bytes(n, n, kp);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  EvalState es;
  DWG_PROPAGATE(eval_prepare(P, N_inout, area, delta, n, P, n, kp, true, ws, st, &es));
  const GwnWork& wk = es.wk;
  EventPair ev;
  DWG_PROPAGATE(ev.create());
  dwg_status result = DWG_NOT_CONVERGED;
  for (int t = 0; t < ip->max_iters; ++t) {
    DWG_TRY_HIP(hipEventRecord(ev.a, st));
    DWG_PROPAGATE(eval_run(P, n, kp, true, es, st));
    DWG_TRY_HIP(hipEventRecord(ev.b, st));
    DWG_PROPAGATE(launch_update(n, kp, N_inout, wk, st));
    DWG_PROPAGATE(launch_stats(n, ip->top_frac, wk, st));
    double hs[4];
    DWG_TRY_HIP(hipMemcpyAsync(hs, wk.stats, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    DWG_TRY_HIP(hipStreamSynchronize(st));
    float kms = 0.0f;
    DWG_TRY_HIP(hipEventElapsedTime(&kms, ev.a, ev.b));
    if (stats_host) {
      stats_host[t].wmean = hs[0];
      stats_host[t].top_mean_deg = hs[1];
      stats_host[t].mean_chord = hs[2];
      stats_host[t].gwn_ms = (double)kms;
    }
    if (iters_done) *iters_done = t + 1;
    if (!std::isfinite(hs[0]) || !std::isfinite(hs[1]) || !std::isfinite(hs[2])) {
      set_error("non-finite statistics at iteration %d (wmean=%g, top=%g, chord=%g)", t + 1, hs[0],
                hs[1], hs[2]);
      return DWG_E_NONFINITE;
    }
    if (ip->fixed_iters) {
      result = DWG_OK;
    } else if (hs[1] <= ip->eps_deg) {
      result = DWG_OK;
      break;
    }
  }
  if (ip->fixed_iters) result = DWG_OK;
  return result;
}

size_t dwg_mc_workspace_bytes(int64_t n, const dwg_kernel_params* kp, const dwg_mc_params* mcp, int64_t cells) {
  McParams mp;
  if (check_mcp(mcp, n, &mp) != DWG_OK || check_kp(kp) != DWG_OK || cells < 0) return 0;
  const dwg_kernel_params k = kp ? *kp : kDefaultKp;
  return align256(mc_bytes(n, k, mp, cells));
}

dwg_status dwg_mc_cells(const float* P, int64_t n, const dwg_mc_params* mcp, int64_t* cells, void* ws,
                        size_t ws_bytes, void* stream) {
  if (cells) *cells = 0;
  DWG_CHECK(P && cells, "P and cells must not be NULL");
  McParams mp;
  DWG_PROPAGATE(check_mcp(mcp, n, &mp));
  const size_t need = mc_bytes(n, kDefaultKp, mp, 0);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  Carver c(ws);
  McWork w;
  carve_mc_grid(c, n, mp, &w);
  return mc_cells(P, n, mp, w, cells, static_cast<hipStream_t>(stream));
}

dwg_status dwg_iterate_mc(const float* P, const float* area, const float* delta, int64_t n, float* N_inout,
                          const dwg_kernel_params* kpp, const dwg_iterate_params* ip, const dwg_mc_params* mcp,
                          dwg_iter_stat* stats_host, int* iters_done, void* ws, size_t ws_bytes, void* stream) {
  if (iters_done) *iters_done = 0;
  DWG_CHECK(P && area && N_inout && ip, "P, area, N_inout and ip must not be NULL");
  DWG_CHECK(ip->max_iters >= 1, "max_iters must be >= 1");
  DWG_CHECK(ip->fixed_iters == 0 || ip->fixed_iters == 1, "fixed_iters must be 0 or 1");
  DWG_CHECK(std::isfinite(ip->eps_deg) && ip->eps_deg >= 0.0, "eps_deg must be finite and >= 0");
  DWG_CHECK(ip->top_frac > 0.0 && ip->top_frac <= 1.0, "top_frac must be in (0, 1]");
  McParams mp;
  DWG_PROPAGATE(check_mcp(mcp, n, &mp));
  DWG_PROPAGATE(check_kp(kpp));
  const dwg_kernel_params kp = kpp ? *kpp : kDefaultKp;
  const size_t need0 = mc_bytes(n, kp, mp, 0);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need0) {
    set_error("workspace too small: %zu bytes given, at least %zu needed", ws_bytes, need0);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  McWork w;
  EvalState es;
  DWG_PROPAGATE(mc_prepare(P, N_inout, area, delta, n, kp, mp, ws, ws_bytes, st, &w, &es));
  EventPair ev;
  DWG_PROPAGATE(ev.create());
  dwg_status result = DWG_NOT_CONVERGED;
  for (int t = 0; t < ip->max_iters; ++t) {
    DWG_TRY_HIP(hipEventRecord(ev.a, st));
    DWG_PROPAGATE(mc_field(kp, mp, w, es, st));
    DWG_TRY_HIP(hipEventRecord(ev.b, st));
    int64_t F = 0;
    DWG_PROPAGATE(mc_faces(w, nullptr, 0, &F, st));
    DWG_PROPAGATE(mc_scatter(mp, w, F, st));
    DWG_PROPAGATE(mc_update(mp, w, es.wk, N_inout, st));
    DWG_PROPAGATE(launch_stats(n, ip->top_frac, es.wk, st));
    DWG_TRY_HIP(hipMemcpyAsync(es.wk.stats, w.iso, sizeof(double), hipMemcpyDeviceToDevice, st));
    double hs[4];
    DWG_TRY_HIP(hipMemcpyAsync(hs, es.wk.stats, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    DWG_TRY_HIP(hipStreamSynchronize(st));
    float kms = 0.0f;
    DWG_TRY_HIP(hipEventElapsedTime(&kms, ev.a, ev.b));
    if (stats_host) {
      stats_host[t].wmean = hs[0];
      stats_host[t].top_mean_deg = hs[1];
      stats_host[t].mean_chord = hs[2];
      stats_host[t].gwn_ms = (double)kms;
    }
    if (iters_done) *iters_done = t + 1;
    if (!std::isfinite(hs[0]) || !std::isfinite(hs[1]) || !std::isfinite(hs[2])) {
      set_error("non-finite statistics at iteration %d (wmean=%g, top=%g, chord=%g)", t + 1, hs[0], hs[1], hs[2]);
      return DWG_E_NONFINITE;
    }
    if (ip->fixed_iters) {
      result = DWG_OK;
    } else if (hs[1] <= ip->eps_deg) {
      result = DWG_OK;
      break;
    }
  }
  if (ip->fixed_iters) result = DWG_OK;
  return result;
}

dwg_status dwg_level_set(const float* P, const float* N, const float* area, const float* delta, int64_t n,
                         const dwg_kernel_params* kpp, const dwg_mc_params* mcp, float* tri, int64_t cap,
                         int64_t* ntri, double* iso, void* ws, size_t ws_bytes, void* stream) {
  if (ntri) *ntri = 0;
  DWG_CHECK(P && N && area && tri && ntri && iso, "P, N, area, tri, ntri and iso must not be NULL");
  DWG_CHECK(cap >= 1, "cap must be >= 1");
  McParams mp;
  DWG_PROPAGATE(check_mcp(mcp, n, &mp));
  DWG_PROPAGATE(check_kp(kpp));
  const dwg_kernel_params kp = kpp ? *kpp : kDefaultKp;
  const size_t need0 = mc_bytes(n, kp, mp, 0);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need0) {
    set_error("workspace too small: %zu bytes given, at least %zu needed", ws_bytes, need0);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  McWork w;
  EvalState es;
  DWG_PROPAGATE(mc_prepare(P, N, area, delta, n, kp, mp, ws, ws_bytes, st, &w, &es));
  DWG_PROPAGATE(mc_field(kp, mp, w, es, st));
  int64_t F = 0;
  DWG_PROPAGATE(mc_faces(w, tri, cap, &F, st));
  DWG_TRY_HIP(hipMemcpyAsync(iso, w.iso, sizeof(double), hipMemcpyDeviceToHost, st));
  DWG_TRY_HIP(hipStreamSynchronize(st));
  *ntri = F;
  if (F > cap) {
    set_error("level set has %lld triangles, output holds %lld", (long long)F, (long long)cap);
    return DWG_E_INVALID;
  }
  return DWG_OK;
}


dwg_status dwg_octree(const float* P, int64_t n, int leaf, int32_t* perm, int32_t* nodes, int64_t cap,
                      int64_t* count, void* ws, size_t ws_bytes, void* stream) {
  if (count) *count = 0;
  DWG_CHECK(P && perm && nodes && count, "P, perm, nodes and count must not be NULL");
  DWG_CHECK(n >= 1 && n < (int64_t(1) << 30), "n must be in [1, 2^30)");
  DWG_CHECK(leaf >= 0 && leaf <= 1024, "leaf must be in [0, 1024]");
  DWG_CHECK(cap >= 1, "cap must be >= 1");
  dwg_kernel_params kp = kDefaultKp;
  kp.tree_beta = 2.3f;
  kp.tree_leaf = leaf;
  const size_t need = gwn_bytes(n, n, kp);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  GwnWork wk;
  TreeWork tw;
  carve_gwn(c, n, n, 1, true, &wk);
  carve_tree(c, n, tree_leaf(kp), kp.tree_beta, &tw);
  DWG_PROPAGATE(tree_build(P, nullptr, nullptr, n, 0.0f, tw, perm, st));
  return tree_export(tw, nodes, cap, count, st);
}

dwg_status dwg_init_normals(dwg_init_kind kind, uint64_t seed, const float* P, int64_t n,
                            const float* mlp_params, float* N_out, void* ws, size_t ws_bytes,
                            void* stream) {
  DWG_CHECK(kind == DWG_INIT_RANDOM || kind == DWG_INIT_MLP || kind == DWG_INIT_PCA || kind == DWG_INIT_GAUSS,
            "unknown init kind %d", (int)kind);
  DWG_CHECK(N_out, "N_out must not be NULL");
  DWG_CHECK(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (kind == DWG_INIT_RANDOM) {
    DWG_PROPAGATE(check_device());
    return launch_random_normals(seed, n, N_out, st);
  }
  if (kind == DWG_INIT_GAUSS) {
    DWG_CHECK(P, "P must not be NULL for DWG_INIT_GAUSS");
    DWG_PROPAGATE(check_device());
    return gauss_normals(P, n, N_out, st);
  }
  if (kind == DWG_INIT_PCA) {
    DWG_CHECK(P, "P must not be NULL for DWG_INIT_PCA");
    DWG_CHECK(n > kMaxK && n < (int64_t(1) << 31), "DWG_INIT_PCA needs %d < n < 2^31", kMaxK);
    const size_t need = aux_bytes(n);
    DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
    if (!ws || ws_bytes < need) {
      set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
      return DWG_E_WORKSPACE;
    }
    DWG_PROPAGATE(check_device());
    return pca_normals(P, n, kMaxK, N_out, ws, st);
  }
  DWG_CHECK(P && mlp_params, "P and mlp_params must not be NULL for DWG_INIT_MLP");
  DWG_CHECK(n >= DWG_FEAT_K + 2, "DWG_INIT_MLP needs at least %d points", DWG_FEAT_K + 2);
  const size_t need = aux_bytes(n);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  // anchors and their grid once, then features and the MLP in chunks of <= 2^20 points,
  // written straight into the planar [3][n] output
  Carver c(ws);
  AnchorCtx x;
  carve_anchor(c, n, feat_chunk(n), DWG_FEAT_ANCHORS, &x);
  DWG_PROPAGATE(anchor_build(P, n, x, st));
  for (int64_t q0 = 0; q0 < n; q0 += x.chunk) {
    const int64_t cnt = std::min<int64_t>(x.chunk, n - q0);
    DWG_PROPAGATE(anchor_features(P, n, q0, cnt, x, x.feat, st));
    DWG_PROPAGATE(mlp_forward(mlp_params, x.feat, cnt, N_out + q0, 1, n, st));
  }
  return DWG_OK;
}

dwg_status dwg_knn(const float* R, int64_t nr, const float* Q, int64_t m, int self_skip, int k,
                   int32_t* idx, float* dist, void* ws, size_t ws_bytes, void* stream) {
  DWG_CHECK(R && Q && idx, "R, Q and idx must not be NULL");
  DWG_CHECK(k >= 1 && k <= kMaxK, "k must be in [1, %d]", kMaxK);
  DWG_CHECK(self_skip == 0 || self_skip == 1, "self_skip must be 0 or 1");
  DWG_CHECK(nr >= k + self_skip && m >= 1 && nr < (int64_t(1) << 31) && m < (int64_t(1) << 31),
            "need nr >= k + self_skip, m >= 1, sizes < 2^31");
  DWG_CHECK(!self_skip || (R == Q && nr == m), "self_skip requires Q == R");
  const size_t need = knn_ws_bytes(nr, m);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return knn_run(R, nr, Q, m, self_skip, nullptr, k, idx, dist, ws, ws_bytes,
                 static_cast<hipStream_t>(stream));
}

dwg_status dwg_delta_knn_mean(const float* P, int64_t n, int k, float scale, float* delta,
                              void* ws, size_t ws_bytes, void* stream) {
  DWG_CHECK(P && delta, "P and delta must not be NULL");
  DWG_CHECK(k >= 1 && k <= kMaxK, "k must be in [1, %d]", kMaxK);
  DWG_CHECK(n > k && n < (int64_t(1) << 31), "need k < n < 2^31");
  DWG_CHECK(std::isfinite(scale) && scale > 0.0f, "scale must be finite and > 0");
  Carver c(nullptr);
  c.take<int32_t>((size_t)n * k);
  c.take<float>((size_t)n * k);
  const size_t head = c.used;
  const size_t need = aux_bytes(n);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver w(ws);
  int32_t* idx = w.take<int32_t>((size_t)n * k);
  float* dist = w.take<float>((size_t)n * k);
  DWG_PROPAGATE(knn_run(P, n, P, n, 1, nullptr, k, idx, dist, static_cast<char*>(ws) + head,
                        ws_bytes - head, st));
  return delta_from_knn(dist, n, k, scale, delta, st);
}

dwg_status dwg_delta_knn_window(const float* P, int64_t n, int k, float vmin, float vmax, float* delta,
                                void* ws, size_t ws_bytes, void* stream) {
  DWG_CHECK(P && delta, "P and delta must not be NULL");
  DWG_CHECK(k >= 1 && k <= kMaxK, "k must be in [1, %d]", kMaxK);
  DWG_CHECK(n > k && n < (int64_t(1) << 31), "need k < n < 2^31");
  DWG_CHECK(std::isfinite(vmin) && std::isfinite(vmax) && vmin >= 0.0f && vmax >= vmin,
            "need finite 0 <= vmin <= vmax");
  const size_t need = aux_bytes(n);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return delta_window(P, n, k, vmin, vmax, delta, ws, static_cast<hipStream_t>(stream));
}

dwg_status dwg_voronoi_area(const float* P, int64_t n, int m, float* area, void* ws, size_t ws_bytes,
                            void* stream) {
  DWG_CHECK(P && area, "P and area must not be NULL");
  DWG_CHECK(m >= 3 && m <= kMaxK, "m must be in [3, %d]", kMaxK);
  DWG_CHECK(n > m && n < (int64_t(1) << 31), "need m < n < 2^31");
  const size_t need = aux_bytes(n);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return voronoi_area(P, n, m, area, ws, static_cast<hipStream_t>(stream));
}

dwg_status dwg_delta_anchor_mean(const float* P, int64_t n, int k, int64_t n_anchor, float scale,
                                 float* delta, void* ws, size_t ws_bytes, void* stream) {
  DWG_CHECK(P && delta, "P and delta must not be NULL");
  DWG_CHECK(k >= 1 && k <= kMaxK, "k must be in [1, %d]", kMaxK);
  DWG_CHECK(n_anchor > k, "n_anchor must exceed k");
  DWG_CHECK(n > k + 1 && n < (int64_t(1) << 31), "need k + 1 < n < 2^31");
  DWG_CHECK(std::isfinite(scale) && scale > 0.0f, "scale must be finite and > 0");
  // the anchor grid grows with n_anchor: the requirement is the larger of the two layouts
  const size_t need = std::max(aux_bytes(n), anchor_ws_bytes(n, feat_chunk(n), n_anchor));
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws);
  AnchorCtx x;
  carve_anchor(c, n, feat_chunk(n), n_anchor, &x);
  DWG_CHECK(x.na > k, "too few anchors (%lld) for k = %d", (long long)x.na, k);
  DWG_PROPAGATE(anchor_build(P, n, x, st));
  return anchor_delta(P, n, x, k, scale, delta, st);
}

int64_t dwg_mlp_param_count(void) {
  return (int64_t)DWG_MLP_HID * DWG_MLP_IN + DWG_MLP_HID + (int64_t)DWG_MLP_HID * DWG_MLP_HID +
         DWG_MLP_HID + (int64_t)DWG_MLP_OUT * DWG_MLP_HID + DWG_MLP_OUT;
}

size_t dwg_mlp_blob_bytes(void) { return (size_t)dwg_mlp_param_count() * sizeof(float); }

dwg_status dwg_features(const float* P, int64_t n, int64_t n_anchor, float* feat, void* ws,
                        size_t ws_bytes, void* stream) {
  DWG_CHECK(P && feat, "P and feat must not be NULL");
  DWG_CHECK(n >= DWG_FEAT_K + 2 && n < (int64_t(1) << 31), "n must be in [%d, 2^31)", DWG_FEAT_K + 2);
  DWG_CHECK(n_anchor >= DWG_FEAT_K + 1, "n_anchor must be >= %d", DWG_FEAT_K + 1);
  const size_t need = std::max(aux_bytes(n), anchor_ws_bytes(n, n, n_anchor));
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return features_run(P, n, n_anchor, feat, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

dwg_status dwg_mlp_infer(const float* params, const float* X, int64_t B, float* Y, void* ws,
                         size_t ws_bytes, void* stream) {
  DWG_CHECK(params && X && Y, "params, X and Y must not be NULL");
  DWG_CHECK(B >= 1 && B < (int64_t(1) << 31), "B must be in [1, 2^31)");
  const size_t need = mlp_ws_bytes(B);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return mlp_infer_run(params, X, B, Y, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

dwg_status dwg_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t step,
                              float lr, const float* X, const float* T, const uint8_t* mask,
                              int64_t B, float* grad_out, float* loss_out, void* ws,
                              size_t ws_bytes, void* stream) {
  DWG_CHECK(params && adam_m && adam_v && X && T, "params, adam_m, adam_v, X, T must not be NULL");
  DWG_CHECK(step >= 1, "step must be >= 1");
  DWG_CHECK(std::isfinite(lr) && lr > 0.0f, "lr must be finite and > 0");
  DWG_CHECK(B >= 1 && B < (int64_t(1) << 31), "B must be in [1, 2^31)");
  const size_t need = mlp_ws_bytes(B);
  DWG_CHECK(ws || ws_bytes == 0, "ws is NULL but ws_bytes > 0");
  if (!ws || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    return DWG_E_WORKSPACE;
  }
  DWG_PROPAGATE(check_device());
  return mlp_train_run(params, adam_m, adam_v, step, lr, X, T, mask, B, grad_out, loss_out, ws,
                       ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
