// Internal declarations shared by the libdwg translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dwg.h"

namespace dwg {

// Records a printf-style detail string for dwg_last_error() on the calling thread.
void set_error(const char* fmt, ...);

#define DWG_TRY_HIP(call)                                                            \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::dwg::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                    \
      return DWG_E_DEVICE;                                                           \
    }                                                                                \
  } while (0)

#define DWG_TRY_LAUNCH() DWG_TRY_HIP(hipGetLastError())

// ----------------------------------------------------------------------------- sizes
constexpr int kBlock = 256;    // threads per block for the all-pairs kernels (4 waves)
constexpr int kTile = 256;     // sources per LDS tile
constexpr int kQpt = 4;        // queries held in registers per thread
constexpr int kQBlock = kBlock * kQpt;  // queries per block
constexpr int kNAcc = 7;       // per-query accumulators with the gradient: w, A[3], B[3]
constexpr int kMaxSplit = 64;
constexpr int kRedBlock = 256;  // threads per block for O(n) epilogue / reductions
constexpr int kMaxK = 16;       // largest k for the kNN kernels

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over the caller's workspace. With base == nullptr it only measures.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = used;
    used = align256(used + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Split count for the all-pairs kernels.
int choose_split(int64_t n_src, int64_t n_qry, int requested);

// Device-side state of one GWN / iteration launch sequence, carved from the workspace.
struct GwnWork {
  float4* src;        // [2 * npad]: (px,py,pz,1/rho_min), (mx,my,mz,0) per source
  float* part;        // [split][kNAcc][mpad] per-split partial sums
  float* kk;          // [npad] a_j / (4 pi), for restaging after the update
  double* theta;      // [m] angle change in degrees (iterate)
  double* blk;        // [2 * nblk] per-block FP64 partial sums
  double* stats;      // [4] device statistics
  uint32_t* hist;     // [256] radix histogram
  uint64_t* sel;      // [2]: radix prefix, remaining count
  int64_t npad, mpad, ntiles;
  int split;
  int nblk;           // blocks of the O(n) epilogue kernels
};

size_t carve_gwn(Carver& c, int64_t n_src, int64_t n_qry, int split, GwnWork* out);

// Workspace bytes of the kNN / features / MLP stages for n points.
size_t knn_ws_bytes(int64_t n_ref, int64_t n_qry);
size_t mlp_ws_bytes(int64_t B);

// Launchers (all enqueue on `stream`; return DWG_OK or DWG_E_DEVICE).
dwg_status launch_stage(const float* P, const float* N, const float* area, const float* delta,
                        int64_t n, float eps, const GwnWork& w, hipStream_t stream);
dwg_status launch_gwn(const float* Q, int64_t m, const dwg_kernel_params& kp, bool grad,
                      const GwnWork& w, hipStream_t stream);
dwg_status launch_combine(int64_t m, const dwg_kernel_params& kp, bool grad, float* wout,
                          float* gout, double* wmean, const GwnWork& w, hipStream_t stream);
dwg_status launch_update(int64_t n, const float* area, const dwg_kernel_params& kp, float* N,
                         const GwnWork& w, hipStream_t stream);
dwg_status launch_stats(int64_t n, double top_frac, const GwnWork& w, hipStream_t stream);
dwg_status launch_random_normals(uint64_t seed, int64_t n, float* N, hipStream_t stream);

dwg_status knn_run(const float* R, int64_t nr, const float* Q, int64_t m, int self_skip,
                   const int64_t* skip_stride, int k, int32_t* idx, float* dist, void* ws,
                   size_t ws_bytes, hipStream_t stream);
dwg_status delta_from_knn(const float* dist, int64_t n, int k, float scale, float* delta,
                          hipStream_t stream);
dwg_status features_run(const float* P, int64_t n, int64_t n_anchor, float* feat, void* ws,
                        size_t ws_bytes, hipStream_t stream);
dwg_status mlp_infer_run(const float* params, const float* X, int64_t B, float* Y, void* ws,
                         size_t ws_bytes, hipStream_t stream);
dwg_status mlp_train_run(float* params, float* m1, float* m2, int64_t step, float lr,
                         const float* X, const float* T, const uint8_t* mask, int64_t B,
                         float* grad_out, float* loss_out, void* ws, size_t ws_bytes,
                         hipStream_t stream);

}  // namespace dwg
