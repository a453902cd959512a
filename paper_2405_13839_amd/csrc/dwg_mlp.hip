// Learned initial normals: MLP 48 -> 128 -> 128 -> 3 (ReLU, normalised output) on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation),
// its backward pass and Adam, all in this file. Not in the paper: it replaces the random /
// PCA / Gauss-map initial normals of Sec. 5.1 ("Normal Initialization").
//
// One block = 256 threads (4 waves) = 64 feature rows; wave w owns rows 16w..16w+15 in the
// row-parallel GEMMs. Weights and activations live in LDS as BF16 (round to nearest even).
// MFMA operand layout (16x16x32): lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; the FP32 result holds D[4 (l / 16) + i][l % 16].
//
// Parameter blob (FP32): W1[128][48] b1[128] W2[128][128] b2[128] W3[3][128] b3[3].
#include <cmath>

#include "dwg_internal.h"

namespace dwg {
namespace {

constexpr int IN = DWG_MLP_IN, HID = DWG_MLP_HID, OUT = DWG_MLP_OUT;
constexpr int INP = 64;  // input width padded to two K=32 steps
constexpr int ROWS = 64; // rows per block
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + HID * IN, OFF_W2 = OFF_B1 + HID,
              OFF_B2 = OFF_W2 + HID * HID, OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + OUT * HID,
              NPAR = OFF_B3 + OUT;
constexpr int NPART = NPAR + 1;  // per-block partial gradient + loss

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ __forceinline__ u16 to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(u16 h) { return __uint_as_float((unsigned)h << 16); }

// 8 consecutive BF16 values (16-byte aligned) from LDS
__device__ __forceinline__ bf16x8 ld8(const u16* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
// 8 BF16 values at stride `ld` from LDS
__device__ __forceinline__ bf16x8 ld8s(const u16* p, int ld) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = __builtin_bit_cast(__bf16, p[j * ld]);
  return r;
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Smem {
  u16 W1[HID][INP];   // 16 KB, k >= 48 zero
  u16 W2[HID][HID];   // 32 KB
  u16 W3[16][HID];    // 4 KB, rows >= 3 zero
  u16 X[ROWS][INP];   // 8 KB
  u16 H1[ROWS][HID];  // 16 KB
  u16 H2[ROWS][HID];  // 16 KB
  float Y[ROWS][4];   // 1 KB
};
struct SmemBwd {
  u16 DZ2[ROWS][HID];  // 16 KB
  u16 DZ1[ROWS][HID];  // 16 KB
  float DY[ROWS][4];   // 1 KB
  float red[2][HID];   // 1 KB bias-gradient halves
  double loss[4];
};

// Load the weights (BF16) into LDS.
__device__ void load_weights(Smem& s, const float* __restrict__ prm) {
  const int t = threadIdx.x;
  for (int i = t; i < HID * INP; i += blockDim.x) {
    const int n = i / INP, k = i % INP;
    s.W1[n][k] = k < IN ? to_bf16(prm[OFF_W1 + n * IN + k]) : (u16)0;
  }
  for (int i = t; i < HID * HID; i += blockDim.x) s.W2[i / HID][i % HID] = to_bf16(prm[OFF_W2 + i]);
  for (int i = t; i < 16 * HID; i += blockDim.x) {
    const int c = i / HID, k = i % HID;
    s.W3[c][k] = c < OUT ? to_bf16(prm[OFF_W3 + c * HID + k]) : (u16)0;
  }
}

// Load the feature rows row0 .. row0 + ROWS - 1 into LDS (BF16). Rows past B read as zero.
__device__ void load_rows(Smem& s, const float* __restrict__ X, int64_t B, int64_t row0) {
  const int t = threadIdx.x;
  for (int i = t; i < ROWS * INP; i += blockDim.x) {
    const int r = i / INP, k = i % INP;
    const int64_t g = row0 + r;
    s.X[r][k] = (k < IN && g < B) ? to_bf16(X[g * IN + k]) : (u16)0;
  }
}

// Forward of the wave's 16 rows: H1, H2 (BF16, post-ReLU) and Y (FP32, pre-normalisation).
__device__ void forward_wave(Smem& s, const float* __restrict__ prm) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 16 * w, lr = l % 16, lg = l / 16;
  // layer 1: H1 = ReLU(X W1^T + b1)
  for (int t = 0; t < HID / 16; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < INP / 32; ++kk)
      acc = mfma(ld8(&s.X[r0 + lr][kk * 32 + 8 * lg]), ld8(&s.W1[t * 16 + lr][kk * 32 + 8 * lg]), acc);
    const int col = t * 16 + lr;
    const float b = prm[OFF_B1 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) s.H1[r0 + 4 * lg + i][col] = to_bf16(fmaxf(acc[i] + b, 0.0f));
  }
  __syncthreads();
  // layer 2: H2 = ReLU(H1 W2^T + b2)
  for (int t = 0; t < HID / 16; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < HID / 32; ++kk)
      acc = mfma(ld8(&s.H1[r0 + lr][kk * 32 + 8 * lg]), ld8(&s.W2[t * 16 + lr][kk * 32 + 8 * lg]), acc);
    const int col = t * 16 + lr;
    const float b = prm[OFF_B2 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) s.H2[r0 + 4 * lg + i][col] = to_bf16(fmaxf(acc[i] + b, 0.0f));
  }
  __syncthreads();
  // layer 3: Y = H2 W3^T + b3 (3 of the 16 output columns are real)
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < HID / 32; ++kk)
      acc = mfma(ld8(&s.H2[r0 + lr][kk * 32 + 8 * lg]), ld8(&s.W3[lr][kk * 32 + 8 * lg]), acc);
    if (lr < OUT) {
      const float b = prm[OFF_B3 + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i) s.Y[r0 + 4 * lg + i][lr] = acc[i] + b;
    }
  }
  __syncthreads();
}

// Inference: Y[r * sr + c * sc] = y_r / |y_r|. Each block stages the weights once and then
// walks the row tiles blockIdx.x, blockIdx.x + gridDim.x, ... (the weights are 52 KB of LDS
// against 2.9 MFLOP per 64-row tile, so staging them per tile would dominate).
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ prm, const float* __restrict__ X,
                                                 int64_t B, float* __restrict__ Y, int64_t sr, int64_t sc) {
  extern __shared__ __align__(16) char smem_raw[];
  Smem& s = *reinterpret_cast<Smem*>(smem_raw);
  load_weights(s, prm);
  const int t = threadIdx.x;
  for (int64_t row0 = (int64_t)blockIdx.x * ROWS; row0 < B; row0 += (int64_t)gridDim.x * ROWS) {
    load_rows(s, X, B, row0);  // the previous tile's last reads of X and Y precede its final barrier
    __syncthreads();
    forward_wave(s, prm);  // ends with a barrier: Y is complete
    if (t < ROWS && row0 + t < B) {
      const float y0 = s.Y[t][0], y1 = s.Y[t][1], y2 = s.Y[t][2];
      const float nr = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
      const float inv = 1.0f / fmaxf(nr, 1e-30f);
      const int64_t g = row0 + t;
      Y[g * sr] = y0 * inv;
      Y[g * sr + sc] = y1 * inv;
      Y[g * sr + 2 * sc] = y2 * inv;
    }
    __syncthreads();  // Y read before the next tile's forward overwrites it
  }
}

__global__ void k_count_mask(const uint8_t* __restrict__ mask, int64_t B, int* __restrict__ nk) {
  __shared__ int lc;
  if (threadIdx.x == 0) lc = 0;
  __syncthreads();
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B; i += (int64_t)gridDim.x * blockDim.x)
    c += mask ? (mask[i] != 0) : 1;
  atomicAdd(&lc, c);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(nk, lc);
}

__global__ void k_zero_int(int* p) { *p = 0; }

// Forward + backward of one block of rows; writes the block's partial gradient (FP32) and
// partial loss sum (as float) to part[block][NPART].
__global__ __launch_bounds__(256) void k_mlp_train(const float* __restrict__ prm, const float* __restrict__ X,
                                                   const float* __restrict__ T, const uint8_t* __restrict__ mask,
                                                   int64_t B, const int* __restrict__ nkp,
                                                   float* __restrict__ part) {
  extern __shared__ __align__(16) char smem_raw[];
  Smem& s = *reinterpret_cast<Smem*>(smem_raw);
  SmemBwd& sb = *reinterpret_cast<SmemBwd*>(smem_raw + sizeof(Smem));
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  const int t = threadIdx.x, l = t & 63, w = t >> 6, lr = l % 16, lg = l / 16;
  load_weights(s, prm);
  load_rows(s, X, B, row0);
  __syncthreads();
  forward_wave(s, prm);
  float* out = part + (int64_t)blockIdx.x * NPART;
  const float inv_nk = 1.0f / (float)max(*nkp, 1);

  // d loss / d y = -(t - <yhat,t> yhat) / |y| / nk for kept rows
  double lossv = 0.0;
  if (t < ROWS) {
    const int64_t g = row0 + t;
    const bool keep = g < B && (!mask || mask[g] != 0);
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
    if (keep) {
      const float y0 = s.Y[t][0], y1 = s.Y[t][1], y2 = s.Y[t][2];
      const float nr = fmaxf(sqrtf(y0 * y0 + y1 * y1 + y2 * y2), 1e-30f);
      const float h0 = y0 / nr, h1 = y1 / nr, h2 = y2 / nr;
      const float t0 = T[g * 3], t1 = T[g * 3 + 1], t2 = T[g * 3 + 2];
      const float cs = h0 * t0 + h1 * t1 + h2 * t2;
      lossv = 1.0 - (double)cs;
      const float f = -inv_nk / nr;
      d0 = f * (t0 - cs * h0);
      d1 = f * (t1 - cs * h1);
      d2 = f * (t2 - cs * h2);
    }
    sb.DY[t][0] = d0;
    sb.DY[t][1] = d1;
    sb.DY[t][2] = d2;
  }
  // block loss sum (rows 0..63 live in wave 0)
  if (w == 0) {
    for (int o = 32; o > 0; o >>= 1) lossv += __shfl_xor(lossv, o, 64);
    if (l == 0) sb.loss[0] = lossv;
  }
  __syncthreads();

  // dW3[c][k] = sum_r dy[r][c] h2[r][k]; db3 = sum_r dy (FP32 VALU, tiny)
  for (int i = t; i < OUT * HID; i += blockDim.x) {
    const int c = i / HID, k = i % HID;
    float a = 0.f;
    for (int r = 0; r < ROWS; ++r) a = fmaf(sb.DY[r][c], from_bf16(s.H2[r][k]), a);
    out[OFF_W3 + i] = a;
  }
  if (t < OUT) {
    float a = 0.f;
    for (int r = 0; r < ROWS; ++r) a += sb.DY[r][t];
    out[OFF_B3 + t] = a;
  }
  // dz2 = (dy W3) * [h2 > 0]: thread -> column k = t % 128, rows (t / 128) * 32 + 0..31
  {
    const int k = t % HID, rh = t / HID;
    float bsum = 0.f;
    for (int r = rh * 32; r < rh * 32 + 32; ++r) {
      float v = sb.DY[r][0] * from_bf16(s.W3[0][k]) + sb.DY[r][1] * from_bf16(s.W3[1][k]) +
                sb.DY[r][2] * from_bf16(s.W3[2][k]);
      v = s.H2[r][k] != 0 ? v : 0.0f;
      bsum += v;
      sb.DZ2[r][k] = to_bf16(v);
    }
    sb.red[rh][k] = bsum;
  }
  __syncthreads();
  if (t < HID) out[OFF_B2 + t] = sb.red[0][t] + sb.red[1][t];
  // dW2[m][n] = sum_r dz2[r][m] h1[r][n]: 64 tiles of 16x16, 16 per wave, K = 64 rows
  for (int tile = w; tile < 64; tile += 4) {
    const int m0 = (tile / 8) * 16, n0 = (tile % 8) * 16;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < ROWS / 32; ++kk)
      acc = mfma(ld8s(&sb.DZ2[kk * 32 + 8 * lg][m0 + lr], HID), ld8s(&s.H1[kk * 32 + 8 * lg][n0 + lr], HID), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[OFF_W2 + (m0 + 4 * lg + i) * HID + n0 + lr] = acc[i];
  }
  // dh1 = dz2 W2 (row-parallel, K = 128): dz1 = dh1 * [h1 > 0]
  {
    const int r0 = 16 * w;
    for (int tn = 0; tn < HID / 16; ++tn) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < HID / 32; ++kk)
        acc = mfma(ld8(&sb.DZ2[r0 + lr][kk * 32 + 8 * lg]), ld8s(&s.W2[kk * 32 + 8 * lg][tn * 16 + lr], HID), acc);
      const int col = tn * 16 + lr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + 4 * lg + i;
        sb.DZ1[r][col] = to_bf16(s.H1[r][col] != 0 ? acc[i] : 0.0f);
      }
    }
  }
  __syncthreads();
  // db1 = sum_r dz1 with dz1 in FP32 (DZ1 holds it rounded to BF16 for the dW1 product),
  // recomputed per column as sum_m dz2[r][m] W2[m][k] on the rows where h1 > 0
  {
    const int k = t % HID, rh = t / HID;
    float bsum = 0.f;
    for (int r = rh * 32; r < rh * 32 + 32; ++r) {
      if (s.H1[r][k] == 0) continue;
      float v = 0.f;
      for (int m = 0; m < HID; ++m) v = fmaf(from_bf16(sb.DZ2[r][m]), from_bf16(s.W2[m][k]), v);
      bsum += v;
    }
    sb.red[rh][k] = bsum;
  }
  __syncthreads();
  if (t < HID) out[OFF_B1 + t] = sb.red[0][t] + sb.red[1][t];
  // dW1[m][n] = sum_r dz1[r][m] x[r][n], n < 48: 8 x 3 tiles
  for (int tile = w; tile < 24; tile += 4) {
    const int m0 = (tile / 3) * 16, n0 = (tile % 3) * 16;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < ROWS / 32; ++kk)
      acc = mfma(ld8s(&sb.DZ1[kk * 32 + 8 * lg][m0 + lr], HID), ld8s(&s.X[kk * 32 + 8 * lg][n0 + lr], INP), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[OFF_W1 + (m0 + 4 * lg + i) * IN + n0 + lr] = acc[i];
  }
  if (t == 0) out[NPAR] = (float)sb.loss[0];
}

// Fixed-order sum of the per-block partials: grad[p] = sum_b part[b][p]; loss = sum / nk.
__global__ void k_grad_reduce(const float* __restrict__ part, int nblk, const int* __restrict__ nkp,
                              float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NPAR) return;
  float s = 0.f, c = 0.f;
  for (int b = 0; b < nblk; ++b) {  // Kahan: thousands of blocks
    const float y = part[(int64_t)b * NPART + p] - c;
    const float tt = s + y;
    c = (tt - s) - y;
    s = tt;
  }
  if (p < NPAR)
    grad[p] = s;
  else if (loss)
    *loss = s / (float)max(*nkp, 1);
}

// Adam with bias correction (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
__global__ void k_adam(float* __restrict__ prm, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, float lr, float bc1, float bc2, float* __restrict__ gout) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  const float gi = g[p];
  const float a = 0.9f * m1[p] + 0.1f * gi;
  const float b = 0.999f * m2[p] + 0.001f * gi * gi;
  m1[p] = a;
  m2[p] = b;
  prm[p] -= lr * (a / bc1) / (sqrtf(b / bc2) + 1e-8f);
  if (gout) gout[p] = gi;
}

constexpr size_t kSmemFwd = sizeof(Smem);
constexpr size_t kSmemTrain = sizeof(Smem) + sizeof(SmemBwd);
static_assert(kSmemTrain <= 160 * 1024, "LDS budget");

}  // namespace

size_t mlp_ws_bytes(int64_t B) {
  Carver c(nullptr);
  c.take<float>((size_t)cdiv(B, ROWS) * NPART);
  c.take<float>(NPAR + 1);
  c.take<int>(1);
  return c.used;
}

static dwg_status set_lds_limits() {
  DWG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_fwd),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmemFwd));
  DWG_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_train),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmemTrain));
  return DWG_OK;
}

dwg_status mlp_forward(const float* params, const float* X, int64_t B, float* Y, int64_t sr, int64_t sc,
                       hipStream_t stream) {
  dwg_status st = set_lds_limits();
  if (st != DWG_OK) return st;
  // 1024 blocks (four per CU at one resident block per CU) stage the weights 1024 times at most
  const int64_t nblk = std::min<int64_t>(cdiv(B, ROWS), 1024);
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)nblk), dim3(256), kSmemFwd, stream, params, X, B, Y, sr, sc);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

dwg_status mlp_infer_run(const float* params, const float* X, int64_t B, float* Y, void*, size_t,
                         hipStream_t stream) {
  return mlp_forward(params, X, B, Y, 3, 1, stream);
}

dwg_status mlp_train_run(float* params, float* m1, float* m2, int64_t step, float lr, const float* X,
                         const float* T, const uint8_t* mask, int64_t B, float* grad_out, float* loss_out,
                         void* ws, size_t, hipStream_t stream) {
  dwg_status st = set_lds_limits();
  if (st != DWG_OK) return st;
  const int nblk = (int)cdiv(B, ROWS);
  Carver c(ws);
  float* part = c.take<float>((size_t)nblk * NPART);
  float* grad = c.take<float>(NPAR + 1);
  int* nk = c.take<int>(1);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, stream, nk);
  hipLaunchKernelGGL(k_count_mask, dim3((unsigned)std::min<int64_t>(cdiv(B, 256), 1024)), dim3(256), 0, stream,
                     mask, B, nk);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_mlp_train, dim3(nblk), dim3(256), kSmemTrain, stream, params, X, T, mask, B, nk, part);
  DWG_TRY_LAUNCH();
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)cdiv(NPAR + 1, 256)), dim3(256), 0, stream, part, nblk, nk,
                     grad, loss_out);
  DWG_TRY_LAUNCH();
  const float bc1 = 1.0f - powf(0.9f, (float)step);
  const float bc2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)cdiv(NPAR, 256)), dim3(256), 0, stream, params, m1, m2, grad, lr, bc1,
                     bc2, grad_out);
  DWG_TRY_LAUNCH();
  return DWG_OK;
}

}  // namespace dwg
