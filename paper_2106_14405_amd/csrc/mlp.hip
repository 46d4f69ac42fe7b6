// mlp.hip -- kernels of the learned warm start's network outside the step:
// batched inference (the same wave-level matrix-core routine the step runs),
// feature statistics, the loss gradient, Adam with global-norm clipping,
// the bf16 export of the weights, and the gather of logged new contacts.
//
// Network: 16 features -> 64 -> ReLU -> 64 -> ReLU -> 3, features z-scored
// with a training-set mean and std (std floored at 1e-6); inference rounds
// weights and layer inputs to bf16 and accumulates in fp32.  The loss is the
// mean squared error over all 3n outputs.  Flat fp32 parameter order:
//   w1 [64][16] | b1 [64] | w2 [64][64] | b2 [64] | w3 [3][64] | b3 [3]
// (row = output unit), 5443 values.  Every reduction here runs in a fixed
// order, so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mlp_mfma.h"
#include "sim_internal.h"

namespace rbs {

constexpr int kNP = 5443;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5440;
constexpr int kGradRows = 64;      // rows per gradient workgroup
constexpr int kGradThreads = 256;
constexpr int kStatBlocks = 256;

__device__ __forceinline__ float bf16r(float x) { return bf2f(f2bf(x)); }

// ---- inference --------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpParams M, const float* __restrict__ x, long n,
                                                          float* __restrict__ y) {
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  const bool ok = r < n;
  float f[16];
  const long rr = ok ? r : 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    float4 v = reinterpret_cast<const float4*>(x + 16 * rr)[k];
    f[4 * k] = v.x;
    f[4 * k + 1] = v.y;
    f[4 * k + 2] = v.z;
    f[4 * k + 3] = v.w;
  }
  float o[3];
  mlp_wave(M, f, ok, o);
  if (ok) {
    y[3 * r] = o[0];
    y[3 * r + 1] = o[1];
    y[3 * r + 2] = o[2];
  }
}

// ---- feature statistics (population mean and std, in double) -----------------
__global__ __launch_bounds__(256) void mlp_stats_partial(const float* __restrict__ x, long n, double* part) {
  // thread t of block b: feature t % 16, rows congruent to (b * 16 + t / 16) mod (kStatBlocks * 16)
  __shared__ double s1[256], s2[256];
  const int t = threadIdx.x, k = t & 15;
  double a = 0.0, b = 0.0;
  for (long r = (long)blockIdx.x * 16 + (t >> 4); r < n; r += (long)kStatBlocks * 16) {
    double v = x[16 * r + k];
    a += v;
    b += v * v;
  }
  s1[t] = a;
  s2[t] = b;
  __syncthreads();
  for (int w = 128; w >= 16; w >>= 1) {
    if (t < w) {
      s1[t] += s1[t + w];
      s2[t] += s2[t + w];
    }
    __syncthreads();
  }
  if (t < 16) {
    part[(long)blockIdx.x * 32 + t] = s1[t];
    part[(long)blockIdx.x * 32 + 16 + t] = s2[t];
  }
}

__global__ __launch_bounds__(64) void mlp_stats_final(const double* part, long n, float* mean, float* stdv) {
  const int k = threadIdx.x;
  if (k >= 16) return;
  double a = 0.0, b = 0.0;
  for (int j = 0; j < kStatBlocks; j++) {
    a += part[32 * j + k];
    b += part[32 * j + 16 + k];
  }
  double m = n > 0 ? a / (double)n : 0.0;
  double var = n > 0 ? b / (double)n - m * m : 0.0;
  mean[k] = (float)m;
  stdv[k] = (float)sqrt(var > 0.0 ? var : 0.0);
}

// ---- loss gradient --------------------------------------------------------------
// One workgroup per 64 rows; the forward rounds exactly where inference does,
// the backward runs in fp32 through the bf16-rounded weights (the gradient
// with respect to the rounded weight is applied to the fp32 master copy).
// Each workgroup writes its partial sums for all 5443 parameters and its
// partial loss; mlp_grad_reduce adds the partials in workgroup order.
struct GradLds {
  float z0[kGradRows][16];
  float a1[kGradRows][64];
  float a2[kGradRows][64];
  float d1[kGradRows][64];
  float d2[kGradRows][64];
  float dy[kGradRows][4];
  float w3[3][64];
  float loss[kGradThreads];
};

__global__ __launch_bounds__(kGradThreads) void mlp_grad_kernel(const float* __restrict__ prm,
                                                               const float* __restrict__ mean,
                                                               const float* __restrict__ stdv,
                                                               const float* __restrict__ x,
                                                               const float* __restrict__ tgt,
                                                               const int32_t* __restrict__ rows, long n,
                                                               float* __restrict__ part) {
  __shared__ GradLds S;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long r0 = (long)blockIdx.x * kGradRows;
  const float inv3n = 1.0f / (3.0f * (float)n);
  __shared__ long src[kGradRows];
  if (t < kGradRows) src[t] = r0 + t < n ? (rows ? (long)rows[r0 + t] : r0 + t) : -1;
  __syncthreads();
  // normalised, rounded features
  for (int e = t; e < kGradRows * 16; e += kGradThreads) {
    const int r = e >> 4, k = e & 15;
    float z = 0.f;
    if (src[r] >= 0) z = bf16r((x[16 * src[r] + k] - mean[k]) / fmaxf(stdv[k], 1e-6f));
    S.z0[r][k] = z;
  }
  for (int e = t; e < 192; e += kGradThreads) S.w3[e >> 6][e & 63] = bf16r(prm[kOffW3 + e]);
  __syncthreads();
  // layer 1: unit = lane, rows wv, wv+4, ...
  {
    float w[16];
#pragma unroll
    for (int i = 0; i < 16; i++) w[i] = bf16r(prm[kOffW1 + 16 * lane + i]);
    const float b = prm[kOffB1 + lane];
    for (int r = wv; r < kGradRows; r += 4) {
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < 16; i++) s = fmaf(w[i], S.z0[r][i], s);
      S.a1[r][lane] = bf16r(fmaxf(s + b, 0.f));
    }
  }
  __syncthreads();
  // layer 2
  {
    float w[64];
#pragma unroll
    for (int i = 0; i < 64; i++) w[i] = bf16r(prm[kOffW2 + 64 * lane + i]);
    const float b = prm[kOffB2 + lane];
    for (int r = wv; r < kGradRows; r += 4) {
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < 64; i++) s = fmaf(w[i], S.a1[r][i], s);
      S.a2[r][lane] = bf16r(fmaxf(s + b, 0.f));
    }
  }
  __syncthreads();
  // output layer, residuals and loss
  float lsum = 0.f;
  if (t < 3 * kGradRows) {
    const int r = t / 3, o = t - 3 * r;
    float dy = 0.f;
    if (src[r] >= 0) {
      float s = 0.f;
      for (int i = 0; i < 64; i++) s = fmaf(S.w3[o][i], S.a2[r][i], s);
      const float e = s + prm[kOffB3 + o] - tgt[3 * src[r] + o];
      lsum = e * e * inv3n;
      dy = 2.f * e * inv3n;
    }
    S.dy[r][o] = dy;
  }
  S.loss[t] = lsum;
  __syncthreads();
  // back through the output layer and the second ReLU
  for (int r = wv; r < kGradRows; r += 4) {
    float s = S.w3[0][lane] * S.dy[r][0] + S.w3[1][lane] * S.dy[r][1] + S.w3[2][lane] * S.dy[r][2];
    S.d2[r][lane] = S.a2[r][lane] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // back through layer 2 and the first ReLU: column `lane` of w2
  {
    float w[64];
#pragma unroll
    for (int o = 0; o < 64; o++) w[o] = bf16r(prm[kOffW2 + 64 * o + lane]);
    for (int r = wv; r < kGradRows; r += 4) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < 64; o++) s = fmaf(w[o], S.d2[r][o], s);
      S.d1[r][lane] = S.a1[r][lane] > 0.f ? s : 0.f;
    }
  }
  __syncthreads();
  // parameter partials, rows summed in order
  float* out = part + (long)blockIdx.x * (kNP + 1);
  for (int p = t; p < kNP; p += kGradThreads) {
    float g = 0.f;
    if (p < kOffB1) {
      const int o = p >> 4, i = p & 15;
      for (int r = 0; r < kGradRows; r++) g = fmaf(S.d1[r][o], S.z0[r][i], g);
    } else if (p < kOffW2) {
      const int o = p - kOffB1;
      for (int r = 0; r < kGradRows; r++) g += S.d1[r][o];
    } else if (p < kOffB2) {
      const int o = (p - kOffW2) >> 6, i = (p - kOffW2) & 63;
      for (int r = 0; r < kGradRows; r++) g = fmaf(S.d2[r][o], S.a1[r][i], g);
    } else if (p < kOffW3) {
      const int o = p - kOffB2;
      for (int r = 0; r < kGradRows; r++) g += S.d2[r][o];
    } else if (p < kOffB3) {
      const int o = (p - kOffW3) >> 6, i = (p - kOffW3) & 63;
      for (int r = 0; r < kGradRows; r++) g = fmaf(S.dy[r][o], S.a2[r][i], g);
    } else {
      const int o = p - kOffB3;
      for (int r = 0; r < kGradRows; r++) g += S.dy[r][o];
    }
    out[p] = g;
  }
  // partial loss: fixed-shape tree
  for (int w = kGradThreads / 2; w > 0; w >>= 1) {
    __syncthreads();
    if (t < w) S.loss[t] += S.loss[t + w];
  }
  if (t == 0) out[kNP] = S.loss[0];
}

__global__ __launch_bounds__(256) void mlp_grad_reduce(const float* __restrict__ part, int nblk,
                                                       float* __restrict__ grad, float* loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kNP) return;
  float g = 0.f;
  for (int b = 0; b < nblk; b++) g += part[(long)b * (kNP + 1) + p];
  if (p < kNP)
    grad[p] = g;
  else if (loss)
    *loss = g;
}

// ---- Adam with global-norm clipping (one workgroup) ------------------------------
__global__ __launch_bounds__(1024) void mlp_adam_kernel(float* __restrict__ prm, float* __restrict__ m1,
                                                        float* __restrict__ m2, const float* __restrict__ grad,
                                                        int step, float lr, float clip, double b1, double b2,
                                                        float eps, float* gnorm) {
  __shared__ float red[1024];
  const int t = threadIdx.x;
  float s = 0.f;
  for (int p = t; p < kNP; p += 1024) s = fmaf(grad[p], grad[p], s);
  red[t] = s;
  for (int w = 512; w > 0; w >>= 1) {
    __syncthreads();
    if (t < w) red[t] += red[t + w];
  }
  __syncthreads();
  const float norm = sqrtf(red[0]);
  const float sc = (clip > 0.f && norm > clip) ? clip / norm : 1.f;
  // 1 - beta and the bias corrections in double: 1 - 0.999f loses 1e-5 in fp32
  const double B1 = b1, B2 = b2;
  const float fb1 = (float)b1, fb2 = (float)b2;
  const float c1 = (float)(1.0 - pow(B1, (double)step)), c2 = (float)(1.0 - pow(B2, (double)step));
  const float o1 = (float)(1.0 - B1), o2 = (float)(1.0 - B2);
  for (int p = t; p < kNP; p += 1024) {
    const float g = grad[p] * sc;
    const float a = fb1 * m1[p] + o1 * g;
    const float v = fb2 * m2[p] + o2 * g * g;
    m1[p] = a;
    m2[p] = v;
    prm[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
  if (t == 0 && gnorm) *gnorm = norm;
}

// ---- bf16 export of the weights -----------------------------------------------
__global__ __launch_bounds__(256) void mlp_export_kernel(const float* __restrict__ prm, uint16_t* __restrict__ wbf,
                                                         float* __restrict__ bias) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kNP) return;
  const float v = prm[p];
  if (p < kOffB1)
    wbf[p] = (uint16_t)f2bf(v);
  else if (p < kOffW2)
    bias[p - kOffB1] = v;
  else if (p < kOffB2)
    wbf[1024 + p - kOffW2] = (uint16_t)f2bf(v);
  else if (p < kOffW3)
    bias[64 + p - kOffB2] = v;
  else if (p < kOffB3)
    wbf[5120 + p - kOffW3] = (uint16_t)f2bf(v);
  else
    bias[128 + p - kOffB3] = v;
}

// ---- gather of logged contacts ---------------------------------------------------
// The network warm-starts new contacts only (a persisting contact keeps its
// previous impulse), so the rows are the new contacts (feature 15 > 0) of
// the scenes whose flags are all clear.  Per-scene counts, an exclusive scan
// of them (one workgroup, fixed order), then an order-preserving copy.
__global__ __launch_bounds__(64) void gather_count(const int32_t* __restrict__ count,
                                                   const int32_t* __restrict__ flags, int CM, long scm,
                                                   const float* __restrict__ feat, int32_t* __restrict__ cnt) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int nc = flags[s] ? 0 : min(count[s], CM);
  const float* share = feat + 15 * scm + (long)s * CM;
  int c = 0;
  for (int q0 = 0; q0 < nc; q0 += 64) {
    const bool fresh = q0 + lane < nc && share[q0 + lane] > 0.f;
    c += __popcll(__ballot(fresh));
  }
  if (lane == 0) cnt[s] = c;
}

__global__ __launch_bounds__(1024) void gather_scan(const int32_t* __restrict__ cnt, int S,
                                                    int64_t* __restrict__ offs, long long* total) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (S + 1023) / 1024;
  const int s0 = t * per, s1 = min(S, s0 + per);
  int64_t a = 0;
  for (int s = s0; s < s1; s++) a += cnt[s];
  part[t] = a;
  __syncthreads();
  // Hillis-Steele inclusive scan
  for (int w = 1; w < 1024; w <<= 1) {
    int64_t v = t >= w ? part[t - w] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t o = t ? part[t - 1] : 0;
  for (int s = s0; s < s1; s++) {
    offs[s] = o;
    o += cnt[s];
  }
  if (t == 1023) *total = part[1023];
}

__global__ __launch_bounds__(64) void gather_rows(const int32_t* __restrict__ count,
                                                  const int32_t* __restrict__ flags, int CM, long scm,
                                                  const float* __restrict__ feat, const float* __restrict__ lam,
                                                  float inv_gdt, float tclip, const int64_t* __restrict__ offs,
                                                  float* __restrict__ x, float* __restrict__ tg, long cap) {
  const int s = blockIdx.x, lane = threadIdx.x;
  if (flags[s]) return;
  const int nc = min(count[s], CM);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  long base = offs[s];
  for (int q0 = 0; q0 < nc; q0 += 64) {
    const int q = q0 + lane;
    const long o = (long)s * CM + (q < nc ? q : 0);
    const bool fresh = q < nc && feat[15 * scm + o] > 0.f;
    const uint64_t m = __ballot(fresh);
    const long row = base + __popcll(m & below);
    base += __popcll(m);
    if (!fresh || row >= cap) continue;
    float f[16];
    for (int k = 0; k < 16; k++) f[k] = feat[k * scm + o];
    for (int k = 0; k < 16; k++) x[16 * row + k] = f[k];
    // target: the converged impulse in units of |g| dt / k_n, with k_n from
    // the features: w_A + w_B + (r_A x n) I_A^-1 (r_A x n) + (r_B x n) I_B^-1 (r_B x n)
    const float sc = (f[4] + f[5] + f[6] + f[7]) * inv_gdt;
    for (int k = 0; k < 3; k++) {
      float v = lam[k * scm + o] * sc;
      if (tclip > 0.f) v = fminf(fmaxf(v, -tclip), tclip);
      tg[3 * row + k] = v;
    }
  }
}

}  // namespace rbs

using namespace rbs;

extern "C" int rbs_mlp_forward(const MlpParams* M, const float* x, long n, float* y, hipStream_t st) {
  if (n <= 0) return 0;
  const long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, st, *M, x, n, y);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" size_t rbs_mlp_work_bytes(long n) {
  const long nblk = (n + kGradRows - 1) / kGradRows;
  size_t g = (size_t)nblk * (kNP + 1) * sizeof(float);
  size_t st = (size_t)kStatBlocks * 32 * sizeof(double);
  return g > st ? g : st;
}

extern "C" int rbs_mlp_stats(const float* x, long n, float* mean, float* stdv, void* work, hipStream_t st) {
  hipLaunchKernelGGL(mlp_stats_partial, dim3(kStatBlocks), dim3(256), 0, st, x, n, (double*)work);
  hipLaunchKernelGGL(mlp_stats_final, dim3(1), dim3(64), 0, st, (const double*)work, n, mean, stdv);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" int rbs_mlp_grad(const float* prm, const float* mean, const float* stdv, const float* x, const float* t,
                            const int32_t* rows, long n, float* grad, float* loss, void* work, hipStream_t st) {
  const long nblk = (n + kGradRows - 1) / kGradRows;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)nblk), dim3(kGradThreads), 0, st, prm, mean, stdv, x, t, rows,
                     n, (float*)work);
  hipLaunchKernelGGL(mlp_grad_reduce, dim3((kNP + 1 + 255) / 256), dim3(256), 0, st, (const float*)work, (int)nblk,
                     grad, loss);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---- the gradient without caller scratch -------------------------------------
// The per-workgroup partial sums of the gradient live in a file-scope device
// array instead of a caller workspace, for callers that cannot allocate.
// Each device holds its own copy; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name is a
// host-side stand-in, not a device address).
constexpr long kStaticGradRows = 16384;  // 256 workgroups of partial sums, 5.6 MB
constexpr int kMaxDevices = 64;
static __device__ __align__(256) float scratch[(kStaticGradRows / kGradRows) * (kNP + 1)];

static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per device.
static int static_scratch(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

extern "C" long rbs_mlp_grad_static_max_rows() { return kStaticGradRows; }

extern "C" int rbs_mlp_grad_static(const float* prm, const float* mean, const float* stdv, const float* x,
                                   const float* t, const int32_t* rows, long n, float* grad, float* loss,
                                   hipStream_t st) {
  if (n < 1 || n > kStaticGradRows) return -2;
  float* work = nullptr;
  if (static_scratch(&work) != 0) return -1;
  return rbs_mlp_grad(prm, mean, stdv, x, t, rows, n, grad, loss, work, st);
}

extern "C" int rbs_mlp_adam(float* prm, float* m1, float* m2, const float* grad, int step, float lr, float clip,
                            float* gnorm, hipStream_t st) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(1), dim3(1024), 0, st, prm, m1, m2, grad, step, lr, clip, 0.9, 0.999,
                     1e-8f, gnorm);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" int rbs_mlp_export(const float* prm, uint16_t* wbf, float* bias, hipStream_t st) {
  hipLaunchKernelGGL(mlp_export_kernel, dim3((kNP + 255) / 256), dim3(256), 0, st, prm, wbf, bias);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" int rbs_gather(const int32_t* count, const int32_t* flags, int S, int CM, long scm, const float* feat,
                          const float* lam, float inv_gdt, float tclip, int64_t* offs, int32_t* cnt, float* x,
                          float* t, long cap, long long* total, hipStream_t st) {
  hipLaunchKernelGGL(gather_count, dim3(S), dim3(64), 0, st, count, flags, CM, scm, feat, cnt);
  hipLaunchKernelGGL(gather_scan, dim3(1), dim3(1024), 0, st, (const int32_t*)cnt, S, offs, total);
  hipLaunchKernelGGL(gather_rows, dim3(S), dim3(64), 0, st, count, flags, CM, scm, feat, lam, inv_gdt, tclip,
                     (const int64_t*)offs, x, t, cap);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
