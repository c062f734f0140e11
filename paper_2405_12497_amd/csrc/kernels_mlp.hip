// Learned per-query nprobe (not part of the paper): features from the
// centroid-scoring and quantisation outputs, and a 96 -> 128 (ReLU) -> 32 MLP
// whose products run on BF16 MFMA with FP32 accumulation (inference and
// training), FP32 master weights and Adam.
#include "rbq_internal.hpp"
#include "rbq_mlp.hpp"

namespace rbq {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float x) {   // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ features
// Quantiser statistics of query q against its r-th nearest list, by one wave:
// b = ||q_r - c|| (raw vectors), v_l = min / b and v_r = max / b of the
// rotated residual q_rot - c_rot, and E[S_q] / (15 dp), the expectation of the
// randomized rounding's sum (unbiased, Theorem 3.3): the mean of
// (r_i - min) / (max - min) over the dp coordinates. out: {b, v_l, v_r, esq}.
__device__ __forceinline__ void list_stats(const FeatDev& f, int64_t q, int r, float* out) {
  const int lane = lane_id();
  const int navail = f.navail;
  const float* qr = f.q + q * f.dim;
  const float* qrot = f.qrot + q * f.dp;
  const int list = uniform_i32(f.probe[q * f.stride + min(r, navail - 1)]);
  const float* c = f.cent + (int64_t)list * f.dim;
  const float* crot = f.crot + (int64_t)list * f.dp;
  float acc = 0.f;
  for (int i = lane; i < f.dim; i += kWave) {
    const float d = qr[i] - c[i];
    acc = fmaf(d, d, acc);
  }
  const float b = sqrtf(wave_sum(acc));
  float rmin = __builtin_inff(), rmax = -__builtin_inff(), rsum = 0.f;
  for (int t = 0; t < f.W; ++t) {
    const float v = qrot[t * kWave + lane] - crot[t * kWave + lane];
    rmin = fminf(rmin, v);
    rmax = fmaxf(rmax, v);
    rsum += v;
  }
  rmin = wave_min(rmin);
  rmax = wave_max(rmax);
  rsum = wave_sum(rsum);
  const float range = rmax - rmin;
  const bool live = (b > 0.f) && (range > 0.f);
  if (lane == 0) {
    out[0] = b;
    out[1] = b > 0.f ? rmin / b : 0.f;
    out[2] = b > 0.f ? rmax / b : 0.f;
    out[3] = live ? (rsum - (float)f.dp * rmin) / (range * (float)f.dp) : 0.f;
  }
}

// Slots 0..63 of query q's features: log d_(1) and log(d_(j) / d_(1)) of its 64
// nearest squared centroid distances (probe_d, nearest first), by one wave.
__device__ __forceinline__ void distance_features(const FeatDev& f, int64_t q, float* out) {
  const int lane = lane_id();
  const float* dq = f.probe_d + q * f.stride;
  const float tiny = 1e-30f;
  const float l1 = logf(fmaxf(dq[0], tiny));
  const int j = lane;   // 64 lanes, 64 slots
  const float dj = fmaxf(dq[min(j, f.navail - 1)], tiny);
  out[j] = j == 0 ? l1 : logf(dj) - l1;
}

// Slots 64..95 from the 8 lists' statistics st[r][0..3] (lanes 0..31).
__device__ __forceinline__ void stats_features(const float* st, float* out) {
  const int lane = lane_id();
  if (lane < 4 * kMlpStats) {
    const int r = lane >> 2, k = lane & 3;
    const float b0 = fmaxf(st[0], 1e-30f);
    const float v = st[4 * r + k];
    out[kMlpNear + lane] = k == 0 ? v / b0 : v;
  }
}

// The 96 features of query q by one wave, written to out (global or LDS).
// probe_d: the query's 64 (or nlist) nearest squared centroid distances,
// nearest first; probe: their list ids.
__device__ __forceinline__ void query_features(const FeatDev& f, int64_t q, float* out) {
  distance_features(f, q, out);
  __shared__ float st_all[4][4 * kMlpStats];   // per wave of a 256-thread block
  float* st = st_all[(threadIdx.x >> 6) & 3];
  for (int r = 0; r < kMlpStats; ++r) list_stats(f, q, r, st + 4 * r);
  __builtin_amdgcn_wave_barrier();
  stats_features(st, out);
}

// One wave per (query, list rank < 8).
__global__ __launch_bounds__(256) void k_list_stats(FeatDev f) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= f.nq * kMlpStats) return;   // whole waves
  const int64_t q = w / kMlpStats;
  const int r = (int)(w - q * kMlpStats);
  list_stats(f, q, r, f.stats + w * 4);
}

// One wave per query.
__global__ __launch_bounds__(256) void k_features(FeatDev f) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= f.nq) return;
  query_features(f, q, f.feats + q * kMlpIn);
}

// ------------------------------------------------------------------ BF16 GEMM
// C[M x N] (+)= A[M x K] * B[K x N] with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn] (FP32 in memory, rounded to BF16 when staged),
// FP32 accumulation on v_mfma_f32_16x16x32_bf16. Block tile 64 x 64, four
// waves with a 32 x 32 quadrant each, K step 32.
constexpr int GT = 64, GK = 32;

__global__ __launch_bounds__(256) void k_gemm_bf16(const float* __restrict__ A, int64_t sam,
                                                   int64_t sak, const float* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, float* __restrict__ C,
                                                   int64_t ldc, int M, int N, int K, int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GT][GK + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GK + 8];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  for (int k0 = 0; k0 < K; k0 += GK) {
    u16x8 av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + lk + i;
      const int m = m0 + lr, n = n0 + lr;
      av[i] = to_bf16((m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.f);
      bv[i] = to_bf16((n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.f);
    }
    *reinterpret_cast<u16x8*>(&As[lr][lk]) = av;
    *reinterpret_cast<u16x8*>(&Bs[lr][lk]) = bv;
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + fr][fk]);
      b[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn + i * 16 + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  const int oc = lane & 15, orow = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 16 + oc;
      if (n >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + i * 16 + orow + e;
        if (m >= M) continue;
        float* c = C + (int64_t)m * ldc + n;
        *c = accumulate ? *c + acc[i][j][e] : acc[i][j][e];
      }
    }
}

// ------------------------------------------------------------------ elementwise
// A <- A + bias (pre-activation kept for the ReLU mask); H = max(A, 0).
__global__ void k_bias_relu(float* __restrict__ A, const float* __restrict__ bias, float* __restrict__ H,
                            int64_t rows, int cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const float a = A[i] + bias[i % cols];
  A[i] = a;
  H[i] = fmaxf(a, 0.f);
}

// Per row: z = Z + b2, p = softmax(z); loss += -log p_y; dZ = (p - onehot(y)) / n.
// One thread per row (32 logits). labels may be null (inference: Z <- z only).
__global__ void k_softmax_ce(float* __restrict__ Z, const float* __restrict__ b2,
                             const int32_t* __restrict__ y, int64_t n, float inv_n,
                             float* __restrict__ dZ, float* __restrict__ loss_sum) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (r < n) {
    float z[kMlpOut];
    float mx = -__builtin_inff();
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) {
      z[j] = Z[r * kMlpOut + j] + b2[j];
      mx = fmaxf(mx, z[j]);
    }
    float se = 0.f;
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) se += expf(z[j] - mx);
    const float lse = mx + logf(se);
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) Z[r * kMlpOut + j] = z[j];
    if (y) {
      const int yr = y[r];
      l = lse - z[yr];
#pragma unroll
      for (int j = 0; j < kMlpOut; ++j) dZ[r * kMlpOut + j] = (expf(z[j] - lse) - (j == yr ? 1.f : 0.f)) * inv_n;
    }
  }
  if (y && loss_sum) {
    l = wave_sum(l);
    if (lane_id() == 0) atomicAdd(loss_sum, l);
  }
}

__global__ void k_relu_grad(float* __restrict__ dH, const float* __restrict__ A, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total && !(A[i] > 0.f)) dH[i] = 0.f;
}

// out[c] = sum over rows of X[r][c]; one block per column, 256 threads.
__global__ void k_colsum(const float* __restrict__ X, int64_t rows, int cols, float* __restrict__ out) {
  __shared__ float part[4];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) s += X[r * cols + c];
  s = wave_sum(s);
  if (lane_id() == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = part[0] + part[1] + part[2] + part[3];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows(const float* __restrict__ X, const int32_t* __restrict__ y,
                              const int32_t* __restrict__ idx, int64_t n, int cols,
                              float* __restrict__ Xo, int32_t* __restrict__ yo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * cols) return;
  const int64_t r = i / cols, c = i - r * cols;
  const int64_t src = idx[r];
  Xo[i] = X[src * cols + c];
  if (c == 0) yo[r] = y[src];
}

// nprobe of the smallest bucket whose cumulative softmax of the logits z
// (stride zs) reaches `thr`, at most nprobe_max. Logits that are not all
// finite give nprobe_max (the fixed-nprobe fallback); *fallback tells which.
__device__ __forceinline__ int policy_pick(const float* z, int zs, float thr, int nprobe_max, bool* fallback) {
  float mx = -__builtin_inff();
  bool finite = true;
  for (int j = 0; j < kMlpOut; ++j) {
    const float v = z[j * zs];
    finite = finite && isfinite(v);
    mx = fmaxf(mx, v);
  }
  *fallback = !finite;
  if (!finite) return nprobe_max;
  float se = 0.f;
  for (int j = 0; j < kMlpOut; ++j) se += expf(z[j * zs] - mx);
  float cum = 0.f;
  int pick = kMlpOut - 1;
  for (int j = 0; j < kMlpOut; ++j) {
    cum += expf(z[j * zs] - mx) / se;
    if (cum >= thr - 1e-6f) {
      pick = j;
      break;
    }
  }
  return min(max(mlp_bucket_nprobe(pick), 1), nprobe_max);
}

__global__ void k_policy(const float* __restrict__ Z, int64_t n, float thr, int nprobe_max,
                         int32_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  bool fb;
  out[r] = policy_pick(Z + r * kMlpOut, 1, thr, nprobe_max, &fb);
}

// ------------------------------------------------------------------ fused inference
// Features, both layers and the policy of 16 queries per block of 4 waves,
// after the probe step: each wave computes the features of 4 queries into
// LDS, then layer 1 (X[16 x 96] W1 + b1, ReLU; wave w takes hidden tiles
// 2w, 2w + 1) and layer 2 (H[16 x 128] W2 + b2; waves 0 and 1 take one
// 16-wide output tile each) run on v_mfma_f32_16x16x32_bf16 with the operands
// rounded to BF16 as the training GEMM stages them, K in the same order, so
// the logits equal those of the separate forward pass. The weights come in
// fragment order (pack_mlp_fragments): one 16-byte load per lane per MFMA.
constexpr int kFuseQ = 16;
__global__ __launch_bounds__(256) void k_learned_front(FeatDev f, const u16x8* __restrict__ wfrag,
                                                       const float* __restrict__ w32, float thr,
                                                       int nprobe_max, int32_t* __restrict__ nprobe_out,
                                                       int32_t* __restrict__ fallback_out) {
  __shared__ float X[kFuseQ][kMlpIn];
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kFuseQ][kMlpHidden + 8];
  __shared__ float Z[kFuseQ][kMlpOut + 1];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t q0 = (int64_t)blockIdx.x * kFuseQ;
  // features: distances from the probe, list statistics from k_list_stats
  for (int r = wave; r < kFuseQ; r += 4) {
    if (q0 + r < f.nq) {
      distance_features(f, q0 + r, X[r]);
      stats_features(f.stats + (q0 + r) * 4 * kMlpStats, X[r]);
    } else {
      for (int j = lane; j < kMlpIn; j += kWave) X[r][j] = 0.f;
    }
  }
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  const int orow = (lane >> 4) * 4;
  // layer 1
  {
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int ks = 0; ks < kMlpIn / 32; ++ks) {
      u16x8 av;
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = to_bf16(X[fr][ks * 32 + fk + i]);
      const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int tile = 2 * wave + t;
        const bf16x8 b = __builtin_bit_cast(bf16x8, wfrag[(tile * (kMlpIn / 32) + ks) * kWave + lane]);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int col = (2 * wave + t) * 16 + fr;
      const float bias = w32[kMlpB1 + col];
#pragma unroll
      for (int e = 0; e < 4; ++e) Hs[orow + e][col] = to_bf16(fmaxf(acc[t][e] + bias, 0.f));
    }
  }
  __syncthreads();
  // layer 2
  if (wave < 2) {
    constexpr int kW1Frags = (kMlpHidden / 16) * (kMlpIn / 32) * kWave;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kMlpHidden / 32; ++ks) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Hs[fr][ks * 32 + fk]);
      const bf16x8 b = __builtin_bit_cast(bf16x8, wfrag[kW1Frags + (wave * (kMlpHidden / 32) + ks) * kWave + lane]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    const int col = wave * 16 + fr;
    const float bias = w32[kMlpB2 + col];
#pragma unroll
    for (int e = 0; e < 4; ++e) Z[orow + e][col] = acc[e] + bias;
  }
  __syncthreads();
  if (threadIdx.x < kFuseQ && q0 + threadIdx.x < f.nq) {
    const int r = threadIdx.x;
    bool fb;
    nprobe_out[q0 + r] = policy_pick(Z[r], 1, thr, nprobe_max, &fb);
    fallback_out[q0 + r] = fb ? 1 : 0;
  }
}

// Per-feature mean and 1/std (population), one block per feature.
__global__ void k_feat_stats(const float* __restrict__ X, int64_t rows, int cols, float* __restrict__ mu,
                             float* __restrict__ inv_sd) {
  __shared__ double part[2][4];
  const int c = blockIdx.x;
  double s = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const double v = X[r * cols + c];
    s += v;
    s2 += v * v;
  }
  s = wave_sum_d(s);
  s2 = wave_sum_d(s2);
  if (lane_id() == 0) {
    part[0][threadIdx.x >> 6] = s;
    part[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = (part[0][0] + part[0][1] + part[0][2] + part[0][3]) / (double)rows;
    const double v = (part[1][0] + part[1][1] + part[1][2] + part[1][3]) / (double)rows - m * m;
    mu[c] = (float)m;
    inv_sd[c] = (float)(v > 1e-20 ? 1.0 / sqrt(v) : 1.0);
  }
}

__global__ void k_standardize(const float* __restrict__ X, int64_t rows, int cols, const float* __restrict__ mu,
                              const float* __restrict__ inv_sd, float* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int c = (int)(i % cols);
  Y[i] = (X[i] - mu[c]) * inv_sd[c];
}

}  // namespace

hipError_t launch_feat_stats(const float* X, int64_t rows, int cols, float* mu, float* inv_sd, hipStream_t st) {
  hipLaunchKernelGGL(k_feat_stats, dim3(cols), dim3(256), 0, st, X, rows, cols, mu, inv_sd);
  return hipGetLastError();
}

hipError_t launch_standardize(const float* X, int64_t rows, int cols, const float* mu, const float* inv_sd,
                              float* Y, hipStream_t st) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, rows, cols, mu,
                     inv_sd, Y);
  return hipGetLastError();
}

hipError_t launch_features(const FeatDev& f, hipStream_t st) {
  if (f.nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((f.nq + 3) / 4)), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                            int64_t sbn, float* C, int64_t ldc, int M, int N, int K, bool accumulate,
                            hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((M + GT - 1) / GT, (N + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_bias_relu(float* A, const float* bias, float* H, int64_t rows, int cols, hipStream_t st) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bias_relu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, bias, H, rows, cols);
  return hipGetLastError();
}

hipError_t launch_softmax_ce(float* Z, const float* b2, const int32_t* y, int64_t n, float* dZ,
                             float* loss_sum, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_softmax_ce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Z, b2, y, n,
                     1.f / (float)n, dZ, loss_sum);
  return hipGetLastError();
}

hipError_t launch_relu_grad(float* dH, const float* A, int64_t total, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_grad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dH, A, total);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int64_t rows, int cols, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, st, X, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, const int32_t* y, const int32_t* idx, int64_t n, int cols,
                              float* Xo, int32_t* yo, hipStream_t st) {
  const int64_t t = n * cols;
  if (t <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, X, y, idx, n,
                     cols, Xo, yo);
  return hipGetLastError();
}

namespace {
// Bucket label of each query: the smallest bucket whose nprobe is at least
// need[i] (the last bucket when none is).
__global__ void k_bucket_labels(const int32_t* __restrict__ need, int64_t n, int32_t* __restrict__ labels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = need[i];
  int j = 0;
  while (j < kMlpOut - 1 && mlp_bucket_nprobe(j) < v) ++j;
  labels[i] = j;
}
}  // namespace

hipError_t launch_bucket_labels(const int32_t* need, int64_t n, int32_t* labels, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bucket_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, need, n, labels);
  return hipGetLastError();
}

hipError_t launch_list_stats(const FeatDev& f, hipStream_t st) {
  if (f.nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_list_stats, dim3((unsigned)((f.nq * kMlpStats + 3) / 4)), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_learned_front(const FeatDev& f, const uint16_t* wfrag, const float* w32, float thr,
                                int nprobe_max, int32_t* nprobe, int32_t* fallback, hipStream_t st) {
  if (f.nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_learned_front, dim3((unsigned)((f.nq + kFuseQ - 1) / kFuseQ)), dim3(256), 0, st, f,
                     reinterpret_cast<const u16x8*>(wfrag), w32, thr, nprobe_max, nprobe, fallback);
  return hipGetLastError();
}

hipError_t launch_policy(const float* Z, int64_t n, float thr, int nprobe_max, int32_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_policy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Z, n, thr, nprobe_max, out);
  return hipGetLastError();
}

}  // namespace rbq
