// Rotation and centroid-scoring GEMMs, and the index-time encoder.
//
// Rows are vectors, so P^T v (the inverse rotation of Sec. 3.1.3 / 3.3) is the
// row product v^T P and a batch of rotations is Y = X * P.
#include "rbq_internal.hpp"

namespace rbq {

// ---------------------------------------------------------------- FP32 tiled GEMM
// 64 x 64 output tile per 256-thread block, 4 x 4 per thread, K step 16.
// MODE 0: Y = (A - sub[sel]) * B.  MODE 1: centroid distances
//   Y[m][n] = an[m] + bn[n] - 2 * (A * B)[m][n], clamped at 0.
namespace {
constexpr int TM = 64, TN = 64, TK = 16;

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ A, int64_t lda,
                                                  const float* __restrict__ sub,
                                                  const int32_t* __restrict__ sel,
                                                  const float* __restrict__ B, int64_t ldb,
                                                  float* __restrict__ Y, int64_t ldy, int64_t M,
                                                  int N, int K, const float* __restrict__ an,
                                                  const float* __restrict__ bn) {
  __shared__ float As[TK][TM + 4];
  __shared__ float Bs[TK][TN + 4];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * TM;
  const int n0 = blockIdx.y * TN;
  float acc[4][4] = {};
  // A tile loader: 64 rows x 16 k, thread loads 4 consecutive k of one row
  const int la_r = tid >> 2, la_k = (tid & 3) * 4;
  // B tile loader: 16 k x 64 n, thread loads 4 consecutive n of one k
  const int lb_k = tid >> 4, lb_n = (tid & 15) * 4;
  const int64_t am = m0 + la_r;
  const float* arow = (am < M) ? A + am * lda : nullptr;
  const float* srow = (am < M && sel) ? sub + (int64_t)sel[am] * K : nullptr;
  for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = k0 + la_k + i;
      float v = 0.f;
      if (arow && kk < K) {
        v = arow[kk];
        if (srow) v -= srow[kk];
      }
      As[la_k + i][la_r] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = k0 + lb_k, nn = n0 + lb_n + i;
      Bs[lb_k][lb_n + i] = (kk < K && nn < N) ? B[(int64_t)kk * ldb + nn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j];
      if (MODE == 1) v = fmaxf(an[m] + bn[n] - 2.f * v, 0.f);
      Y[m * ldy + n] = v;
    }
  }
}

// 128 x 128 output tile, 8 x 8 per thread (rows ty*4 + {0..3, 64..67}, cols
// tx*4 + {0..3, 64..67}), K step 8. Same modes as k_gemm_f32.
constexpr int BM = 128, BN = 128, BKF = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_f32_big(const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ sub,
                                                      const int32_t* __restrict__ sel,
                                                      const float* __restrict__ B, int64_t ldb,
                                                      float* __restrict__ Y, int64_t ldy, int64_t M,
                                                      int N, int K, const float* __restrict__ an,
                                                      const float* __restrict__ bn) {
  __shared__ __attribute__((aligned(16))) float As[BKF][BM];
  __shared__ __attribute__((aligned(16))) float Bs[BKF][BN];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  float acc[8][8] = {};
  // A loader: 128 rows x 8 k: thread loads 4 consecutive k of row tid>>1
  const int la_r = tid >> 1, la_k = (tid & 1) * 4;
  const int64_t am = m0 + la_r;
  const float* arow = (am < M) ? A + am * lda : nullptr;
  const float* srow = (am < M && sel) ? sub + (int64_t)sel[am] * K : nullptr;
  // B loader: 8 k x 128 n: thread loads 4 consecutive n of k = tid>>5
  const int lb_k = tid >> 5, lb_n = (tid & 31) * 4;
  for (int k0 = 0; k0 < K; k0 += BKF) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = k0 + la_k + i;
      float v = 0.f;
      if (arow && kk < K) {
        v = arow[kk];
        if (srow) v -= srow[kk];
      }
      As[la_k + i][la_r] = v;
    }
    {
      const int kk = k0 + lb_k;
      const int nn = n0 + lb_n;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kk < K) {
        const float* brow = B + (int64_t)kk * ldb;
        if (nn + 3 < N && ((ldb & 3) == 0)) {
          v = *reinterpret_cast<const float4*>(brow + nn);
        } else {
          if (nn < N) v.x = brow[nn];
          if (nn + 1 < N) v.y = brow[nn + 1];
          if (nn + 2 < N) v.z = brow[nn + 2];
          if (nn + 3 < N) v.w = brow[nn + 3];
        }
      }
      *reinterpret_cast<float4*>(&Bs[lb_k][lb_n]) = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BKF; ++kk) {
      const float4 a0 = *reinterpret_cast<const float4*>(&As[kk][ty * 4]);
      const float4 a1 = *reinterpret_cast<const float4*>(&As[kk][ty * 4 + 64]);
      const float4 b0 = *reinterpret_cast<const float4*>(&Bs[kk][tx * 4]);
      const float4 b1 = *reinterpret_cast<const float4*>(&Bs[kk][tx * 4 + 64]);
      const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const float b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t m = m0 + ty * 4 + (i & 3) + (i >> 2) * 64;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = n0 + tx * 4 + (j & 3) + (j >> 2) * 64;
      if (n >= N) continue;
      float v = acc[i][j];
      if (MODE == 1) v = fmaxf(an[m] + bn[n] - 2.f * v, 0.f);
      Y[m * ldy + n] = v;
    }
  }
}

__global__ void k_rownorm(const float* __restrict__ X, int64_t M, int K, float* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= M) return;
  float s = 0.f;
  for (int i = lane_id(); i < K; i += kWave) {
    const float v = X[row * K + i];
    s = fmaf(v, v, s);
  }
  s = wave_sum(s);
  if (lane_id() == 0) out[row] = s;
}

// ---------------------------------------------------------------- split-BF16 MFMA GEMM
// Y = X * P with X split per element as hi = bf16(x), lo = bf16(x - hi) and P
// given as transposed BF16 hi/lo planes Bt[n][k]. Each 16x16 output block sums
// hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16 (FP32 accumulation).
// Block tile 64 x 64, K step 32, 4 waves each owning a 32 x 32 quadrant.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float x) {   // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int BK = 32;

__global__ __launch_bounds__(256) void k_gemm_bf16x3(const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ sub,
                                                     const int32_t* __restrict__ sel,
                                                     const uint16_t* __restrict__ Bhi,
                                                     const uint16_t* __restrict__ Blo,
                                                     float* __restrict__ Y, int64_t ldy, int64_t M,
                                                     int N, int K) {
  // k-contiguous rows, padded by 8 elements so 16-byte reads stay aligned
  __shared__ __attribute__((aligned(16))) uint16_t Ah[TM][BK + 8], Al[TM][BK + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[TN][BK + 8], Bl[TN][BK + 8];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.x * TM;
  const int n0 = blockIdx.y * TN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A loader: row tid>>2, 8 consecutive k starting at (tid&3)*8
  const int la_r = tid >> 2, la_k = (tid & 3) * 8;
  const int64_t am = m0 + la_r;
  const float* arow = (am < M) ? A + am * lda : nullptr;
  const float* srow = (am < M && sel) ? sub + (int64_t)sel[am] * K : nullptr;
  // B loader: n row tid>>2, 8 consecutive k
  const int lb_n = tid >> 2, lb_k = (tid & 3) * 8;
  const int bn = n0 + lb_n;
  for (int k0 = 0; k0 < K; k0 += BK) {
    u16x8 hv, lv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int kk = k0 + la_k + i;
      float v = 0.f;
      if (arow && kk < K) {
        v = arow[kk];
        if (srow) v -= srow[kk];
      }
      const uint16_t h = f2bf(v);
      hv[i] = h;
      lv[i] = f2bf(v - bf2f(h));
    }
    *reinterpret_cast<u16x8*>(&Ah[la_r][la_k]) = hv;
    *reinterpret_cast<u16x8*>(&Al[la_r][la_k]) = lv;
    u16x8 bh = {}, bl = {};
    if (bn < N) {
      const int64_t o = (int64_t)bn * K + k0 + lb_k;
      if (k0 + lb_k + 8 <= K && (o & 7) == 0) {
        bh = *reinterpret_cast<const u16x8*>(Bhi + o);
        bl = *reinterpret_cast<const u16x8*>(Blo + o);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (k0 + lb_k + i < K) {
            bh[i] = Bhi[o + i];
            bl[i] = Blo[o + i];
          }
        }
      }
    }
    *reinterpret_cast<u16x8*>(&Bh[lb_n][lb_k]) = bh;
    *reinterpret_cast<u16x8*>(&Bl[lb_n][lb_k]) = bl;
    __syncthreads();
    // operand fragments: row (or column) lane%16, k = (lane/16)*8 .. +7
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 ah[2], al[2], bh2[2], bl2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[wm + i * 16 + fr][fk]);
      al[i] = *reinterpret_cast<const bf16x8*>(&Al[wm + i * 16 + fr][fk]);
      bh2[i] = *reinterpret_cast<const bf16x8*>(&Bh[wn + i * 16 + fr][fk]);
      bl2[i] = *reinterpret_cast<const bf16x8*>(&Bl[wn + i * 16 + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh2[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl2[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh2[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  // output fragment: column lane%16, rows (lane/16)*4 + 0..3
  const int oc = lane & 15, orow = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 16 + oc;
      if (n >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm + i * 16 + orow + e;
        if (m < M) Y[m * ldy + n] = acc[i][j][e];
      }
    }
}

// ---------------------------------------------------------------- FP64 rotation (centroids)
__global__ void k_rotate_f64(const float* __restrict__ X, int64_t M, int K,
                             const double* __restrict__ P, int N, float* __restrict__ Y) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = blockIdx.y;
  if (n >= N || m >= M) return;
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += (double)X[m * K + k] * P[(int64_t)k * N + n];
  Y[m * N + n] = (float)s;
}

// ---------------------------------------------------------------- encoder (Sec. 3.1.3, Alg. 1)
// One wave per vector: bits = [y_i > 0] with y = (o_r - c) P; ||o_r - c|| from
// the raw residual; <o_bar, o> = sum |y_i| / (sqrt(D) ||o_r - c||)  (the code
// takes the signs of P^{-1} o, so <x_bar, P^{-1} o> is the scaled l1 norm).
__global__ __launch_bounds__(256) void k_encode(const float* __restrict__ Y, int64_t m, int W,
                                                const float* __restrict__ raw,
                                                const float* __restrict__ cent,
                                                const int32_t* __restrict__ list_of, int dim,
                                                int64_t pos0, uint64_t* __restrict__ codes,
                                                float2* __restrict__ fac) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  const int lane = lane_id();
  const int64_t pos = pos0 + r;
  const int list = list_of[pos];
  double a2 = 0.0;
  for (int i = lane; i < dim; i += kWave) {
    const double d = (double)raw[pos * dim + i] - (double)cent[(int64_t)list * dim + i];
    a2 += d * d;
  }
  a2 = wave_sum_d(a2);
  const double a = sqrt(a2);
  const int dp = W * 64;
  double sabs = 0.0;
  for (int t = 0; t < W; ++t) {
    const float y = Y[r * dp + t * 64 + lane];
    sabs += fabs((double)y);
    const uint64_t word = (a > 0.0) ? __ballot(y > 0.f) : 0ull;
    if (lane == 0) codes[code_word_index(pos, t, W)] = word;
  }
  sabs = wave_sum_d(sabs);
  if (lane == 0) {
    const double ipo = (a > 0.0) ? sabs / (sqrt((double)dp) * a) : 1.0;
    fac[pos] = make_float2((float)a, (float)fmin(ipo, 1.0));
  }
}
}  // namespace

hipError_t launch_gemm_f32(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                           const float* B, int64_t ldb, float* Y, int64_t ldy, int64_t M, int N,
                           int K, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (M >= 2048) {
    dim3 grid((unsigned)((M + BM - 1) / BM), (N + BN - 1) / BN);
    hipLaunchKernelGGL(k_gemm_f32_big<0>, grid, dim3(256), 0, st, A, lda, sub, sel, B, ldb, Y, ldy,
                       M, N, K, nullptr, nullptr);
  } else {
    dim3 grid((unsigned)((M + TM - 1) / TM), (N + TN - 1) / TN);
    hipLaunchKernelGGL(k_gemm_f32<0>, grid, dim3(256), 0, st, A, lda, sub, sel, B, ldb, Y, ldy, M,
                       N, K, nullptr, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_bf16x3(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                              const uint16_t* Bhi, const uint16_t* Blo, float* Y, int64_t ldy,
                              int64_t M, int N, int K, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + TM - 1) / TM), (N + TN - 1) / TN);
  hipLaunchKernelGGL(k_gemm_bf16x3, grid, dim3(256), 0, st, A, lda, sub, sel, Bhi, Blo, Y, ldy, M,
                     N, K);
  return hipGetLastError();
}

hipError_t launch_centroid_dist(const float* Q, int64_t nq, int dim, const float* Ct,
                                const float* cn, int nlist, float* D, hipStream_t st) {
  // ||q||^2 is written into the tail of D's first row block scratch: use a
  // separate small buffer carved after D (caller provides nq floats there).
  float* qn = D + nq * (int64_t)nlist;
  hipLaunchKernelGGL(k_rownorm, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, Q, nq, dim, qn);
  if (nq >= 256 && nlist >= 128) {
    dim3 grid((unsigned)((nq + BM - 1) / BM), (nlist + BN - 1) / BN);
    hipLaunchKernelGGL(k_gemm_f32_big<1>, grid, dim3(256), 0, st, Q, (int64_t)dim, nullptr, nullptr,
                       Ct, (int64_t)nlist, D, (int64_t)nlist, nq, nlist, dim, qn, cn);
  } else {
    dim3 grid((unsigned)((nq + TM - 1) / TM), (nlist + TN - 1) / TN);
    hipLaunchKernelGGL(k_gemm_f32<1>, grid, dim3(256), 0, st, Q, (int64_t)dim, nullptr, nullptr, Ct,
                       (int64_t)nlist, D, (int64_t)nlist, nq, nlist, dim, qn, cn);
  }
  return hipGetLastError();
}

hipError_t launch_rotate_f64(const float* X, int64_t M, int K, const double* P, int N, float* Y,
                             hipStream_t st) {
  if (M <= 0) return hipSuccess;
  dim3 grid((N + 255) / 256, (unsigned)M);
  hipLaunchKernelGGL(k_rotate_f64, grid, dim3(256), 0, st, X, M, K, P, N, Y);
  return hipGetLastError();
}

hipError_t launch_encode(const float* Y, int64_t m, int W, const float* raw, const float* cent,
                         const int32_t* list_of, int dim, int64_t pos0, uint64_t* codes,
                         float2* fac, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, Y, m, W, raw, cent,
                     list_of, dim, pos0, codes, fac);
  return hipGetLastError();
}

}  // namespace rbq
