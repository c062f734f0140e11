// Rotation and centroid-scoring GEMMs, and the index-time encoder.
//
// Rows are vectors, so P^T v (the inverse rotation of Sec. 3.1.3 / 3.3) is the
// row product v^T P and a batch of rotations is Y = X * P.
#include "rbq_internal.hpp"

namespace rbq {

// ---------------------------------------------------------------- FP32 GEMM modes
// MODE 0: Y = (A - sub[sel]) * B.  MODE 1: centroid distances
//   Y[m][n] = ||A[m]||^2 + bn[n] - 2 * (A * B)[m][n], clamped at 0 (the row
//   norms are summed from the A tiles as they pass through), and, when gmin
//   is given (128-wide tiles only), gmin[m][g] = the minimum of Y[m][c] over
//   the 16 columns c of group g: c = 64 (g / 4) + 4 (g % 4) + 16 j + e,
//   j, e < 4, c < N (ceil(N / 64) * 4 groups per row). A group is the 16
//   values one lane holds of a row of its wave's 64-column tile.
namespace {

// ---------------------------------------------------------------- FP32 MFMA GEMM
// Same modes on the matrix cores (v_mfma_f32_16x16x4_f32: FP32 products, FP32
// accumulation). Four waves in a 2 x 2 grid, each owning WT x WT blocks of
// 16 x 16 outputs, so the block tile is 32 WT square; K steps of 16. In MFMA
// sub-step s, lane l contributes k = 4 s + l / 16 of its row (A, LDS [m][k])
// and column (B, LDS [k][n]); the B rows are padded by 16 floats so the four
// k rows a wave reads fall in different banks. The instruction is given the
// B fragment first, so it forms the transposed block and lane l ends with row
// l % 16 and the four adjacent columns 4 (l / 16) .. + 3: one 16-byte store
// per block instead of four scattered 4-byte ones.
typedef float f32x4v __attribute__((ext_vector_type(4)));
constexpr int MKS = 16, MKP = MKS + 4;

// One product (or centroid-distance) problem of the FP32 MFMA GEMM.
struct GemmJob {
  const float* A;
  int64_t lda;
  const float* sub;
  const int32_t* sel;
  const float* B;
  int64_t ldb;
  float* Y;
  int64_t ldy;
  int64_t M;
  int N, K;
  const float* bn;
  float* gmin;
};

// LDS of one block: double-buffered A and B tiles, and MODE 1's row norms.
template <int WT>
struct GemmLds {
  static constexpr int BT = 32 * WT;
  float As[2][BT][MKP];
  float Bs[2][MKS][BT + 16];
  float an[BT];
};

// Output tile (tm, tn) of job j (rows tm * 32 WT.., columns tn * 32 WT..).
template <int MODE, int WT>
__device__ __forceinline__ void gemm_tile(const GemmJob& j, int64_t tm, int tn, GemmLds<WT>& L) {
  constexpr int BT = 32 * WT;        // block tile (rows and columns)
  constexpr int NLD = BT * 4 / 256;  // float4 loads per thread per operand and K step
  const float* __restrict__ A = j.A;
  const int64_t lda = j.lda;
  const float* __restrict__ sub = j.sub;
  const int32_t* __restrict__ sel = j.sel;
  const float* __restrict__ B = j.B;
  const int64_t ldb = j.ldb;
  float* __restrict__ Y = j.Y;
  const int64_t ldy = j.ldy, M = j.M;
  const int N = j.N, K = j.K;
  const float* __restrict__ bn = j.bn;
  float* __restrict__ gmin = j.gmin;
  auto& As = L.As;
  auto& Bs = L.Bs;
  float* an_s = L.an;   // ||A[m]||^2 of the tile's rows (MODE 1)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = tm * BT;
  const int n0 = tn * BT;
  const int wm = (wave >> 1) * (16 * WT), wn = (wave & 1) * (16 * WT);
  f32x4v acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = f32x4v{0.f, 0.f, 0.f, 0.f};
  const bool a_vec = (lda & 3) == 0 && (K & 3) == 0;   // rows (and centroid rows) 16-byte aligned
  const bool b_vec = (ldb & 3) == 0;
  // tiles entirely inside the matrices take unconditional float4 loads
  const bool interior = a_vec && b_vec && m0 + BT <= M && n0 + BT <= N;
  const float* arow[NLD];
  const float* srow[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int64_t m = m0 + ((tid + 256 * u) >> 2);
    arow[u] = m < M ? A + m * lda : nullptr;
    srow[u] = (m < M && sel) ? sub + (int64_t)sel[m] * K : nullptr;
  }
  float4 ra[NLD], rb[NLD];
  auto fetch = [&](int k0) {
    if (interior && k0 + MKS <= K) {
#pragma unroll
      for (int u = 0; u < NLD; ++u) {
        const int f = tid + 256 * u;
        ra[u] = *reinterpret_cast<const float4*>(arow[u] + k0 + (f & 3) * 4);
        rb[u] = *reinterpret_cast<const float4*>(B + (int64_t)(k0 + f / (BT / 4)) * ldb + n0 + (f % (BT / 4)) * 4);
      }
      if (sel) {
        float4 c[NLD];
#pragma unroll
        for (int u = 0; u < NLD; ++u) c[u] = *reinterpret_cast<const float4*>(srow[u] + k0 + ((tid + 256 * u) & 3) * 4);
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
          ra[u].x -= c[u].x;
          ra[u].y -= c[u].y;
          ra[u].z -= c[u].z;
          ra[u].w -= c[u].w;
        }
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int f = tid + 256 * u;
      const int kq = (f & 3) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (arow[u]) {
        const int k = k0 + kq;
        float t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) t[i] = (k + i < K) ? arow[u][k + i] - (srow[u] ? srow[u][k + i] : 0.f) : 0.f;
        v = make_float4(t[0], t[1], t[2], t[3]);
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int f = tid + 256 * u;
      const int kr = f / (BT / 4), nq = (f % (BT / 4)) * 4;
      const int k = k0 + kr, n = n0 + nq;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k < K) {
        const float* brow = B + (int64_t)k * ldb;
        if (n < N) v.x = brow[n];
        if (n + 1 < N) v.y = brow[n + 1];
        if (n + 2 < N) v.z = brow[n + 2];
        if (n + 3 < N) v.w = brow[n + 3];
      }
      rb[u] = v;
    }
  };
  // MODE 1: thread f accumulates the squares of its four columns of row f / 4
  // as each A tile is stashed; the row's four threads (f % 4) add up at the end
  float asq[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) asq[u] = 0.f;
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int f = tid + 256 * u;
      *reinterpret_cast<float4*>(&As[buf][f >> 2][(f & 3) * 4]) = ra[u];
      *reinterpret_cast<float4*>(&Bs[buf][f / (BT / 4)][(f % (BT / 4)) * 4]) = rb[u];
      if (MODE == 1) {
        asq[u] = fmaf(ra[u].x, ra[u].x, asq[u]);
        asq[u] = fmaf(ra[u].y, ra[u].y, asq[u]);
        asq[u] = fmaf(ra[u].z, ra[u].z, asq[u]);
        asq[u] = fmaf(ra[u].w, ra[u].w, asq[u]);
      }
    }
  };
  // double-buffered K steps: the next step's global loads are in flight
  // during this step's MFMAs and land in the other LDS buffer; one barrier
  // per step
  fetch(0);
  stash(0);
  __syncthreads();
  const int fr = lane & 15, fg = lane >> 4;
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += MKS) {
    const bool more = k0 + MKS < K;
    if (more) fetch(k0 + MKS);
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) {
      float a[WT], b[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) a[i] = As[buf][wm + i * 16 + fr][4 * ss + fg];
#pragma unroll
      for (int j = 0; j < WT; ++j) b[j] = Bs[buf][4 * ss + fg][wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (MODE == 1) {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      float v = asq[u];
      v += __shfl_xor(v, 1, kWave);
      v += __shfl_xor(v, 2, kWave);
      if ((tid & 3) == 0) an_s[(tid + 256 * u) >> 2] = v;
    }
    __syncthreads();
  }
  // output block (i, j): lane holds row fr, columns 4 fg .. 4 fg + 3
  const bool y_vec = (ldy & 3) == 0 && ((uintptr_t)Y & 15) == 0;
  const bool want_gmin = MODE == 1 && WT == 4 && gmin != nullptr && n0 + wn < N;
  const int G = ((N + 63) >> 6) * 4;
#pragma unroll
  for (int i = 0; i < WT; ++i) {
    const int64_t m = m0 + wm + i * 16 + fr;
    if (m >= M) continue;
    const float am = MODE == 1 ? an_s[wm + i * 16 + fr] : 0.f;
    float gv = __builtin_inff();
#pragma unroll
    for (int j = 0; j < WT; ++j) {
      const int n = n0 + wn + j * 16 + 4 * fg;
      f32x4v o = acc[i][j];
      if (MODE == 1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          o[e] = fmaxf(am + bn[min(n + e, N - 1)] - 2.f * o[e], 0.f);
          gv = (n + e < N) ? fminf(gv, o[e]) : gv;
        }
      }
      if (n >= N) continue;
      float* y = Y + m * ldy + n;
      if (y_vec && n + 3 < N) {
        *reinterpret_cast<f32x4v*>(y) = o;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < N) y[e] = o[e];
      }
    }
    if (want_gmin) gmin[m * G + ((n0 + wn) >> 6) * 4 + fg] = gv;
  }
}

template <int MODE, int WT>
__global__ __launch_bounds__(256) void k_gemm_f32_mfma(GemmJob j) {
  __shared__ __attribute__((aligned(16))) GemmLds<WT> L;
  gemm_tile<MODE, WT>(j, blockIdx.x, blockIdx.y, L);
}

// The query rotation (MODE 0) and the centroid distances (MODE 1) in one
// launch: they read the same queries and are independent, so the rotation's
// few tiles run beside the distance tiles instead of before them. Tiles are
// numbered row tile fastest; the rotation's come first.
__global__ __launch_bounds__(256) void k_gemm_rot_cdist(GemmJob rot, GemmJob cd, int rot_tm, int rot_tiles,
                                                        int cd_tm) {
  __shared__ __attribute__((aligned(16))) GemmLds<4> L;
  const int t = blockIdx.x;
  if (t < rot_tiles)
    gemm_tile<0, 4>(rot, t % rot_tm, t / rot_tm, L);
  else
    gemm_tile<1, 4>(cd, (t - rot_tiles) % cd_tm, (t - rot_tiles) / cd_tm, L);
}

// ---------------------------------------------------------------- few-query centroid distances
// MODE 1 for at most MQ <= 8 query rows, as dot products over the transposed
// centroids B = Ct [K][N] (a GEMM tile would leave most of its rows empty and
// walk K in short steps). Block b covers columns 64 b .. 64 b + 63, one per
// lane; its 16 waves split K into 16 slices, each lane summing its column's
// MQ products over its wave's slice (each load a contiguous 256-byte row piece
// per wave), and the wave partials (and the slices' squared row norms) are
// added in wave order.
constexpr int kCdThreads = 1024, kCdWaves = kCdThreads / kWave;

template <int MQ>
__global__ __launch_bounds__(kCdThreads) void k_cdist_few(const float* __restrict__ A, int64_t lda, int64_t M,
                                                          const float* __restrict__ B, int64_t ldb, int N, int K,
                                                          const float* __restrict__ bn, float* __restrict__ Y,
                                                          int64_t ldy) {
  __shared__ float part[kCdWaves][MQ][kWave];
  __shared__ float nrm[kCdWaves][MQ];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = blockIdx.x * kWave + lane;
  const int nc = min(n, N - 1);
  const int ks = (K + kCdWaves - 1) / kCdWaves;
  const int k0 = min(K, wave * ks), k1 = min(K, k0 + ks);
  const float* arow[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) arow[m] = A + (int64_t)min<int64_t>(m, M - 1) * lda;   // rows >= M: discarded
  float acc[MQ], sq[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) acc[m] = sq[m] = 0.f;
  // a wave's whole slice (48 rows at D = 768) in one batch of reads where the
  // registers allow it
  constexpr int kCdUnroll = MQ <= 4 ? 48 : 16;
  for (int kb = k0; kb < k1; kb += kCdUnroll) {
    float c[kCdUnroll];
#pragma unroll
    for (int u = 0; u < kCdUnroll; ++u) c[u] = B[(int64_t)min(kb + u, k1 - 1) * ldb + nc];
#pragma unroll
    for (int u = 0; u < kCdUnroll; ++u) {
      if (kb + u < k1) {
#pragma unroll
        for (int m = 0; m < MQ; ++m) {
          const float a = arow[m][kb + u];
          acc[m] = fmaf(a, c[u], acc[m]);
          sq[m] = fmaf(a, a, sq[m]);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < MQ; ++m) part[wave][m][lane] = acc[m];
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < MQ; ++m) nrm[wave][m] = sq[m];
  }
  __syncthreads();
  if (wave == 0 && n < N) {
    const float cb = bn[n];
#pragma unroll
    for (int m = 0; m < MQ; ++m) {
      if (m >= M) break;
      float dot = 0.f, an = 0.f;
#pragma unroll
      for (int w = 0; w < kCdWaves; ++w) {
        dot += part[w][m][lane];
        an += nrm[w][m];
      }
      Y[(int64_t)m * ldy + n] = fmaxf(an + cb - 2.f * dot, 0.f);
    }
  }
}

constexpr int kCdFewMax = 8;   // query rows handled by k_cdist_few

}  // namespace

bool gemm_f32_wide_tile(int64_t M, int N) { return ((M + 127) / 128) * (((int64_t)N + 127) / 128) >= 1024; }

namespace {

template <int MODE>
void launch_f32_mfma(const float* A, int64_t lda, const float* sub, const int32_t* sel, const float* B,
                     int64_t ldb, float* Y, int64_t ldy, int64_t M, int N, int K, const float* bn,
                     float* gmin, hipStream_t st) {
  // the 128 tile when it still gives at least 1024 blocks, else the 64 tile
  const GemmJob j{A, lda, sub, sel, B, ldb, Y, ldy, M, N, K, bn, gmin};
  if (M <= 0) return;
  if (MODE == 1 && M <= kCdFewMax && !sel && !gmin) {
    const dim3 grid((unsigned)((N + kWave - 1) / kWave));
    if (M <= 1)
      hipLaunchKernelGGL(k_cdist_few<1>, grid, dim3(kCdThreads), 0, st, A, lda, M, B, ldb, N, K, bn, Y, ldy);
    else if (M <= 2)
      hipLaunchKernelGGL(k_cdist_few<2>, grid, dim3(kCdThreads), 0, st, A, lda, M, B, ldb, N, K, bn, Y, ldy);
    else if (M <= 4)
      hipLaunchKernelGGL(k_cdist_few<4>, grid, dim3(kCdThreads), 0, st, A, lda, M, B, ldb, N, K, bn, Y, ldy);
    else
      hipLaunchKernelGGL(k_cdist_few<8>, grid, dim3(kCdThreads), 0, st, A, lda, M, B, ldb, N, K, bn, Y, ldy);
    return;
  }
  if (gemm_f32_wide_tile(M, N)) {
    dim3 grid((unsigned)((M + 127) / 128), (N + 127) / 128);
    hipLaunchKernelGGL((k_gemm_f32_mfma<MODE, 4>), grid, dim3(256), 0, st, j);
  } else {
    dim3 grid((unsigned)((M + 63) / 64), (N + 63) / 64);
    hipLaunchKernelGGL((k_gemm_f32_mfma<MODE, 2>), grid, dim3(256), 0, st, j);
  }
}

// ---------------------------------------------------------------- split-BF16 MFMA GEMM
// Y = X * P with X split per element as hi = bf16(x), lo = bf16(x - hi) and P
// given as transposed BF16 hi/lo planes Bt[n][k]. Each 16x16 output block sums
// hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16 (FP32 accumulation).
// Block tile T x T (T = 64, or 32 when 64-wide tiles would leave most of the
// chip idle), K step 32, 4 waves each owning a T/2 x T/2 quadrant. The next K
// step's global reads are issued before this step's MFMAs. The tile size does
// not change any output's sum (same K steps, same products, same order).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {   // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int BK = 32;

template <int T>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ sub,
                                                     const int32_t* __restrict__ sel,
                                                     const uint16_t* __restrict__ Bhi,
                                                     const uint16_t* __restrict__ Blo,
                                                     float* __restrict__ Y, int64_t ldy, int64_t M,
                                                     int N, int K) {
  constexpr int EPT = T * BK / 256;   // operand elements per thread and K step (8 or 4)
  constexpr int TPR = BK / EPT;       // threads per tile row
  constexpr int WB = T / 32;          // 16x16 blocks per wave and dimension
  // k-contiguous rows, padded by 8 elements so 16-byte reads stay aligned
  __shared__ __attribute__((aligned(16))) uint16_t Ah[T][BK + 8], Al[T][BK + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[T][BK + 8], Bl[T][BK + 8];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.x * T;
  const int n0 = blockIdx.y * T;
  const int wm = (wave >> 1) * (T / 2), wn = (wave & 1) * (T / 2);
  f32x4 acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A loader: row tid / TPR, EPT consecutive k from (tid % TPR) * EPT
  const int la_r = tid / TPR, la_k = (tid % TPR) * EPT;
  const int64_t am = m0 + la_r;
  const float* arow = (am < M) ? A + am * lda : nullptr;
  const float* srow = (am < M && sel) ? sub + (int64_t)sel[am] * K : nullptr;
  // B loader: n row tid / TPR, EPT consecutive k
  const int lb_n = tid / TPR, lb_k = (tid % TPR) * EPT;
  const int bn = n0 + lb_n;
  float av[EPT];
  uint16_t bhv[EPT], blv[EPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int kk = k0 + la_k + i;
      float v = 0.f;
      if (arow && kk < K) {
        v = arow[kk];
        if (srow) v -= srow[kk];
      }
      av[i] = v;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) bhv[i] = blv[i] = 0;
    if (bn < N) {
      const int64_t o = (int64_t)bn * K + k0 + lb_k;
      if constexpr (EPT == 8) {
        if (k0 + lb_k + 8 <= K && (o & 7) == 0) {
          const u16x8 h = *reinterpret_cast<const u16x8*>(Bhi + o);
          const u16x8 l = *reinterpret_cast<const u16x8*>(Blo + o);
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            bhv[i] = h[i];
            blv[i] = l[i];
          }
          return;
        }
      } else {
        if (k0 + lb_k + 4 <= K && (o & 3) == 0) {
          const u16x4 h = *reinterpret_cast<const u16x4*>(Bhi + o);
          const u16x4 l = *reinterpret_cast<const u16x4*>(Blo + o);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            bhv[i] = h[i];
            blv[i] = l[i];
          }
          return;
        }
      }
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        if (k0 + lb_k + i < K) {
          bhv[i] = Bhi[o + i];
          blv[i] = Blo[o + i];
        }
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint16_t h = f2bf(av[i]);
      Ah[la_r][la_k + i] = h;
      Al[la_r][la_k + i] = f2bf(av[i] - bf2f(h));
      Bh[lb_n][lb_k + i] = bhv[i];
      Bl[lb_n][lb_k + i] = blv[i];
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    stash();
    __syncthreads();
    if (k0 + BK < K) fetch(k0 + BK);   // in flight during this step's MFMAs
    // operand fragments: row (or column) lane%16, k = (lane/16)*8 .. +7
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 ah[WB], al[WB], bh2[WB], bl2[WB];
#pragma unroll
    for (int i = 0; i < WB; ++i) {
      ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[wm + i * 16 + fr][fk]);
      al[i] = *reinterpret_cast<const bf16x8*>(&Al[wm + i * 16 + fr][fk]);
      bh2[i] = *reinterpret_cast<const bf16x8*>(&Bh[wn + i * 16 + fr][fk]);
      bl2[i] = *reinterpret_cast<const bf16x8*>(&Bl[wn + i * 16 + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < WB; ++i)
#pragma unroll
      for (int j = 0; j < WB; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh2[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl2[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh2[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  // output fragment: column lane%16, rows (lane/16)*4 + 0..3
  const int oc = lane & 15, orow = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) {
      const int n = n0 + wn + j * 16 + oc;
      if (n >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm + i * 16 + orow + e;
        if (m < M) Y[m * ldy + n] = acc[i][j][e];
      }
    }
}

// ---------------------------------------------------------------- split-BF16 centroid distances
// MODE 1 of the FP32 GEMM with the product <A[m], C[n]> summed as
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (FP32 accumulation): A is
// split per element as it is stashed, the centroids C come as hi/lo planes
// [n][k]. Tile 128 x 128, K step 32, four waves in a 2 x 2 grid each owning
// 4 x 4 blocks of 16 x 16. The MFMA takes the centroid fragment first, so
// lane l ends with row l % 16 and columns 4 (l / 16) .. + 3 of each block: the
// output and the group minima are laid out as in the FP32 kernel. The next K
// step's global reads are in flight during this step's MFMAs.
constexpr int CDT = 128, CDK = 32, CDP = CDK + 8;   // tile, K step, padded LDS row (bf16)
__global__ __launch_bounds__(256) void k_cd_bf16x3(const float* __restrict__ A, int64_t lda,
                                                   const uint16_t* __restrict__ Chi,
                                                   const uint16_t* __restrict__ Clo, const float* __restrict__ bn,
                                                   float* __restrict__ Y, int64_t ldy, int64_t M, int N, int K,
                                                   float* __restrict__ gmin) {
  // two buffers of the four operand tiles (80 KiB: two blocks per CU); the
  // row norms reuse buffer 0 after the K loop
  __shared__ __attribute__((aligned(16))) uint16_t Ts[2][4][CDT][CDP];
  float* an_s = reinterpret_cast<float*>(&Ts[0][0][0][0]);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.x * CDT;
  const int n0 = blockIdx.y * CDT;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // loaders: thread t takes row t / 2 of both tiles, 16 consecutive k from (t % 2) * 16
  const int lr = tid >> 1, lk = (tid & 1) * 16;
  const int64_t am = m0 + lr;
  const int bnr = n0 + lr;
  const float* arow = am < M ? A + am * lda : nullptr;
  const uint16_t* hrow = bnr < N ? Chi + (int64_t)bnr * K : nullptr;
  const uint16_t* lrow = bnr < N ? Clo + (int64_t)bnr * K : nullptr;
  const bool kvec = (K & 15) == 0 && (lda & 3) == 0;
  float av[16];
  u16x8 bh[2], bl[2];
  auto fetch = [&](int k0) {
    const int k = k0 + lk;
    if (kvec && k < K) {   // 16 consecutive k inside the row
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (arow) v = *reinterpret_cast<const float4*>(arow + k + 4 * q);
        av[4 * q] = v.x;
        av[4 * q + 1] = v.y;
        av[4 * q + 2] = v.z;
        av[4 * q + 3] = v.w;
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bh[q] = hrow ? *reinterpret_cast<const u16x8*>(hrow + k + 8 * q) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        bl[q] = lrow ? *reinterpret_cast<const u16x8*>(lrow + k + 8 * q) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const bool in = k + i < K;
      av[i] = (arow && in) ? arow[k + i] : 0.f;
      bh[i >> 3][i & 7] = (hrow && in) ? hrow[k + i] : (uint16_t)0;
      bl[i >> 3][i & 7] = (lrow && in) ? lrow[k + i] : (uint16_t)0;
    }
  };
  // the A tile's squared row norms, summed as the tiles are stashed (the two
  // threads of a row add up at the end)
  float asq = 0.f;
  auto stash = [&](int buf) {
    auto& Ah = Ts[buf][0];
    auto& Al = Ts[buf][1];
    auto& Bh = Ts[buf][2];
    auto& Bl = Ts[buf][3];
    // hardware conversions, round to nearest even (as f2bf)
    bf16x8 h[2], l[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const __bf16 hv = (__bf16)av[i];
      h[i >> 3][i & 7] = hv;
      l[i >> 3][i & 7] = (__bf16)(av[i] - (float)hv);
      asq = fmaf(av[i], av[i], asq);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<bf16x8*>(&Ah[lr][lk + 8 * q]) = h[q];
      *reinterpret_cast<bf16x8*>(&Al[lr][lk + 8 * q]) = l[q];
      *reinterpret_cast<u16x8*>(&Bh[lr][lk + 8 * q]) = bh[q];
      *reinterpret_cast<u16x8*>(&Bl[lr][lk + 8 * q]) = bl[q];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += CDK) {
    const bool more = k0 + CDK < K;
    if (more) fetch(k0 + CDK);   // in flight during this step's MFMAs
    const auto& Ah = Ts[buf][0];
    const auto& Al = Ts[buf][1];
    const auto& Bh = Ts[buf][2];
    const auto& Bl = Ts[buf][3];
    bf16x8 a_h[4], a_l[4], b_h[4], b_l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a_h[i] = *reinterpret_cast<const bf16x8*>(&Ah[wm + 16 * i + fr][fk]);
      a_l[i] = *reinterpret_cast<const bf16x8*>(&Al[wm + 16 * i + fr][fk]);
      b_h[i] = *reinterpret_cast<const bf16x8*>(&Bh[wn + 16 * i + fr][fk]);
      b_l[i] = *reinterpret_cast<const bf16x8*>(&Bl[wn + 16 * i + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b_l[j], a_h[i], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b_h[j], a_l[i], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b_h[j], a_h[i], acc[i][j], 0, 0, 0);
      }
    if (more) stash(buf ^ 1);   // the other buffer: last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  asq += __shfl_xor(asq, 1, kWave);
  if ((tid & 1) == 0) an_s[lr] = asq;
  __syncthreads();
  // output block (i, j): lane holds row fr, columns 4 fg .. 4 fg + 3
  const int fg = lane >> 4;
  const bool y_vec = (ldy & 3) == 0 && ((uintptr_t)Y & 15) == 0;
  const bool want_gmin = gmin != nullptr && n0 + wn < N;
  const int G = ((N + 63) >> 6) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + wm + i * 16 + fr;
    if (m >= M) continue;
    const float amv = an_s[wm + i * 16 + fr];
    float gv = __builtin_inff();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn + j * 16 + 4 * fg;
      f32x4 o = acc[i][j];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[e] = fmaxf(amv + bn[min(n + e, N - 1)] - 2.f * o[e], 0.f);
        gv = (n + e < N) ? fminf(gv, o[e]) : gv;
      }
      if (n >= N) continue;
      float* y = Y + m * ldy + n;
      if (y_vec && n + 3 < N) {
        *reinterpret_cast<f32x4*>(y) = o;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < N) y[e] = o[e];
      }
    }
    if (want_gmin) gmin[m * G + ((n0 + wn) >> 6) * 4 + fg] = gv;
  }
}

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
// Scan factors per code (see estimate), in FP64 from the stored factors.
__global__ void k_scan_factors(const float2* __restrict__ fac, int64_t n, float2* __restrict__ sfac) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = fac[i].x, ipo = fac[i].y;
  const double g = ipo > 0.0 ? a / ipo : 0.0;
  sfac[i] = make_float2((float)g, (float)(g * sqrt(fmax(1.0 - ipo * ipo, 0.0))));
}
}  // namespace

hipError_t launch_gemm_f32(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                           const float* B, int64_t ldb, float* Y, int64_t ldy, int64_t M, int N,
                           int K, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  launch_f32_mfma<0>(A, lda, sub, sel, B, ldb, Y, ldy, M, N, K, nullptr, nullptr, st);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16x3(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                              const uint16_t* Bhi, const uint16_t* Blo, float* Y, int64_t ldy,
                              int64_t M, int N, int K, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (((M + 63) / 64) * (((int64_t)N + 63) / 64) >= 256) {
    dim3 grid((unsigned)((M + 63) / 64), (N + 63) / 64);
    hipLaunchKernelGGL(k_gemm_bf16x3<64>, grid, dim3(256), 0, st, A, lda, sub, sel, Bhi, Blo, Y, ldy, M, N, K);
  } else {
    dim3 grid((unsigned)((M + 31) / 32), (N + 31) / 32);
    hipLaunchKernelGGL(k_gemm_bf16x3<32>, grid, dim3(256), 0, st, A, lda, sub, sel, Bhi, Blo, Y, ldy, M, N, K);
  }
  return hipGetLastError();
}

hipError_t launch_centroid_dist(const float* Q, int64_t nq, int dim, const float* Ct,
                                const float* cn, int nlist, float* D, float* gmin, hipStream_t st,
                                const uint16_t* Chi, const uint16_t* Clo) {
  if (Chi != nullptr && nq > kCdFewMax) {   // split-BF16 products, always the 128 tile (gmin when asked)
    const dim3 grid((unsigned)((nq + CDT - 1) / CDT), (unsigned)((nlist + CDT - 1) / CDT));
    hipLaunchKernelGGL(k_cd_bf16x3, grid, dim3(256), 0, st, Q, (int64_t)dim, Chi, Clo, cn, D, (int64_t)nlist, nq,
                       nlist, dim, gmin);
    return hipGetLastError();
  }
  launch_f32_mfma<1>(Q, (int64_t)dim, nullptr, nullptr, Ct, (int64_t)nlist, D, (int64_t)nlist, nq, nlist, dim,
                     cn, gemm_f32_wide_tile(nq, nlist) ? gmin : nullptr, st);
  return hipGetLastError();
}

hipError_t launch_rotate_centroid(const float* Q, int64_t nq, int dim, const float* P, int dp, float* qrot,
                                  const float* Ct, const float* cn, int nlist, float* D, float* gmin,
                                  hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  if (!gemm_f32_wide_tile(nq, nlist)) {
    launch_f32_mfma<0>(Q, (int64_t)dim, nullptr, nullptr, P, (int64_t)dp, qrot, (int64_t)dp, nq, dp, dim, nullptr,
                       nullptr, st);
    return launch_centroid_dist(Q, nq, dim, Ct, cn, nlist, D, gmin, st);
  }
  const GemmJob rot{Q, (int64_t)dim, nullptr, nullptr, P, (int64_t)dp, qrot, (int64_t)dp, nq, dp, dim, nullptr, nullptr};
  const GemmJob cd{Q, (int64_t)dim, nullptr, nullptr, Ct, (int64_t)nlist, D, (int64_t)nlist, nq, nlist, dim, cn, gmin};
  const int tm = (int)((nq + 127) / 128);
  const int rot_tiles = tm * ((dp + 127) / 128), cd_tiles = tm * ((nlist + 127) / 128);
  hipLaunchKernelGGL(k_gemm_rot_cdist, dim3((unsigned)(rot_tiles + cd_tiles)), dim3(256), 0, st, rot, cd, tm,
                     rot_tiles, tm);
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

hipError_t launch_scan_factors(const float2* fac, int64_t n, float2* sfac, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fac, n, sfac);
  return hipGetLastError();
}

}  // namespace rbq
