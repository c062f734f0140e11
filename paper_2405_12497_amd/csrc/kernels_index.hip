// Index-time helpers that run on the device: raw vectors reordered into list
// order when the caller's data already lives in device memory.
#include <algorithm>

#include "rbq_internal.hpp"

namespace rbq {
namespace {

// dst[p] = src[ids[p]] for rows of D floats; one wave per row, lanes over
// the row (consecutive lanes read consecutive floats).
__global__ __launch_bounds__(256) void k_gather_raw(const float* __restrict__ src, const int64_t* __restrict__ ids,
                                                    int64_t n, int D, float* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const int lane = lane_id();
  const float* s = src + ids[r] * (int64_t)D;
  float* d = dst + r * (int64_t)D;
  for (int i = lane; i < D; i += kWave) d[i] = s[i];
}

__global__ void k_xor_u8(uint8_t* __restrict__ x, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] ^= v;
}

// ------------------------------------------------------------------ k-means (IVF lists)
// Lloyd's k-means for the IVF lists (Sec. 4 clusters the data with k-means).
// The update sums the members of each list in 64-bit fixed point (value *
// 2^shift, rounded): integer additions commute, so the sums, and with them
// the centroids, do not depend on the order in which atomics land.

// max |x| over n values, as float bits (non-negative floats order like their bits)
__global__ void k_absmax(const float* __restrict__ x, int64_t n, uint32_t* __restrict__ out) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
  m = wave_max(m);
  if (lane_id() == 0) atomicMax(out, __float_as_uint(m));
}

// Per row: the list with the smallest distance (ties to the lower list), one wave per row.
__global__ __launch_bounds__(256) void k_row_argmin(const float* __restrict__ D, int64_t rows, int nlist,
                                                    int32_t* __restrict__ lab) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = lane_id();
  const float* row = D + r * (int64_t)nlist;
  float best = __builtin_inff();
  int bi = nlist;
  for (int l = lane; l < nlist; l += kWave) {
    const float v = row[l];
    if (v < best) {   // lanes visit their lists in increasing order: the first minimum is kept
      best = v;
      bi = l;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float ob = __shfl_xor(best, o, kWave);
    const int oi = __shfl_xor(bi, o, kWave);
    if (ob < best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) lab[r] = bi < nlist ? bi : 0;
}

// sums[lab[r]][d] += round(x[r][d] * 2^shift); cnt[lab[r]] += 1.
__global__ __launch_bounds__(256) void k_fixed_sums(const float* __restrict__ x, const int32_t* __restrict__ lab,
                                                    int64_t rows, int dim, double scale,
                                                    unsigned long long* __restrict__ sums,
                                                    unsigned int* __restrict__ cnt) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = lane_id();
  const int l = lab[r];
  const float* xr = x + r * (int64_t)dim;
  unsigned long long* sr = sums + (int64_t)l * dim;
  for (int d = lane; d < dim; d += kWave)
    atomicAdd(&sr[d], (unsigned long long)(long long)llrint((double)xr[d] * scale));
  if (lane == 0) atomicAdd(&cnt[l], 1u);
}

// Centroids of non-empty lists = sum / count (FP64, stored FP32); empty lists
// keep theirs. Also the transposed copy and squared norms the distance GEMM reads.
__global__ __launch_bounds__(256) void k_update_centroids(const unsigned long long* __restrict__ sums,
                                                          const unsigned int* __restrict__ cnt, int nlist,
                                                          int dim, double inv_scale, float* __restrict__ cent,
                                                          float* __restrict__ centT, float* __restrict__ cnorm) {
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= nlist) return;
  const int lane = lane_id();
  const unsigned int c = cnt[l];
  double nn = 0.0;
  for (int d = lane; d < dim; d += kWave) {
    float v = cent[(int64_t)l * dim + d];
    if (c > 0) {
      v = (float)((double)(long long)sums[(int64_t)l * dim + d] * inv_scale / (double)c);
      cent[(int64_t)l * dim + d] = v;
    }
    centT[(int64_t)d * nlist + l] = v;
    nn += (double)v * v;
  }
  nn = wave_sum_d(nn);
  if (lane == 0) cnorm[l] = (float)nn;
}

// ------------------------------------------------------------------ inner product
// Per code: <o_r - c, c> (FP64 sum) and ||o_r||^2 (max over codes by atomicMax
// on float bits); one wave per row.
__global__ __launch_bounds__(256) void k_ip_terms(const float* __restrict__ raw, const float* __restrict__ cent,
                                                  const int32_t* __restrict__ list_of, int64_t n, int dim,
                                                  float* __restrict__ fip, uint32_t* __restrict__ r2max) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const int lane = lane_id();
  const float* o = raw + r * (int64_t)dim;
  const float* c = cent + (int64_t)list_of[r] * dim;
  double f = 0.0, nn = 0.0;
  for (int i = lane; i < dim; i += kWave) {
    const double ci = c[i], oi = o[i];
    f += (oi - ci) * ci;
    nn += oi * oi;
  }
  f = wave_sum_d(f);
  nn = wave_sum_d(nn);
  if (lane == 0) {
    fip[r] = (float)f;
    atomicMax(r2max, __float_as_uint((float)nn));
  }
}

// y = x / ||x|| per row (zero rows stay zero); one wave per row.
__global__ __launch_bounds__(256) void k_normalize_rows(const float* __restrict__ x, int64_t n, int dim,
                                                        float* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const int lane = lane_id();
  const float* xr = x + r * (int64_t)dim;
  double nn = 0.0;
  for (int i = lane; i < dim; i += kWave) nn += (double)xr[i] * xr[i];
  nn = wave_sum_d(nn);
  const float inv = nn > 0.0 ? (float)(1.0 / sqrt(nn)) : 0.f;
  float* yr = y + r * (int64_t)dim;
  for (int i = lane; i < dim; i += kWave) yr[i] = xr[i] * inv;
}

// M_q = ||q|| rmax (1 + 1e-5): no exact inner product can exceed it, so
// M_q - <o_r, q_r> >= 0 for every code; one wave per query.
__global__ __launch_bounds__(256) void k_query_m(const float* __restrict__ q, int64_t nq, int dim, float rmax,
                                                 float* __restrict__ q_m) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nq) return;
  const int lane = lane_id();
  double nn = 0.0;
  for (int i = lane; i < dim; i += kWave) nn += (double)q[r * (int64_t)dim + i] * q[r * (int64_t)dim + i];
  nn = wave_sum_d(nn);
  if (lane == 0) q_m[r] = (float)(sqrt(nn) * (double)rmax * (1.0 + 1e-5)) + 1e-30f;
}

}  // namespace

hipError_t launch_ip_terms(const float* raw, const float* cent, const int32_t* list_of, int64_t n, int dim,
                           float* fip, uint32_t* r2max, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ip_terms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, raw, cent, list_of, n, dim, fip,
                     r2max);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(const float* x, int64_t n, int dim, float* y, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, x, n, dim, y);
  return hipGetLastError();
}

hipError_t launch_query_m(const float* q, int64_t nq, int dim, float rmax, float* q_m, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_query_m, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, q, nq, dim, rmax, q_m);
  return hipGetLastError();
}

hipError_t launch_absmax(const float* x, int64_t n, uint32_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, st, x, n, out);
  return hipGetLastError();
}

hipError_t launch_row_argmin(const float* D, int64_t rows, int nlist, int32_t* lab, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_argmin, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, D, rows, nlist, lab);
  return hipGetLastError();
}

hipError_t launch_fixed_sums(const float* x, const int32_t* lab, int64_t rows, int dim, double scale,
                             unsigned long long* sums, unsigned int* cnt, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fixed_sums, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, x, lab, rows, dim, scale,
                     sums, cnt);
  return hipGetLastError();
}

hipError_t launch_update_centroids(const unsigned long long* sums, const unsigned int* cnt, int nlist, int dim,
                                   double inv_scale, float* cent, float* centT, float* cnorm, hipStream_t st) {
  hipLaunchKernelGGL(k_update_centroids, dim3((unsigned)((nlist + 3) / 4)), dim3(256), 0, st, sums, cnt, nlist, dim,
                     inv_scale, cent, centT, cnorm);
  return hipGetLastError();
}

hipError_t launch_xor_u8(uint8_t* x, int64_t n, uint8_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xor_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

hipError_t launch_gather_raw(const float* src, const int64_t* ids, int64_t n, int D, float* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_raw, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, src, ids, n, D, dst);
  return hipGetLastError();
}

}  // namespace rbq
