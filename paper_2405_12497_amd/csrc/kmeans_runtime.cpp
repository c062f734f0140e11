// Lloyd's k-means on the GPU for the IVF lists (the clustering that Sec. 4
// puts in front of RaBitQ): rbq_kmeans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/rabitq.h"
#include "rbq_internal.hpp"
#include "rbq_runtime.hpp"

using namespace rbq;

namespace {

rbq_status fail(rbq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return rbq::set_error(st, buf);
}

#define HIPCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      (void)hipGetLastError();                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? RBQ_ENOMEM : RBQ_EDEVICE, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                  \
    }                                                                                          \
  } while (0)

// The first `take` entries of a seeded Fisher-Yates shuffle of 0..n-1
// (SplitMix64 counter stream), in increasing order when `sorted`.
std::vector<int64_t> seeded_choice(int64_t n, int64_t take, uint64_t seed, bool sorted) {
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t i = 0; i < take; ++i) {
    const uint64_t r = host_splitmix64(seed ^ (0x4B4D000000000000ull + (uint64_t)i));
    const int64_t j = i + (int64_t)(r % (uint64_t)(n - i));
    std::swap(perm[i], perm[j]);
  }
  perm.resize(take);
  if (sorted) std::sort(perm.begin(), perm.end());
  return perm;
}

// Nearest centroid of each row of X [rows x dim] (FP32 distances on the
// matrix cores, ties to the lower list), in chunks whose distance matrix
// stays within 1 GiB.
rbq_status assign_rows(const float* X, int64_t rows, int dim, int nlist, const float* centT, const float* cnorm,
                       DBuf& D, int32_t* lab, hipStream_t st) {
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(rows, (1ll << 30) / ((int64_t)nlist * 4)));
  HIPCHK(D.ensure((size_t)chunk * nlist * 4));
  for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
    const int64_t m = std::min(chunk, rows - r0);
    HIPCHK(launch_centroid_dist(X + r0 * dim, m, dim, centT, cnorm, nlist, (float*)D.p, nullptr, st));
    HIPCHK(launch_row_argmin((const float*)D.p, m, nlist, lab + r0, st));
  }
  return RBQ_OK;
}

}  // namespace

extern "C" rbq_status rbq_kmeans(const float* data, int64_t n, int32_t dim, int32_t nlist, int32_t iters,
                                 int64_t sample, uint64_t seed, const float* init, float* centroids,
                                 int32_t* assign, void* stream) {
  if (!data || !centroids || !assign) return fail(RBQ_EINVAL, "data, centroids and assign are required");
  if (n < 1 || n > (int64_t)INT32_MAX) return fail(RBQ_EINVAL, "n=%lld out of range", (long long)n);
  if (dim < 1 || dim > kMaxCodeBits) return fail(RBQ_EINVAL, "dim %d out of range [1, %d]", dim, kMaxCodeBits);
  if (iters < 0 || sample < 0) return fail(RBQ_EINVAL, "iters and sample must be >= 0");
  const int64_t m = sample > 0 ? std::min(sample, n) : n;
  if (nlist < 1 || nlist > kMaxNlist || nlist > m)
    return fail(RBQ_EINVAL, "nlist=%d outside [1, min(%d, sample rows %lld)]", nlist, kMaxNlist, (long long)m);
  hipStream_t st = (hipStream_t)stream;
  TmpBuf xdev, xs, ids, cent, centT, cnorm, lab, sums, cnt, D, absmax, out_assign;
  // the data on the device
  const float* X = data;
  if (!is_device_ptr(data)) {
    HIPCHK(xdev.ensure((size_t)n * dim * 4));
    HIPCHK(hipMemcpyAsync(xdev.p, data, (size_t)n * dim * 4, hipMemcpyHostToDevice, st));
    X = (const float*)xdev.p;
  }
  // the training rows: a seeded sample of m rows (all rows when m = n)
  const float* S = X;
  if (m < n) {
    const std::vector<int64_t> pick = seeded_choice(n, m, seed, true);
    HIPCHK(ids.ensure((size_t)m * 8));
    HIPCHK(xs.ensure((size_t)m * dim * 4));
    HIPCHK(hipMemcpyAsync(ids.p, pick.data(), (size_t)m * 8, hipMemcpyHostToDevice, st));
    HIPCHK(launch_gather_raw(X, (const int64_t*)ids.p, m, dim, (float*)xs.p, st));
    HIPCHK(hipStreamSynchronize(st));   // `pick` is released on return from this scope
    S = (const float*)xs.p;
  }
  // initial centroids: the caller's, or nlist distinct seeded training rows
  HIPCHK(cent.ensure((size_t)nlist * dim * 4));
  HIPCHK(centT.ensure((size_t)nlist * dim * 4));
  HIPCHK(cnorm.ensure((size_t)nlist * 4));
  HIPCHK(cnt.ensure((size_t)nlist * 4));
  HIPCHK(sums.ensure((size_t)nlist * dim * 8));
  if (init) {
    HIPCHK(hipMemcpyAsync(cent.p, init, (size_t)nlist * dim * 4, hipMemcpyDefault, st));
  } else {
    const std::vector<int64_t> pick = seeded_choice(m, nlist, seed ^ 0x696E6974ull, false);
    TmpBuf pid;
    HIPCHK(pid.ensure((size_t)nlist * 8));
    HIPCHK(hipMemcpyAsync(pid.p, pick.data(), (size_t)nlist * 8, hipMemcpyHostToDevice, st));
    HIPCHK(launch_gather_raw(S, (const int64_t*)pid.p, nlist, dim, (float*)cent.p, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  HIPCHK(launch_zero_u32(cnt.p, nlist, st));   // count 0: the update only derives centT and norms
  HIPCHK(launch_update_centroids((const unsigned long long*)sums.p, (const unsigned int*)cnt.p, nlist, dim, 1.0,
                                 (float*)cent.p, (float*)centT.p, (float*)cnorm.p, st));
  // fixed-point scale: |sum| <= m max|x| 2^shift < 2^62
  HIPCHK(absmax.ensure(4));
  HIPCHK(launch_zero_u32(absmax.p, 1, st));
  HIPCHK(launch_absmax(S, m * dim, (uint32_t*)absmax.p, st));
  uint32_t amx_bits = 0;
  HIPCHK(hipMemcpyAsync(&amx_bits, absmax.p, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float amx;
  std::memcpy(&amx, &amx_bits, 4);
  if (!std::isfinite(amx)) return fail(RBQ_EINVAL, "data has non-finite values");
  int shift = 0;
  if (amx > 0.f) shift = (int)std::floor(std::log2(std::ldexp(1.0, 62) / ((double)amx * (double)m)));
  shift = std::max(0, std::min(shift, 62));
  const double scale = std::ldexp(1.0, shift);
  HIPCHK(lab.ensure((size_t)m * 4));
  for (int it = 0; it < iters; ++it) {
    rbq_status rs = assign_rows(S, m, dim, nlist, (const float*)centT.p, (const float*)cnorm.p, D, (int32_t*)lab.p, st);
    if (rs != RBQ_OK) return rs;
    HIPCHK(launch_zero_u32(sums.p, (int64_t)nlist * dim * 2, st));
    HIPCHK(launch_zero_u32(cnt.p, nlist, st));
    HIPCHK(launch_fixed_sums(S, (const int32_t*)lab.p, m, dim, scale, (unsigned long long*)sums.p,
                             (unsigned int*)cnt.p, st));
    HIPCHK(launch_update_centroids((const unsigned long long*)sums.p, (const unsigned int*)cnt.p, nlist, dim,
                                   1.0 / scale, (float*)cent.p, (float*)centT.p, (float*)cnorm.p, st));
  }
  // final assignment of every row
  int32_t* asg_dev = assign;
  const bool asg_host = !is_device_ptr(assign);
  if (asg_host) {
    HIPCHK(out_assign.ensure((size_t)n * 4));
    asg_dev = (int32_t*)out_assign.p;
  }
  rbq_status rs = assign_rows(X, n, dim, nlist, (const float*)centT.p, (const float*)cnorm.p, D, asg_dev, st);
  if (rs != RBQ_OK) return rs;
  HIPCHK(hipMemcpyAsync(centroids, cent.p, (size_t)nlist * dim * 4, hipMemcpyDefault, st));
  if (asg_host) HIPCHK(hipMemcpyAsync(assign, asg_dev, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));   // the work buffers are freed on return
  return RBQ_OK;
}
