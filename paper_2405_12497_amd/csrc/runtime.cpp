// Host runtime behind the C ABI of include/rabitq.h: index construction
// (Algorithm 1), search orchestration (Algorithm 2 + the Sec. 4 rerank),
// workspace management, persistence and the debug exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/rabitq.h"
#include "rbq_internal.hpp"
#include "rbq_mlp.hpp"
#include "rbq_runtime.hpp"

using namespace rbq;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;

rbq_status fail(rbq_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
}  // namespace

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError();                                                                \
      return fail(e_ == hipErrorOutOfMemory ? RBQ_ENOMEM : RBQ_EDEVICE, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                 \
    }                                                                                         \
  } while (0)

namespace rbq {

rbq_status set_error(rbq_status st, const char* msg) {
  g_err = msg;
  return st;
}

// test hook: make the n-th following device allocation fail (0 = off)
static int g_fail_alloc_after = 0;

hipError_t dmalloc(void** p, size_t bytes) {
  if (g_fail_alloc_after > 0 && --g_fail_alloc_after == 0) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  if (bytes == 0) bytes = 16;
  return hipMalloc(p, bytes);
}

namespace {
std::atomic<uint64_t> g_buffer_gen{1};
std::atomic<int64_t> g_seg_budget{0};   // 0: a quarter of free device memory (at least kSegBudget)
}

int64_t seg_budget() {
  int64_t b = g_seg_budget.load();
  if (b > 0) return b;
  size_t fr = 0, tot = 0;
  b = kSegBudget;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess) b = std::max<int64_t>(kSegBudget, (int64_t)(fr / 4));
  g_seg_budget.store(b);
  return b;
}
void g_seg_budget_set(int64_t b) { g_seg_budget.store(b); }

uint64_t buffer_generation() { return g_buffer_gen.load(); }

namespace {
thread_local Arena* g_arena = nullptr;
}

hipError_t DBuf::ensure(size_t bytes) {
  if (bytes <= cap) return hipSuccess;
  if (g_arena) {   // carve from the caller's memory; nothing is allocated
    const size_t want = (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
    if (g_arena->used + want > g_arena->cap) {
      g_arena->used += want;   // record what the call would need
      return hipErrorOutOfMemory;
    }
    p = g_arena->base + g_arena->used;
    g_arena->used += want;
    cap = want;
    return hipSuccess;
  }
  release();
  g_buffer_gen.fetch_add(1);
  size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = dmalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    cap = 0;
    return e;
  }
  cap = want;
  return hipSuccess;
}

void DBuf::release() {
  if (p) g_buffer_gen.fetch_add(1);
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

bool is_device_ptr(const void* ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

uint64_t host_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace rbq

// ------------------------------------------------------------------ helpers
namespace {

uint16_t f2bf_host(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf2f_host(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Standard Gaussian draws from the seed (used only when the caller gives no
// matrix): SplitMix64 counter stream -> Box-Muller.
void gaussian_from_seed(uint64_t seed, int dp, std::vector<double>& g) {
  g.resize((size_t)dp * dp);
  const double two_pi = 6.283185307179586476925286766559;
  for (size_t i = 0; i < g.size(); i += 2) {
    const uint64_t a = host_splitmix64(seed ^ (0x5052000000000000ull + 2 * i));
    const uint64_t b = host_splitmix64(seed ^ (0x5052000000000000ull + 2 * i + 1));
    const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);   // (0, 1]
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    const double r = std::sqrt(-2.0 * std::log(u1));
    g[i] = r * std::cos(two_pi * u2);
    if (i + 1 < g.size()) g[i + 1] = r * std::sin(two_pi * u2);
  }
}

// Rows of G orthonormalised in order (Gram-Schmidt, as the random rotation is
// built in Appendix B), each projection applied twice for numerical
// orthogonality. Returns false if a row is (numerically) dependent.
bool orthonormalise_rows(std::vector<double>& p, int d) {
  for (int i = 0; i < d; ++i) {
    double* pi = &p[(size_t)i * d];
    const double n0 = std::sqrt(std::inner_product(pi, pi + d, pi, 0.0));
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < i; ++j) {
        const double* pj = &p[(size_t)j * d];
        const double c = std::inner_product(pi, pi + d, pj, 0.0);
        for (int t = 0; t < d; ++t) pi[t] -= c * pj[t];
      }
    }
    const double nrm = std::sqrt(std::inner_product(pi, pi + d, pi, 0.0));
    if (!(nrm > 1e-10 * n0) || !std::isfinite(nrm)) return false;
    for (int t = 0; t < d; ++t) pi[t] /= nrm;
  }
  return true;
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* c = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

int device_cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cus = pr.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

rbq_status check_params(const rbq_params* p) {
  if (!p) return fail(RBQ_EINVAL, "params is NULL");
  if (p->dim < 1 || p->dim > kMaxCodeBits) return fail(RBQ_EINVAL, "dim %d out of range [1, %d]", p->dim, kMaxCodeBits);
  if (p->code_bits != 0 && (p->code_bits % 64 != 0 || p->code_bits < p->dim || p->code_bits > kMaxCodeBits))
    return fail(RBQ_EINVAL, "code_bits %d must be 0 or a multiple of 64 in [dim, %d]", p->code_bits, kMaxCodeBits);
  if (p->nlist < 1 || p->nlist > kMaxNlist)
    return fail(RBQ_EINVAL, "nlist %d outside [1, %d]", p->nlist, kMaxNlist);
  if (p->bq < 1 || p->bq > 8) return fail(RBQ_EINVAL, "bq=%d outside [1, 8]", p->bq);
  if (!(p->eps0 >= 0.f) || !std::isfinite(p->eps0)) return fail(RBQ_EINVAL, "eps0 must be finite and >= 0");
  if (p->rot_precision != RBQ_ROT_FP32 && p->rot_precision != RBQ_ROT_BF16X3)
    return fail(RBQ_EINVAL, "unknown rot_precision %d", p->rot_precision);
  if (p->metric < RBQ_METRIC_L2 || p->metric > RBQ_METRIC_COSINE) return fail(RBQ_EINVAL, "unknown metric %d", p->metric);
  return RBQ_OK;
}

}  // namespace

// ------------------------------------------------------------------ index object
void rbq_index::graphs_clear() {
  for (rbq::GraphEntry& g : graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

rbq_index::~rbq_index() {
  graphs_clear();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (DBuf* b : {&g_q, &g_ids, &g_d, &g_npq, &h_stage_q, &h_stage_npq, &h_stage_ids, &h_stage_d}) b->release();
  prof.clear();
  prof.acc.release();
  for (DBuf* b : all_buffers()) b->release();
  if (done_event) (void)hipEventDestroy(done_event);
}

std::vector<DBuf*> rbq_index::all_buffers() {
  return {&d_codes, &d_fac, &d_sfac, &d_raw, &d_ids, &d_list_off, &d_cent, &d_centT, &d_cnorm, &d_crot,
          &d_P32, &d_Phi, &d_Plo, &d_chi, &d_clo, &d_id2list, &d_fip, &d_cnorm_probe, &ws.qrot, &ws.cd, &ws.cgmin, &ws.probe, &ws.probe_d, &ws.pairs,
          &ws.planes, &ws.qu8, &ws.pair_choff, &ws.pair_codeoff, &ws.q_nch, &ws.q_p0, &ws.q_n0,
          &ws.q_ncode, &ws.offs, &ws.counters, &ws.seg, &ws.seg_count, &ws.p0buf, &ws.tau,
          &ws.chunk_qcode,
          &ws.seedk, &ws.q_order, &ws.order_hist, &ws.lstats, &ws.q_boot, &ws.q_rerank, &ws.q_cand, &ws.pair_pt, &ws.q_m, &ws.qn, &ws.nprobe_q, &ws.q_fb, &ws.feats, &ws.tmp,
          &ws.mf_cnt, &ws.mf_fill, &ws.mf_pair_off, &ws.mf_unit_off, &ws.mf_pairs, &ws.units0,
          &ws.units1, &ws.fin_part, &ws.fin_pst, &ws.tau_part,
          &mlp.w32, &mlp.wbf, &mlp.wfrag, &mlp.grad, &mlp.m, &mlp.v, &mlp.act};
}

int64_t rbq_index::max_codes(int nprobe) const {
  const int p = std::min<int>(nprobe, (int)sizes_desc.size());
  return p > 0 ? codes_prefix[p - 1] : 0;
}

int64_t rbq_index::max_chunks(int nprobe, int chunk) const {
  int64_t s = 0;
  const int p = std::min<int>(nprobe, (int)sizes_desc.size());
  for (int i = 0; i < p; ++i) s += (sizes_desc[i] + chunk - 1) / chunk;
  return s;
}

extern "C" {

const char* rbq_last_error(void) { return g_err.c_str(); }

rbq_status rbq_params_default(rbq_params* p, int32_t dim, int32_t nlist) {
  if (!p) return fail(RBQ_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->dim = dim;
  p->code_bits = 0;
  p->nlist = nlist;
  p->bq = 4;
  p->eps0 = 1.9f;
  p->rot_precision = RBQ_ROT_FP32;
  p->seed = 0;
  return RBQ_OK;
}

rbq_status rbq_index_create(const rbq_params* p, rbq_index** out) {
  if (!out) return fail(RBQ_EINVAL, "out is NULL");
  rbq_status st = check_params(p);
  if (st != RBQ_OK) return st;
  rbq_index* idx = new (std::nothrow) rbq_index();
  if (!idx) return fail(RBQ_ENOMEM, "host allocation failed");
  idx->prm = *p;
  idx->dim = p->dim;
  idx->dp = p->code_bits ? p->code_bits : 64 * ((p->dim + 63) / 64);
  idx->W = idx->dp / 64;
  idx->nlist = p->nlist;
  *out = idx;
  return RBQ_OK;
}

rbq_status rbq_index_destroy(rbq_index* idx) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  delete idx;
  return RBQ_OK;
}

rbq_status rbq_index_set_eps0(rbq_index* idx, float eps0) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!(eps0 >= 0.f) || !std::isfinite(eps0)) return fail(RBQ_EINVAL, "eps0 must be finite and >= 0");
  std::lock_guard<std::mutex> lock(idx->mu);
  idx->prm.eps0 = eps0;
  idx->graphs_clear();   // captured searches hold the old bound
  return RBQ_OK;
}

rbq_status rbq_index_info_get(const rbq_index* idx, rbq_index_info* out) {
  if (!idx || !out) return fail(RBQ_EINVAL, "NULL argument");
  out->dim = idx->dim;
  out->code_bits = idx->dp;
  out->nlist = idx->nlist;
  out->rot_precision = idx->prm.rot_precision;
  out->n = idx->n;
  out->device_bytes = idx->device_bytes;
  out->graph_captures = idx->graph_captures;
  out->graphs_cached = (int64_t)idx->graphs.size();
  return RBQ_OK;
}

rbq_status rbq_index_list_sizes(const rbq_index* idx, int64_t* sizes) {
  if (!idx || !sizes) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  for (int k = 0; k < idx->nlist; ++k) sizes[k] = idx->h_list_off[k + 1] - idx->h_list_off[k];
  return RBQ_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ build
namespace rbq {

// Uploads P-derived tensors and centroid tensors; assumes h_P, h_cent set.
rbq_status upload_model(rbq_index* idx, hipStream_t st) {
  const int D = idx->dim, dp = idx->dp, L = idx->nlist;
  // P restricted to the first D rows: [D x dp] (rows of a zero-padded vector beyond D add nothing)
  std::vector<float> p32((size_t)D * dp);
  std::vector<uint16_t> phi((size_t)dp * D), plo((size_t)dp * D);
  for (int k = 0; k < D; ++k)
    for (int n = 0; n < dp; ++n) {
      const float v = (float)idx->h_P[(size_t)k * dp + n];
      p32[(size_t)k * dp + n] = v;
      const uint16_t h = f2bf_host(v);
      phi[(size_t)n * D + k] = h;
      plo[(size_t)n * D + k] = f2bf_host(v - bf2f_host(h));
    }
  HIPCHK(idx->d_P32.ensure(p32.size() * 4));
  HIPCHK(idx->d_Phi.ensure(phi.size() * 2));
  HIPCHK(idx->d_Plo.ensure(plo.size() * 2));
  HIPCHK(hipMemcpyAsync(idx->d_P32.p, p32.data(), p32.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(idx->d_Phi.p, phi.data(), phi.size() * 2, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(idx->d_Plo.p, plo.data(), plo.size() * 2, hipMemcpyHostToDevice, st));
  // centroids, transposed centroids, squared norms
  std::vector<float> ct((size_t)D * L), cn(L);
  for (int k = 0; k < L; ++k) {
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
      const float v = idx->h_cent[(size_t)k * D + i];
      ct[(size_t)i * L + k] = v;
      s += (double)v * v;
    }
    cn[k] = (float)s;
  }
  HIPCHK(idx->d_cent.ensure((size_t)L * D * 4));
  HIPCHK(idx->d_centT.ensure((size_t)L * D * 4));
  HIPCHK(idx->d_cnorm.ensure((size_t)L * 4));
  HIPCHK(idx->d_crot.ensure((size_t)L * dp * 4));
  HIPCHK(hipMemcpyAsync(idx->d_cent.p, idx->h_cent.data(), (size_t)L * D * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(idx->d_centT.p, ct.data(), ct.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(idx->d_cnorm.p, cn.data(), cn.size() * 4, hipMemcpyHostToDevice, st));
  if (idx->prm.rot_precision == RBQ_ROT_BF16X3) {   // centroid hi/lo planes for the split-BF16 distances
    std::vector<uint16_t> chi((size_t)L * D), clo((size_t)L * D);
    for (size_t e = 0; e < chi.size(); ++e) {
      const float v = idx->h_cent[e];
      chi[e] = f2bf_host(v);
      clo[e] = f2bf_host(v - bf2f_host(chi[e]));
    }
    HIPCHK(idx->d_chi.ensure(chi.size() * 2));
    HIPCHK(idx->d_clo.ensure(clo.size() * 2));
    HIPCHK(hipMemcpyAsync(idx->d_chi.p, chi.data(), chi.size() * 2, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(idx->d_clo.p, clo.data(), clo.size() * 2, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    idx->d_chi.release();
    idx->d_clo.release();
  }
  if (idx->prm.metric != RBQ_METRIC_L2) {   // the probe ranks by <q, c>: every centroid norm set to the largest
    const float cmax2 = *std::max_element(cn.begin(), cn.end());
    std::vector<float> cp(L, cmax2);
    HIPCHK(idx->d_cnorm_probe.ensure((size_t)L * 4));
    HIPCHK(hipMemcpyAsync(idx->d_cnorm_probe.p, cp.data(), cp.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // P^T c_k in FP64 on the device, stored as FP32
  TmpBuf p64;
  HIPCHK(p64.ensure((size_t)D * dp * 8));
  HIPCHK(hipMemcpyAsync(p64.p, idx->h_P.data(), (size_t)D * dp * 8, hipMemcpyHostToDevice, st));
  for (int k0 = 0; k0 < L; k0 += 32768) {
    const int m = std::min(32768, L - k0);
    HIPCHK(launch_rotate_f64((const float*)idx->d_cent.p + (size_t)k0 * D, m, D,
                             (const double*)p64.p, dp, (float*)idx->d_crot.p + (size_t)k0 * dp, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  p64.release();
  std::vector<int32_t> lo(L + 1);
  for (int k = 0; k <= L; ++k) lo[k] = (int32_t)idx->h_list_off[k];
  HIPCHK(idx->d_list_off.ensure(lo.size() * 4));
  HIPCHK(hipMemcpyAsync(idx->d_list_off.p, lo.data(), lo.size() * 4, hipMemcpyHostToDevice, st));
  // bounds for workspace sizing
  idx->sizes_desc.resize(L);
  for (int k = 0; k < L; ++k) idx->sizes_desc[k] = idx->h_list_off[k + 1] - idx->h_list_off[k];
  std::sort(idx->sizes_desc.begin(), idx->sizes_desc.end(), std::greater<int64_t>());
  idx->codes_prefix.resize(L);
  int64_t run = 0;
  for (int k = 0; k < L; ++k) idx->codes_prefix[k] = (run += idx->sizes_desc[k]);
  HIPCHK(hipStreamSynchronize(st));
  return RBQ_OK;
}

rbq_status rotate_rows(rbq_index* idx, const float* X, int64_t lda, const float* sub,
                       const int32_t* sel, int64_t M, float* Y, hipStream_t st) {
  if (idx->prm.rot_precision == RBQ_ROT_BF16X3) {
    HIPCHK(launch_gemm_bf16x3(X, lda, sub, sel, (const uint16_t*)idx->d_Phi.p,
                              (const uint16_t*)idx->d_Plo.p, Y, idx->dp, M, idx->dp, idx->dim, st));
  } else {
    HIPCHK(launch_gemm_f32(X, lda, sub, sel, (const float*)idx->d_P32.p, idx->dp, Y, idx->dp, M,
                           idx->dp, idx->dim, st));
  }
  return RBQ_OK;
}

void account_bytes(rbq_index* idx) {
  int64_t b = 0;
  for (DBuf* d : {&idx->d_codes, &idx->d_fac, &idx->d_sfac, &idx->d_raw, &idx->d_ids, &idx->d_list_off,
                  &idx->d_cent, &idx->d_centT, &idx->d_cnorm, &idx->d_crot, &idx->d_P32,
                  &idx->d_Phi, &idx->d_Plo, &idx->d_chi, &idx->d_clo, &idx->d_fip, &idx->d_cnorm_probe})
    b += (int64_t)d->cap;
  idx->device_bytes = b;
}

}  // namespace rbq

namespace rbq {

// Copy of `count` elements of a buffer that lives in host or device memory.
template <typename T>
rbq_status host_copy(const T* src, size_t count, std::vector<T>& out) {
  try {
    out.resize(count);
  } catch (...) {
    return fail(RBQ_ENOMEM, "host allocation failed");
  }
  if (count == 0) return RBQ_OK;
  if (is_device_ptr(src)) {
    HIPCHK(hipMemcpy(out.data(), src, count * sizeof(T), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out.data(), src, count * sizeof(T));
  }
  return RBQ_OK;
}

// Algorithm 1 for data (host or device), host centroids and assignments, and
// the rotation P (rows of the matrix whose transpose rotates: P^T v).
rbq_status build_impl(rbq_index* idx, const float* data, int64_t n, const std::vector<float>& cent,
                      const std::vector<int32_t>& assign, std::vector<double>& P, hipStream_t st) {
  const int D = idx->dim, L = idx->nlist, W = idx->W;
  const bool data_dev = is_device_ptr(data);
  // list layout (counting sort, stable in the original id)
  std::vector<int64_t> off(L + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t a = assign[i];
    if (a < 0 || a >= L) return fail(RBQ_EINVAL, "assign[%lld]=%d outside [0, %d)", (long long)i, a, L);
    off[a + 1]++;
  }
  for (int k = 0; k < L; ++k) off[k + 1] += off[k];
  std::vector<int64_t> ids(n);
  {
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) ids[fill[assign[i]]++] = i;
  }
  for (float v : cent)
    if (!std::isfinite(v)) return fail(RBQ_EINVAL, "centroids have non-finite entries");
  // release an old build
  idx->built = false;
  for (DBuf* b : idx->all_buffers()) b->release();
  idx->graphs_clear();
  idx->mlp.has_model = false;   // a model's features refer to the old lists
  idx->h_P.swap(P);
  idx->h_cent = cent;
  idx->h_list_off = off;
  idx->h_ids = ids;
  idx->n = n;
  rbq_status rs = upload_model(idx, st);
  if (rs != RBQ_OK) return rs;
  const int64_t npad = (n + 63) / 64 * 64;
  HIPCHK(idx->d_codes.ensure((size_t)npad * W * 8));
  HIPCHK(idx->d_fac.ensure((size_t)npad * sizeof(float2)));
  HIPCHK(idx->d_raw.ensure((size_t)n * D * 4));
  HIPCHK(idx->d_ids.ensure((size_t)n * 8));
  HIPCHK(launch_zero_u32(idx->d_codes.p, (int64_t)npad * W * 2, st));
  HIPCHK(launch_zero_u32(idx->d_fac.p, (int64_t)npad * 2, st));
  HIPCHK(hipMemcpyAsync(idx->d_ids.p, ids.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
  TmpBuf listof;
  HIPCHK(listof.ensure((size_t)n * 4));
  {
    std::vector<int32_t> lof(n);
    for (int k = 0; k < L; ++k)
      for (int64_t p = off[k]; p < off[k + 1]; ++p) lof[p] = k;
    HIPCHK(hipMemcpyAsync(listof.p, lof.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // raw vectors in list order: gathered on the device, or staged from the host in blocks
  if (data_dev) {
    HIPCHK(launch_gather_raw(data, (const int64_t*)idx->d_ids.p, n, D, (float*)idx->d_raw.p, st));
  } else {
    const int64_t blk = std::max<int64_t>(1, (int64_t)(64ll << 20) / ((int64_t)D * 4));
    std::vector<float> stage((size_t)std::min(blk, n) * D);
    for (int64_t p0 = 0; p0 < n; p0 += blk) {
      const int64_t m = std::min(blk, n - p0);
      for (int64_t r = 0; r < m; ++r)
        std::memcpy(&stage[(size_t)r * D], data + (size_t)ids[p0 + r] * D, (size_t)D * 4);
      HIPCHK(hipMemcpy((float*)idx->d_raw.p + (size_t)p0 * D, stage.data(), (size_t)m * D * 4,
                       hipMemcpyHostToDevice));
    }
  }
  if (idx->prm.metric == RBQ_METRIC_COSINE)   // cosine: the index holds unit vectors
    HIPCHK(launch_normalize_rows((const float*)idx->d_raw.p, n, D, (float*)idx->d_raw.p, st));
  // rotate residuals and encode, in blocks of rows
  {
    const int dp = idx->dp;
    const int64_t blk = std::max<int64_t>(64, std::min<int64_t>(n, (int64_t)(256ll << 20) / ((int64_t)dp * 4)));
    TmpBuf y;
    HIPCHK(y.ensure((size_t)blk * dp * 4));
    for (int64_t p0 = 0; p0 < n; p0 += blk) {
      const int64_t m = std::min(blk, n - p0);
      rs = rotate_rows(idx, (const float*)idx->d_raw.p + (size_t)p0 * D, D, (const float*)idx->d_cent.p,
                       (const int32_t*)listof.p + p0, m, (float*)y.p, st);
      if (rs != RBQ_OK) return rs;
      HIPCHK(launch_encode((const float*)y.p, m, W, (const float*)idx->d_raw.p, (const float*)idx->d_cent.p,
                           (const int32_t*)listof.p, D, p0, (uint64_t*)idx->d_codes.p,
                           (float2*)idx->d_fac.p, st));
    }
    HIPCHK(hipStreamSynchronize(st));
  }
  rs = scan_factors(idx, st);
  if (rs != RBQ_OK) return rs;
  rs = ip_factors(idx, (const int32_t*)listof.p, st);
  if (rs != RBQ_OK) return rs;
  account_bytes(idx);
  idx->built = true;
  return RBQ_OK;
}

rbq_status build_checks(rbq_index* idx, const float* data, int64_t n, const float* centroids,
                        const int32_t* assign) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!data || !centroids || !assign) return fail(RBQ_EINVAL, "data, centroids and assign are required");
  if (n < 1 || n > (int64_t)INT32_MAX - 64) return fail(RBQ_EINVAL, "n=%lld out of range", (long long)n);
  if ((uint64_t)((n + 63) / 64 * 64) * (uint64_t)idx->W >= (1ull << 32))
    return fail(RBQ_EINVAL, "n=%lld codes of %d words exceed 2^32 words", (long long)n, idx->W);
  return RBQ_OK;
}

}  // namespace rbq

extern "C" rbq_status rbq_index_build(rbq_index* idx, const float* data, int64_t n,
                                      const float* centroids, const int32_t* assign,
                                      const double* gauss, void* stream) {
  rbq_status rs = build_checks(idx, data, n, centroids, assign);
  if (rs != RBQ_OK) return rs;
  std::lock_guard<std::mutex> lock(idx->mu);
  const int dp = idx->dp;
  std::vector<float> cent;
  std::vector<int32_t> asg;
  std::vector<double> P;
  if ((rs = host_copy(centroids, (size_t)idx->nlist * idx->dim, cent)) != RBQ_OK) return rs;
  if ((rs = host_copy(assign, (size_t)n, asg)) != RBQ_OK) return rs;
  // rotation P: the Gaussian draw given or drawn from the seed, rows orthonormalised
  if (gauss) {
    if ((rs = host_copy(gauss, (size_t)dp * dp, P)) != RBQ_OK) return rs;
  } else {
    gaussian_from_seed(idx->prm.seed, dp, P);
  }
  for (double v : P)
    if (!std::isfinite(v)) return fail(RBQ_EINVAL, "gauss has non-finite entries");
  if (!orthonormalise_rows(P, dp)) return fail(RBQ_EINVAL, "gauss is rank deficient");
  return build_impl(idx, data, n, cent, asg, P, (hipStream_t)stream);
}

extern "C" rbq_status rbq_index_build_rotation(rbq_index* idx, const float* data, int64_t n,
                                               const float* centroids, const int32_t* assign,
                                               const double* P, void* stream) {
  rbq_status rs = build_checks(idx, data, n, centroids, assign);
  if (rs != RBQ_OK) return rs;
  if (!P) return fail(RBQ_EINVAL, "P is required (rbq_index_build draws one)");
  std::lock_guard<std::mutex> lock(idx->mu);
  const int dp = idx->dp;
  std::vector<float> cent;
  std::vector<int32_t> asg;
  std::vector<double> p;
  if ((rs = host_copy(centroids, (size_t)idx->nlist * idx->dim, cent)) != RBQ_OK) return rs;
  if ((rs = host_copy(assign, (size_t)n, asg)) != RBQ_OK) return rs;
  if ((rs = host_copy(P, (size_t)dp * dp, p)) != RBQ_OK) return rs;
  for (double v : p)
    if (!std::isfinite(v)) return fail(RBQ_EINVAL, "P has non-finite entries");
  // orthogonality, checked on a few seeded vectors: ||P (P^T x) - x|| <= 1e-6 ||x||
  std::vector<double> x(dp), y(dp), z(dp);
  for (int t = 0; t < 4; ++t) {
    double nx = 0.0;
    for (int i = 0; i < dp; ++i) {
      x[i] = (double)(host_splitmix64(0x4F5254ull * 1000003ull + (uint64_t)t * dp + i) >> 11) * 0x1.0p-53 - 0.5;
      nx += x[i] * x[i];
    }
    for (int j = 0; j < dp; ++j) {   // y = P^T x
      double a = 0.0;
      for (int i = 0; i < dp; ++i) a += p[(size_t)i * dp + j] * x[i];
      y[j] = a;
    }
    double err = 0.0;
    for (int i = 0; i < dp; ++i) {   // z = P y
      double a = 0.0;
      for (int j = 0; j < dp; ++j) a += p[(size_t)i * dp + j] * y[j];
      err += (a - x[i]) * (a - x[i]);
    }
    if (!(err <= 1e-12 * nx)) return fail(RBQ_EINVAL, "P is not orthogonal (||P P^T x - x|| / ||x|| = %.3g)",
                                          std::sqrt(err / nx));
  }
  return build_impl(idx, data, n, cent, asg, p, (hipStream_t)stream);
}

// ------------------------------------------------------------------ search
namespace rbq {

rbq_status ensure_workspace(rbq_index* idx, int64_t nq, int nprobe, int k, int chunk, bool mfma, int fin_w,
                            bool seg_exact) {
  Workspace& w = idx->ws;
  const int dp = idx->dp, W = idx->W;
  const int64_t np = nq * nprobe;
  HIPCHK(w.qrot.ensure((size_t)nq * dp * 4));
  HIPCHK(w.cd.ensure((size_t)nq * (size_t)idx->nlist * 4));
  HIPCHK(w.cgmin.ensure((size_t)nq * (((size_t)idx->nlist + 63) / 64 * 4) * 4));
  HIPCHK(w.probe.ensure((size_t)np * 4));
  HIPCHK(w.probe_d.ensure((size_t)np * 4));
  HIPCHK(w.pairs.ensure((size_t)np * sizeof(PairRec)));
  HIPCHK(w.planes.ensure((size_t)np * (idx->prm.bq <= 4 ? 4 : 8) * W * 8));
  if (mfma) {
    HIPCHK(w.qu8.ensure((size_t)np * dp));
    HIPCHK(w.mf_cnt.ensure((size_t)idx->nlist * 4));
    HIPCHK(w.mf_fill.ensure((size_t)idx->nlist * 4));
    HIPCHK(w.mf_pair_off.ensure((size_t)(idx->nlist + 1) * 8));
    HIPCHK(w.mf_unit_off.ensure((size_t)(idx->nlist + 1) * 8));
    HIPCHK(w.mf_pairs.ensure((size_t)np * 4));
  }
  HIPCHK(w.pair_choff.ensure((size_t)nq * (nprobe + 1) * 4));
  HIPCHK(w.pair_codeoff.ensure((size_t)nq * (nprobe + 1) * 4));
  HIPCHK(w.q_nch.ensure((size_t)nq * 4));
  HIPCHK(w.q_p0.ensure((size_t)nq * 4));
  HIPCHK(w.q_n0.ensure((size_t)nq * 4));
  HIPCHK(w.q_ncode.ensure((size_t)nq * 8));
  HIPCHK(w.offs.ensure((size_t)5 * (nq + 1 + (nq + kOffQ - 1) / kOffQ) * 8));
  HIPCHK(w.counters.ensure(kCounterBytes));
  if (!seg_exact) HIPCHK(w.seg.ensure((size_t)nq * std::max<int64_t>(1, idx->max_codes(nprobe)) * sizeof(Cand)));
  HIPCHK(w.seg_count.ensure((size_t)nq * std::max<int64_t>(1, idx->max_chunks(nprobe, chunk)) * 4));
  HIPCHK(w.chunk_qcode.ensure((size_t)nq * std::max<int64_t>(1, idx->max_chunks(nprobe, chunk)) * 4));
  HIPCHK(w.units0.ensure((size_t)nq * std::max<int64_t>(1, idx->max_chunks(nprobe, chunk)) * sizeof(UnitDesc)));
  HIPCHK(w.units1.ensure((size_t)nq * std::max<int64_t>(1, idx->max_chunks(nprobe, chunk)) * sizeof(UnitDesc)));
  HIPCHK(w.p0buf.ensure((size_t)nq * (boot_codes(k, chunk) - 1 + chunk) * sizeof(EstEnt)));
  HIPCHK(w.tau.ensure((size_t)nq * 4));
  HIPCHK(w.seedk.ensure((size_t)nq * k * sizeof(SeedEnt)));
  HIPCHK(w.q_boot.ensure((size_t)nq * 4));
  HIPCHK(w.q_rerank.ensure((size_t)nq * 4));
  HIPCHK(w.q_cand.ensure((size_t)nq * 4));
  if (idx->prm.metric != RBQ_METRIC_L2) {
    HIPCHK(w.pair_pt.ensure((size_t)np * 4));
    HIPCHK(w.q_m.ensure((size_t)nq * 4));
    if (idx->prm.metric == RBQ_METRIC_COSINE) HIPCHK(w.qn.ensure((size_t)nq * idx->dim * 4));
  }
  if (fin_w > 1) {
    HIPCHK(w.fin_part.ensure((size_t)nq * fin_w * k * 8));
    HIPCHK(w.fin_pst.ensure((size_t)nq * fin_w * 2 * 4));
  }
  if (tau_split(fin_w, k) > 1) HIPCHK(w.tau_part.ensure((size_t)nq * std::min(kMaxK, 4 * k) * 8));
  return RBQ_OK;
}

SearchDev make_dev(rbq_index* idx, const float* queries, int64_t nq, int nprobe, int k, int chunk,
                   const int32_t* nprobe_q, int64_t qid_base, bool mfma, int64_t* out_ids,
                   float* out_d) {
  Workspace& w = idx->ws;
  SearchDev s;
  std::memset(&s, 0, sizeof(s));
  s.codes = (const uint64_t*)idx->d_codes.p;
  s.fac = (const float2*)idx->d_fac.p;
  s.sfac = (const float2*)idx->d_sfac.p;
  s.raw = (const float*)idx->d_raw.p;
  s.ids = (const int64_t*)idx->d_ids.p;
  s.list_off = (const int32_t*)idx->d_list_off.p;
  s.cent = (const float*)idx->d_cent.p;
  s.crot = (const float*)idx->d_crot.p;
  s.cnorm = (const float*)idx->d_cnorm.p;
  s.dim = idx->dim;
  s.dp = idx->dp;
  s.rd = std::sqrt((double)idx->dp);
  s.prof_acc = nullptr;
  s.ird = 1.0 / s.rd;
  s.W = idx->W;
  s.nlist = idx->nlist;
  s.qmax = (1 << idx->prm.bq) - 1;
  s.npl = idx->prm.bq <= 4 ? 4 : 8;
  s.qoff = idx->prm.bq == 8 ? 128 : 0;
  s.metric = idx->prm.metric != RBQ_METRIC_L2 ? 1 : 0;
  s.fip = (const float*)idx->d_fip.p;
  s.pair_pt = (float*)w.pair_pt.p;
  s.q_m = (float*)w.q_m.p;
  s.eps0 = idx->prm.eps0;
  s.seed = idx->prm.seed;
  s.q = queries;
  s.qrot = (const float*)w.qrot.p;
  s.nq = nq;
  s.qid_base = qid_base;
  s.nprobe = nprobe;
  s.k = k;
  s.chunk = chunk;
  s.boot = boot_codes(k, chunk);
  s.probe = (const int32_t*)w.probe.p;
  s.nprobe_q = nprobe_q;
  s.pairs = (PairRec*)w.pairs.p;
  s.planes = (uint64_t*)w.planes.p;
  s.qu8 = mfma ? (int8_t*)w.qu8.p : nullptr;
  s.pair_choff = (int32_t*)w.pair_choff.p;
  s.pair_codeoff = (int32_t*)w.pair_codeoff.p;
  s.q_nch = (int32_t*)w.q_nch.p;
  s.q_p0 = (int32_t*)w.q_p0.p;
  s.q_n0 = (int32_t*)w.q_n0.p;
  s.q_ncode = (int64_t*)w.q_ncode.p;
  int64_t* offs = (int64_t*)w.offs.p;
  s.off_ch = offs;
  s.off_p0 = offs + (nq + 1);
  s.off_p1 = offs + 2 * (nq + 1);
  s.off_seg = offs + 3 * (nq + 1);
  s.off_n0 = offs + 4 * (nq + 1);
  s.blk_sums = offs + 5 * (nq + 1);
  s.counters = (unsigned long long*)w.counters.p;
  s.seg = (Cand*)w.seg.p;
  s.seg_count = (int32_t*)w.seg_count.p;
  s.p0buf = (EstEnt*)w.p0buf.p;
  s.tau = (float*)w.tau.p;
  s.seedk = (SeedEnt*)w.seedk.p;
  s.q_boot = (int32_t*)w.q_boot.p;
  s.q_rerank = (int32_t*)w.q_rerank.p;
  s.q_cand = (int32_t*)w.q_cand.p;
  s.mf_cnt = (int32_t*)w.mf_cnt.p;
  s.mf_fill = (int32_t*)w.mf_fill.p;
  s.mf_pair_off = (int64_t*)w.mf_pair_off.p;
  s.mf_unit_off = (int64_t*)w.mf_unit_off.p;
  s.mf_pairs = (int32_t*)w.mf_pairs.p;
  s.units0 = (UnitDesc*)w.units0.p;
  s.units1 = (UnitDesc*)w.units1.p;
  s.chunk_qcode = (int32_t*)w.chunk_qcode.p;
  s.out_ids = out_ids;
  s.out_d = out_d;
  return s;
}

// Scan factors per code from the stored (a, <o_bar,o>); run after every
// build and load, so saved indexes do not carry them.
rbq_status scan_factors(rbq_index* idx, hipStream_t st) {
  const int64_t npad = (idx->n + 63) / 64 * 64;
  HIPCHK(idx->d_sfac.ensure((size_t)std::max<int64_t>(1, npad) * sizeof(float2)));
  HIPCHK(launch_scan_factors((const float2*)idx->d_fac.p, npad, (float2*)idx->d_sfac.p, st));
  HIPCHK(hipStreamSynchronize(st));
  return RBQ_OK;
}

rbq_status ip_factors(rbq_index* idx, const int32_t* list_of, hipStream_t st) {
  if (idx->prm.metric == RBQ_METRIC_L2) return RBQ_OK;
  const int64_t npad = (idx->n + 63) / 64 * 64;
  HIPCHK(idx->d_fip.ensure((size_t)std::max<int64_t>(1, npad) * 4));
  HIPCHK(launch_zero_u32(idx->d_fip.p, npad, st));
  TmpBuf r2;
  HIPCHK(r2.ensure(4));
  HIPCHK(launch_zero_u32(r2.p, 1, st));
  HIPCHK(launch_ip_terms((const float*)idx->d_raw.p, (const float*)idx->d_cent.p, list_of, idx->n, idx->dim,
                         (float*)idx->d_fip.p, (uint32_t*)r2.p, st));
  uint32_t bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, r2.p, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float r2max;
  std::memcpy(&r2max, &bits, 4);
  idx->rmax = std::sqrt(r2max);
  return RBQ_OK;
}

rbq_status prepare_queries(rbq_index* idx, const float* queries, int64_t nq, hipStream_t st, const float** out) {
  *out = queries;
  if (idx->prm.metric == RBQ_METRIC_L2) return RBQ_OK;
  Workspace& w = idx->ws;
  HIPCHK(w.q_m.ensure((size_t)nq * 4));
  if (idx->prm.metric == RBQ_METRIC_COSINE) {
    HIPCHK(w.qn.ensure((size_t)nq * idx->dim * 4));
    HIPCHK(launch_normalize_rows(queries, nq, idx->dim, (float*)w.qn.p, st));
    *out = (const float*)w.qn.p;
  }
  HIPCHK(launch_query_m(*out, nq, idx->dim, idx->rmax, (float*)w.q_m.p, st));
  return RBQ_OK;
}

// Rotation, centroid scoring and probe selection for a batch.
rbq_status front(rbq_index* idx, const float* queries, int64_t nq, int nprobe,
                 const int32_t* nprobe_q, hipStream_t st) {
  Workspace& w = idx->ws;
  if (idx->prm.rot_precision == RBQ_ROT_FP32) {
    HIPCHK(launch_rotate_centroid(queries, nq, idx->dim, (const float*)idx->d_P32.p, idx->dp, (float*)w.qrot.p,
                                  (const float*)idx->d_centT.p, idx->probe_cnorm(), idx->nlist,
                                  (float*)w.cd.p, (float*)w.cgmin.p, st));
  } else {
    rbq_status rs = rotate_rows(idx, queries, idx->dim, nullptr, nullptr, nq, (float*)w.qrot.p, st);
    if (rs != RBQ_OK) return rs;
    HIPCHK(launch_centroid_dist(queries, nq, idx->dim, (const float*)idx->d_centT.p,
                                idx->probe_cnorm(), idx->nlist, (float*)w.cd.p, (float*)w.cgmin.p, st, idx->cent_hi(), idx->cent_lo()));
  }
  HIPCHK(launch_select_probe((const float*)w.cd.p, (const float*)w.cgmin.p, nq, idx->nlist, nprobe, nprobe_q,
                             (int32_t*)w.probe.p, (float*)w.probe_d.p, st));
  return RBQ_OK;
}

// Persistent scan grid: the blocks that fit on the device at once (per the
// kernel's occupancy), or fewer when there are fewer units than waves.
int scan_grid(rbq_index* idx, int64_t nq, int64_t units_per_query, int blocks_per_cu) {
  const int64_t ub = std::max<int64_t>(1, nq * units_per_query);
  const int64_t g = std::min<int64_t>((int64_t)device_cu_count() * blocks_per_cu, (ub + 3) / 4);
  return (int)std::max<int64_t>(1, g);
}

rbq_status run_search(rbq_index* idx, const float* queries, int64_t nq, const rbq_search_opts& opts,
                      int scan_kernel, int chunk, int mf_rg, bool learned, int64_t* out_ids, float* out_d,
                      hipStream_t st, const int32_t** used_npq, int* used_stride, int64_t seg_cap,
                      int64_t* done) {
  if (done) *done = nq;
  const bool mfma = scan_kernel == RBQ_SCAN_MFMA || scan_kernel == RBQ_SCAN_MFMA_FP4;
  rbq_search_opts o = opts;
  const int32_t* nprobe_q = o.nprobe_per_query;
  // The learned path runs one probe selection of at least the 64 nearest
  // lists: the features read those, and the search reuses the selection with
  // its per-query nprobe (at most the caller's nprobe).
  if (learned) o.nprobe = std::max(o.nprobe, std::min(kMlpNear, idx->nlist));
  const int fin_w = fin_waves(o.rerank_waves, nq, o.k);
  rbq_status rs = ensure_workspace(idx, nq, o.nprobe, o.k, chunk, mfma, fin_w, seg_cap > 0);
  if (rs != RBQ_OK) return rs;
  rs = prepare_queries(idx, queries, nq, st, &queries);
  if (rs != RBQ_OK) return rs;
  ProfState& pf = idx->prof;
  hipEvent_t ev[7] = {};
  // stage boundaries recorded: all seven, or (scan level) those of the main
  // scan and the rerank; unrecorded ones stay null
  auto rec = [&](int i) -> hipError_t {
    if (!pf.on || (pf.level == RBQ_PROFILE_SCAN && i < 4)) return hipSuccess;
    return hipEventRecord(ev[i], st);
  };
  if (pf.on) {
    // timing-only events: no system-scope fence (cache write-back) at each
    // record; rbq_profile_read synchronizes the device before reading them
    for (int i = 0; i < 7; ++i) {
      if (pf.level == RBQ_PROFILE_SCAN && i < 4) {
        pf.events.push_back(nullptr);
        continue;
      }
      HIPCHK(hipEventCreateWithFlags(&ev[i], hipEventDisableSystemFence));
      pf.events.push_back(ev[i]);
    }
  }
  HIPCHK(rec(0));
  if (learned) {
    rs = learned_nprobe(idx, queries, nq, opts.nprobe, o.nprobe, o.qid_base, st, &nprobe_q);
  } else {
    rs = front(idx, queries, nq, o.nprobe, nprobe_q, st);
  }
  if (rs != RBQ_OK) return rs;
  *used_npq = nprobe_q;
  *used_stride = o.nprobe;
  SearchDev s = make_dev(idx, queries, nq, o.nprobe, o.k, chunk, nprobe_q, o.qid_base, mfma,
                         out_ids, out_d);
  s.mfma_f4 = scan_kernel == RBQ_SCAN_MFMA_FP4 ? 1 : 0;
  s.mf_rg = mfma_row_groups(idx->dp, s.mfma_f4 != 0, mf_rg);
  s.boot_planes_only = mfma ? 1 : 0;
  HIPCHK(rec(1));
  HIPCHK(launch_plan(s, st));
  if (seg_cap > 0) {
    // the plan's exact code counts: the longest prefix of the batch whose
    // segments fit in seg_cap (the rest is searched by the caller's next call)
    std::vector<int64_t> off((size_t)nq + 1);
    HIPCHK(hipMemcpyAsync(off.data(), s.off_seg, off.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t cap_codes = seg_cap / (int64_t)sizeof(Cand);
    int64_t m = (int64_t)(std::upper_bound(off.begin() + 1, off.end(), cap_codes) - off.begin()) - 1;
    m = std::max<int64_t>(1, std::min(m, nq));
    HIPCHK(idx->ws.seg.ensure((size_t)std::max<int64_t>(1, off[(size_t)m]) * sizeof(Cand)));
    s.seg = (Cand*)idx->ws.seg.p;
    s.nq = m;
    nq = m;
    if (done) *done = m;
  }
  HIPCHK(launch_prep(s, true, st));
  const int64_t chunks = idx->max_chunks(o.nprobe, chunk);
  const int bpc = scan_popcnt_blocks_per_cu(idx->W, s.npl);
  // bootstrap chunks per query: whole chunks until >= boot codes, so at most boot of them
  const int grid0 = scan_grid(idx, nq, std::min<int64_t>(chunks, s.boot), bpc);
  const int grid = scan_grid(idx, nq, chunks, bpc);
  HIPCHK(rec(2));
  HIPCHK(launch_scan_popcnt(s, 0, grid0, st));
  HIPCHK(rec(3));
  HIPCHK(launch_tau_split(s, tau_split(fin_w, o.k), (uint64_t*)idx->ws.tau_part.p, st));
  // the batched scan's grouping of pairs by list (timed with the bootstrap
  // rerank, so that the phase-1 events bound the scan kernel alone)
  if (mfma) HIPCHK(launch_group_mfma(s, st));
  HIPCHK(rec(4));
  if (mfma) {
    HIPCHK(launch_scan_mfma(s, 1, scan_grid(idx, nq, chunks, scan_mfma_blocks_per_cu(idx->dp, s.mfma_f4 != 0, s.mf_rg, s.npl == 4)),
                            st));
  } else {
    HIPCHK(launch_scan_popcnt(s, 1, grid, st));
  }
  HIPCHK(rec(5));
  s.prof_acc = pf.on ? (unsigned long long*)pf.acc.p : nullptr;   // codes counted by finalize
  if (nprobe_q) {   // uneven reranks: the largest nprobe first
    HIPCHK(idx->ws.q_order.ensure((size_t)nq * 4));
    HIPCHK(idx->ws.order_hist.ensure(128 * 4));
    HIPCHK(launch_query_order(nprobe_q, nq, o.nprobe, (int32_t*)idx->ws.order_hist.p, (int32_t*)idx->ws.q_order.p,
                              st));
    s.q_order = (const int32_t*)idx->ws.q_order.p;
  }
  HIPCHK(launch_finalize_split(s, fin_w, (uint64_t*)idx->ws.fin_part.p, (int32_t*)idx->ws.fin_pst.p, st));
  HIPCHK(rec(6));
  return RBQ_OK;
}

// ------------------------------------------------------------------ graph replay
namespace {
constexpr size_t kMaxGraphs = 192;

// Rows of the captured batch for nq queries: exact up to 32, else rounded up
// to a multiple of 1/16 of the largest power of two <= nq (<= 6.25% extra).
int64_t graph_rows(int64_t nq) {
  if (nq <= 32) return nq;
  int64_t p = 1;
  while (p * 2 <= nq) p *= 2;
  const int64_t step = p / 16;
  return (nq + step - 1) / step * step;
}

__attribute__((unused)) bool same_shape(const GraphEntry& g, const GraphEntry& k) {
  return g.nqb == k.nqb && g.k == k.k && g.nprobe == k.nprobe && g.kernel == k.kernel &&
         g.chunk == k.chunk && g.mf_rg == k.mf_rg && g.learned == k.learned && g.per_query == k.per_query &&
         g.qid_base == k.qid_base && g.fin_w == k.fin_w;
}
}  // namespace

// rbq_search with use_graph = 1 (the caller holds idx->mu).
rbq_status search_graph(rbq_index* idx, const float* queries, int64_t nq, const rbq_search_opts& o,
                        int kernel, int chunk, int mf_rg, bool learned, int64_t* out_ids, float* out_d,
                        hipStream_t st, const int32_t** used_npq, int* used_stride) {
  GraphEntry key;
  key.nqb = graph_rows(nq);
  key.k = o.k;
  key.nprobe = o.nprobe;
  key.kernel = kernel;
  key.chunk = chunk;
  key.mf_rg = mf_rg;
  key.learned = learned;
  key.per_query = !learned;   // non-learned graphs always read a staged per-query nprobe
  key.qid_base = o.qid_base;
  key.fin_w = fin_waves(o.rerank_waves, nq, o.k);
  const int64_t nqb = key.nqb;
  // Graph mode sizes the workspace and staging for a row count that grows by
  // powers of two (at least 1024), so that batches of varying size do not
  // reallocate buffers (and invalidate every captured graph) one after another.
  if (idx->graph_rows_hint < nqb) {
    int64_t h = std::max<int64_t>(1024, idx->graph_rows_hint);
    while (h < nqb) h *= 2;
    idx->graph_rows_hint = h;
  }
  const int stride = learned ? std::max(o.nprobe, std::min(kMlpNear, idx->nlist)) : o.nprobe;
  int64_t hint = idx->graph_rows_hint;
  // ... as long as the candidate segments stay below a quarter of the device
  // memory that was free when graph mode was first used
  if (idx->graph_mem_cap == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    idx->graph_mem_cap = std::max<int64_t>(1ll << 30, (int64_t)(fr / 4));
  }
  const int64_t seg_row = std::max<int64_t>(1, idx->max_codes(stride)) * (int64_t)sizeof(Cand);
  while (hint > nqb && hint * seg_row > idx->graph_mem_cap) hint = std::max(nqb, hint / 2);
  {
    // the split-rerank buffers sized for the most waves any batch size can get,
    // so that a later batch with more rerank waves does not reallocate them
    // (which would invalidate every captured graph)
    rbq_status rs = ensure_workspace(idx, hint, stride, o.k, chunk, kernel == RBQ_SCAN_MFMA || kernel == RBQ_SCAN_MFMA_FP4,
                                     std::max(key.fin_w, fin_waves(kFinSplitMaxWaves, 1, o.k)));
    if (rs != RBQ_OK) return rs;
    if (learned) {
      HIPCHK(idx->ws.nprobe_q.ensure((size_t)hint * 4));
      HIPCHK(idx->ws.q_fb.ensure((size_t)hint * 4));
      HIPCHK(idx->ws.lstats.ensure((size_t)hint * kMlpStats * 4 * sizeof(float)));
      rs = mlp_reserve(idx, hint);
      if (rs != RBQ_OK) return rs;
    }
  }
  // staging buffers; a fresh query buffer is zero-filled so rows past nq are finite
  const size_t qbytes = (size_t)hint * idx->dim * 4;
  if (idx->g_q.cap < qbytes) {
    HIPCHK(idx->g_q.ensure(qbytes));
    HIPCHK(launch_zero_u32(idx->g_q.p, (int64_t)(idx->g_q.cap / 4), st));
  }
  HIPCHK(idx->g_ids.ensure((size_t)hint * kMaxK * 8));
  HIPCHK(idx->g_d.ensure((size_t)hint * kMaxK * 4));
  HIPCHK(idx->g_npq.ensure((size_t)hint * 4));
  // Padding rows [nq, nqb) repeat real queries (a zero vector would tie every
  // distance and rerank whole lists); without a model they probe one list.
  const size_t row_bytes = (size_t)idx->dim * 4;
  HIPCHK(hipMemcpyAsync(idx->g_q.p, queries, (size_t)nq * row_bytes, hipMemcpyDeviceToDevice, st));
  if (nqb > nq)
    HIPCHK(hipMemcpyAsync((char*)idx->g_q.p + (size_t)nq * row_bytes, idx->g_q.p, (size_t)(nqb - nq) * row_bytes,
                          hipMemcpyDeviceToDevice, st));
  rbq_search_opts og = o;
  if (!learned) {
    int32_t* npq = (int32_t*)idx->g_npq.p;
    if (o.nprobe_per_query) {
      HIPCHK(hipMemcpyAsync(npq, o.nprobe_per_query, (size_t)nq * 4, hipMemcpyDeviceToDevice, st));
    } else {
      HIPCHK(launch_fill_i32(npq, nq, o.nprobe, st));
    }
    HIPCHK(launch_fill_i32(npq + nq, nqb - nq, 1, st));
    og.nprobe_per_query = npq;
  }
  const float* gq = (const float*)idx->g_q.p;
  int64_t* gi = (int64_t*)idx->g_ids.p;
  float* gd = (float*)idx->g_d.p;
  GraphEntry* ent = nullptr;
  for (size_t i = 0; i < idx->graphs.size(); ++i) {
    if (!same_shape(idx->graphs[i], key)) continue;
    if (idx->graphs[i].gen == buffer_generation()) {
      ent = &idx->graphs[i];
    } else {   // captured before some buffer moved: recapture
      (void)hipGraphExecDestroy(idx->graphs[i].exec);
      idx->graphs.erase(idx->graphs.begin() + (long)i);
    }
    break;
  }
  if (!ent) {
    // eager run of the staged batch: allocates and sizes everything the capture replays
    rbq_status rs = run_search(idx, gq, nqb, og, kernel, chunk, mf_rg, learned, gi, gd, st, used_npq, used_stride);
    if (rs != RBQ_OK) return rs;
    if (!idx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&idx->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamSynchronize(st));
    const uint64_t gen0 = buffer_generation();
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(idx->cap_stream, hipStreamCaptureModeRelaxed));
    const int32_t* npq_c = nullptr;
    int stride_c = 0;
    rs = run_search(idx, gq, nqb, og, kernel, chunk, mf_rg, learned, gi, gd, idx->cap_stream, &npq_c, &stride_c);
    const hipError_t ec = hipStreamEndCapture(idx->cap_stream, &graph);
    if (rs != RBQ_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rs;
    }
    if (ec != hipSuccess || !graph) return fail(RBQ_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    if (buffer_generation() != gen0) {
      (void)hipGraphDestroy(graph);
      return fail(RBQ_EDEVICE, "a buffer was allocated during graph capture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(RBQ_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    if (idx->graphs.size() >= kMaxGraphs) {   // evict the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < idx->graphs.size(); ++i)
        if (idx->graphs[i].last_use < idx->graphs[lru].last_use) lru = i;
      (void)hipGraphExecDestroy(idx->graphs[lru].exec);
      idx->graphs.erase(idx->graphs.begin() + (long)lru);
    }
    key.gen = gen0;
    key.exec = exec;
    ++idx->graph_captures;
    idx->graphs.push_back(key);
    ent = &idx->graphs.back();
    *used_npq = npq_c;
    *used_stride = stride_c;
  } else {
    // the pointers a replay uses are the ones captured: workspace and staging
    *used_stride = learned ? std::max(o.nprobe, std::min(kMlpNear, idx->nlist)) : o.nprobe;
    *used_npq = learned ? (const int32_t*)idx->ws.nprobe_q.p : og.nprobe_per_query;
  }
  ent->last_use = ++idx->graph_clock;
  HIPCHK(hipGraphLaunch(ent->exec, st));
  HIPCHK(hipMemcpyAsync(out_ids, gi, (size_t)nq * o.k * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(out_d, gd, (size_t)nq * o.k * 4, hipMemcpyDeviceToDevice, st));
  return RBQ_OK;
}

}  // namespace rbq

extern "C" rbq_status rbq_search(rbq_index* idx, const float* queries, int64_t nq,
                                 const rbq_search_opts* opts, int64_t* out_ids, float* out_dists,
                                 rbq_search_stats* stats, void* stream) {
  if (!idx || !opts) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  rbq_search_opts o = *opts;
  if (o.k < 1 || o.k > kMaxK) return fail(RBQ_EINVAL, "k=%d outside [1, %d]", o.k, kMaxK);
  if (o.nprobe < 1 || o.nprobe > std::min(idx->nlist, kMaxNprobe))
    return fail(RBQ_EINVAL, "nprobe=%d outside [1, %d]", o.nprobe, std::min(idx->nlist, kMaxNprobe));
  if (o.use_graph != 0 && o.use_graph != 1) return fail(RBQ_EINVAL, "use_graph must be 0 or 1");
  if (o.rerank_waves < 0) return fail(RBQ_EINVAL, "rerank_waves must be >= 0");
  if (o.scan_kernel < RBQ_SCAN_AUTO || o.scan_kernel > RBQ_SCAN_MFMA_FP4)
    return fail(RBQ_EINVAL, "unknown scan_kernel %d", o.scan_kernel);
  if (o.scan_kernel == RBQ_SCAN_MFMA_FP4 && idx->prm.bq > 4)
    return fail(RBQ_EUNSUPPORTED, "the FP8 x FP4 scan holds query values up to 15 exactly (B_q <= 4)");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (nq == 0) return RBQ_OK;
  if (!queries || !out_ids || !out_dists) return fail(RBQ_EINVAL, "queries, out_ids and out_dists are required");
  if (o.qid_base < 0 || o.qid_base + nq > (1ll << 24))
    return fail(RBQ_EINVAL, "query ids must stay below 2^24 (qid_base %lld, nq %lld)",
                (long long)o.qid_base, (long long)nq);
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  return rbq::search_locked(idx, queries, nq, o, out_ids, out_dists, stats, st, nullptr);
}

// The body of rbq_search for validated arguments, with idx->mu held. `force`
// (the autotuner's trials) fixes the chunk length, scan kernel and rerank
// waves instead of the tuned or default choice.
rbq_status rbq::search_locked(rbq_index* idx, const float* queries, int64_t nq, rbq_search_opts o,
                              int64_t* out_ids, float* out_dists, rbq_search_stats* stats, hipStream_t st,
                              const TuneEntry* force) {
  if (idx->done_event) HIPCHK(hipStreamWaitEvent(st, idx->done_event, 0));
  // Host buffers are staged through device copies (the copies are part of the call).
  int64_t* const user_ids = out_ids;
  float* const user_d = out_dists;
  const bool ids_host = !is_device_ptr(out_ids), d_host = !is_device_ptr(out_dists);
  if (!is_device_ptr(queries)) {
    HIPCHK(idx->h_stage_q.ensure((size_t)nq * idx->dim * 4));
    HIPCHK(hipMemcpyAsync(idx->h_stage_q.p, queries, (size_t)nq * idx->dim * 4, hipMemcpyHostToDevice, st));
    queries = (const float*)idx->h_stage_q.p;
  }
  if (o.nprobe_per_query && !is_device_ptr(o.nprobe_per_query)) {
    HIPCHK(idx->h_stage_npq.ensure((size_t)nq * 4));
    HIPCHK(hipMemcpyAsync(idx->h_stage_npq.p, o.nprobe_per_query, (size_t)nq * 4, hipMemcpyHostToDevice, st));
    o.nprobe_per_query = (const int32_t*)idx->h_stage_npq.p;
  }
  if (ids_host) {
    HIPCHK(idx->h_stage_ids.ensure((size_t)nq * o.k * 8));
    out_ids = (int64_t*)idx->h_stage_ids.p;
  }
  if (d_host) {
    HIPCHK(idx->h_stage_d.ensure((size_t)nq * o.k * 4));
    out_dists = (float*)idx->h_stage_d.p;
  }
  // chunk length, scan kernel and rerank waves: forced, tuned for this batch size, or the defaults
  const TuneEntry tc = force ? *force : idx->tuned_for(nq);
  int kernel = o.scan_kernel == RBQ_SCAN_AUTO ? tc.kernel : o.scan_kernel;
  const int chunk = std::min(tc.chunk, kMaxP0 + 1 - o.k);   // bootstrap codes (k - 1 + chunk) fit the seed sort
  const int mf_rg = tc.mf_rg;
  if (o.rerank_waves == 0) o.rerank_waves = tc.fin_w;
  if (kernel == RBQ_SCAN_AUTO || (kernel == RBQ_SCAN_MFMA && !rbq::mfma_available())) {
    if (kernel == RBQ_SCAN_MFMA && o.scan_kernel == RBQ_SCAN_MFMA)
      return fail(RBQ_EUNSUPPORTED, "the MFMA scan kernel is not available in this library");
    kernel = RBQ_SCAN_POPCNT;
  }
  const bool learned = !o.nprobe_per_query && o.use_learned_nprobe && idx->mlp.has_model;
  // A query's candidate segment reserves a slot for each probed code, so a
  // batch is searched in sub-batches whose segments stay within kSegBudget
  // (same stream and workspace; queries keep their ids qid_base + i).
  const int stride_req = learned ? std::max(o.nprobe, std::min(kMlpNear, idx->nlist)) : o.nprobe;
  const int64_t seg_row = std::max<int64_t>(1, idx->max_codes(stride_req)) * (int64_t)sizeof(Cand);
  const int64_t budget = seg_budget();
  const int64_t sub = std::max<int64_t>(1, std::min<int64_t>(nq, budget / seg_row));
  const bool graph = o.use_graph && !idx->prof.on && sub == nq;
  // Where the worst case would split an eager batch, the segments are sized
  // from the plan's exact code counts instead (one synchronisation per
  // sub-batch); the sub-batch is then bounded by the other per-query buffers.
  const bool exact = !graph && sub < nq;
  const bool mf = kernel == RBQ_SCAN_MFMA || kernel == RBQ_SCAN_MFMA_FP4;
  const int64_t chunks_row = std::max<int64_t>(1, idx->max_chunks(stride_req, chunk));
  const int64_t other_row = (int64_t)idx->nlist * 4 +
                            (int64_t)stride_req * (int64_t)(8 + 8 + sizeof(PairRec) + 8 * 8 * idx->W + (mf ? idx->dp + 8 : 0)) +
                            chunks_row * (int64_t)(2 * sizeof(UnitDesc) + 8);
  const int64_t rows = exact ? std::max<int64_t>(sub, std::min<int64_t>(nq, budget / other_row)) : sub;
  auto add_stats = [&](int64_t m, const int32_t* npq, int stride) -> rbq_status {
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int32_t> rb(m), rr(m), cc(m);
    std::vector<int64_t> nc(m);
    HIPCHK(hipMemcpy(rb.data(), idx->ws.q_boot.p, m * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(rr.data(), idx->ws.q_rerank.p, m * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(cc.data(), idx->ws.q_cand.p, m * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(nc.data(), idx->ws.q_ncode.p, m * 8, hipMemcpyDeviceToHost));
    std::vector<int32_t> probe((size_t)m * stride);
    HIPCHK(hipMemcpy(probe.data(), idx->ws.probe.p, probe.size() * 4, hipMemcpyDeviceToHost));
    stats->queries += m;
    for (int64_t i = 0; i < m; ++i) {
      stats->reranked += rb[i] + rr[i];
      stats->reranked_bootstrap += rb[i];
      stats->candidates += cc[i];
      stats->codes_scanned += nc[i];
    }
    std::vector<int32_t> pq;
    if (npq) {
      pq.resize(m);
      HIPCHK(hipMemcpy(pq.data(), npq, m * 4, hipMemcpyDeviceToHost));
    }
    if (learned) {
      std::vector<int32_t> fb(m);
      HIPCHK(hipMemcpy(fb.data(), idx->ws.q_fb.p, m * 4, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < m; ++i) stats->nonfinite_fallbacks += fb[i];
    }
    for (int64_t i = 0; i < m; ++i) {
      const int P = npq ? std::min(std::max(pq[i], 1), stride) : stride;
      for (int r = 0; r < P; ++r) stats->pairs += (probe[(size_t)i * stride + r] >= 0);
    }
    return RBQ_OK;
  };
  for (int64_t q0 = 0; q0 < nq;) {
    int64_t m = std::min(rows, nq - q0);
    rbq_search_opts os = o;
    // from the whole call's size, rounded as graph replay rounds it, so that eager
    // and graph searches of one batch agree and a graph serves its size bucket
    os.rerank_waves = fin_waves(o.rerank_waves, graph_rows(nq), o.k);
    os.qid_base = o.qid_base + q0;
    if (o.nprobe_per_query) os.nprobe_per_query = o.nprobe_per_query + q0;
    const float* qs = queries + q0 * idx->dim;
    int64_t* oi = out_ids + q0 * o.k;
    float* od = out_dists + q0 * o.k;
    const int32_t* npq = nullptr;
    int stride = o.nprobe;
    rbq_status rs = graph ? rbq::search_graph(idx, qs, m, os, kernel, chunk, mf_rg, learned, oi, od, st, &npq, &stride)
                          : run_search(idx, qs, m, os, kernel, chunk, mf_rg, learned, oi, od, st, &npq, &stride,
                                       exact ? budget : 0, &m);
    if (rs != RBQ_OK) return rs;
    if (stats) {
      rs = add_stats(m, npq, stride);
      if (rs != RBQ_OK) return rs;
    }
    q0 += m;
  }
  if (idx->prof.on) idx->prof.searches++;   // one per call, however many sub-batches it ran
  if (ids_host) HIPCHK(hipMemcpyAsync(user_ids, out_ids, (size_t)nq * o.k * 8, hipMemcpyDeviceToHost, st));
  if (d_host) HIPCHK(hipMemcpyAsync(user_d, out_dists, (size_t)nq * o.k * 4, hipMemcpyDeviceToHost, st));
  if (!idx->done_event) HIPCHK(hipEventCreateWithFlags(&idx->done_event, hipEventDisableTiming));
  HIPCHK(hipEventRecord(idx->done_event, st));
  if (ids_host || d_host) HIPCHK(hipStreamSynchronize(st));
  return RBQ_OK;
}

// ------------------------------------------------------------------ allocation-free search
rbq_status rbq::search_in_arena(rbq_index* idx, const float* queries, int64_t nq, const rbq_search_opts* opts,
                                int64_t* out_ids, float* out_dists, void* base, size_t cap, hipStream_t st) {
  if (!idx || !opts) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  rbq_search_opts o = *opts;
  if (o.k < 1 || o.k > kMaxK) return fail(RBQ_EINVAL, "k=%d outside [1, %d]", o.k, kMaxK);
  if (o.nprobe < 1 || o.nprobe > std::min(idx->nlist, kMaxNprobe))
    return fail(RBQ_EINVAL, "nprobe=%d outside [1, %d]", o.nprobe, std::min(idx->nlist, kMaxNprobe));
  if (o.use_graph != 0) return fail(RBQ_EINVAL, "rbq_search_noalloc does not replay graphs (use_graph must be 0)");
  if (o.rerank_waves < 0) return fail(RBQ_EINVAL, "rerank_waves must be >= 0");
  if (o.scan_kernel < RBQ_SCAN_AUTO || o.scan_kernel > RBQ_SCAN_MFMA_FP4)
    return fail(RBQ_EINVAL, "unknown scan_kernel %d", o.scan_kernel);
  if (o.scan_kernel == RBQ_SCAN_MFMA_FP4 && idx->prm.bq > 4)
    return fail(RBQ_EUNSUPPORTED, "the FP8 x FP4 scan holds query values up to 15 exactly (B_q <= 4)");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (o.qid_base < 0 || o.qid_base + nq > (1ll << 24))
    return fail(RBQ_EINVAL, "query ids must stay below 2^24 (qid_base %lld, nq %lld)",
                (long long)o.qid_base, (long long)nq);
  if (!is_device_ptr(queries) || !is_device_ptr(out_ids) || !is_device_ptr(out_dists) ||
      (o.nprobe_per_query && !is_device_ptr(o.nprobe_per_query)))
    return fail(RBQ_EINVAL, "rbq_search_noalloc takes device queries, outputs and nprobe_per_query");
  std::lock_guard<std::mutex> lock(idx->mu);
  if (idx->prof.on) return fail(RBQ_ESTATE, "profiling is enabled (its events would be allocated)");
  if (idx->done_event) HIPCHK(hipStreamWaitEvent(st, idx->done_event, 0));
  const TuneEntry tc = idx->tuned_for(nq);   // as rbq_search chooses them
  int kernel = o.scan_kernel == RBQ_SCAN_AUTO ? tc.kernel : o.scan_kernel;
  const int chunk = std::min(tc.chunk, kMaxP0 + 1 - o.k);
  const int mf_rg = tc.mf_rg;
  if (o.rerank_waves == 0) o.rerank_waves = tc.fin_w;
  if (kernel == RBQ_SCAN_AUTO || (kernel == RBQ_SCAN_MFMA && !rbq::mfma_available())) {
    if (kernel == RBQ_SCAN_MFMA && o.scan_kernel == RBQ_SCAN_MFMA)
      return fail(RBQ_EUNSUPPORTED, "the MFMA scan kernel is not available in this library");
    kernel = RBQ_SCAN_POPCNT;
  }
  const bool learned = !o.nprobe_per_query && o.use_learned_nprobe && idx->mlp.has_model;
  o.rerank_waves = fin_waves(o.rerank_waves, graph_rows(nq), o.k);
  // the index's own workspace is set aside; every buffer the search ensures is carved
  Workspace mine;
  std::swap(idx->ws, mine);
  Arena arena;
  arena.base = (char*)base;
  arena.cap = cap;
  g_arena = &arena;
  const int32_t* npq = nullptr;
  int stride = 0;
  rbq_status rs = run_search(idx, queries, nq, o, kernel, chunk, mf_rg, learned, out_ids, out_dists, st, &npq, &stride);
  g_arena = nullptr;
  std::swap(idx->ws, mine);
  if (rs != RBQ_OK && arena.used > arena.cap)
    return fail(RBQ_EINVAL, "rbq_search_noalloc: this search needs more than its %zu-byte scratch (at least %zu "
                "bytes); use fewer queries or a smaller nprobe, or rbq_search", cap, arena.used);
  return rs;
}

// ------------------------------------------------------------------ persistence
namespace {
const char kMagic[8] = {'R', 'B', 'Q', 'I', 'D', 'X', '0', '1'};
struct FileHeader {
  char magic[8];
  uint32_t version;
  int32_t dim, dp, nlist, bq, rot_precision;
  float eps0;
  uint32_t pad;
  uint64_t seed;
  int64_t n;
};
}  // namespace

extern "C" rbq_status rbq_index_save(const rbq_index* cidx, const char* path) {
  rbq_index* idx = const_cast<rbq_index*>(cidx);
  if (!idx || !path) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  std::lock_guard<std::mutex> lock(idx->mu);
  const int64_t n = idx->n, npad = (n + 63) / 64 * 64;
  std::vector<uint64_t> codes((size_t)npad * idx->W);
  std::vector<float2> fac(npad);
  std::vector<float> raw((size_t)n * idx->dim);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(codes.data(), idx->d_codes.p, codes.size() * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(fac.data(), idx->d_fac.p, fac.size() * sizeof(float2), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(raw.data(), idx->d_raw.p, raw.size() * 4, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(RBQ_EINVAL, "cannot open %s for writing", path);
  FileHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.dim = idx->dim;
  h.dp = idx->dp;
  h.nlist = idx->nlist;
  h.bq = idx->prm.bq;
  h.rot_precision = idx->prm.rot_precision;
  h.eps0 = idx->prm.eps0;
  h.pad = (uint32_t)idx->prm.metric;
  h.seed = idx->prm.seed;
  h.n = n;
  uint64_t sum = 0xcbf29ce484222325ull;
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
  auto put = [&](const void* p, size_t bytes) {
    if (!ok) return;
    sum = fnv1a(sum, p, bytes);
    ok = std::fwrite(p, 1, bytes, f) == bytes;
  };
  put(idx->h_P.data(), idx->h_P.size() * 8);
  put(idx->h_cent.data(), idx->h_cent.size() * 4);
  put(idx->h_list_off.data(), idx->h_list_off.size() * 8);
  put(idx->h_ids.data(), idx->h_ids.size() * 8);
  put(raw.data(), raw.size() * 4);
  put(codes.data(), codes.size() * 8);
  put(fac.data(), fac.size() * sizeof(float2));
  if (ok) ok = std::fwrite(&sum, 8, 1, f) == 1;
  std::fclose(f);
  if (!ok) return fail(RBQ_EINVAL, "write to %s failed", path);
  return RBQ_OK;
}

extern "C" rbq_status rbq_index_load(const char* path, rbq_index** out) {
  if (!path || !out) return fail(RBQ_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(RBQ_EINVAL, "cannot open %s", path);
  FileHeader h;
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1) {
    std::fclose(f);
    return fail(RBQ_EFORMAT, "%s: not an index file (bad header)", path);
  }
  rbq_params p;
  rbq_params_default(&p, h.dim, h.nlist);
  p.code_bits = h.dp;
  p.bq = h.bq;
  p.eps0 = h.eps0;
  p.rot_precision = h.rot_precision;
  p.seed = h.seed;
  p.metric = (int32_t)h.pad;
  if (check_params(&p) != RBQ_OK || h.n < 1 || h.n > (int64_t)INT32_MAX) {
    std::fclose(f);
    return fail(RBQ_EFORMAT, "%s: invalid header fields", path);
  }
  rbq_index* idx = nullptr;
  if (rbq_index_create(&p, &idx) != RBQ_OK) {
    std::fclose(f);
    return RBQ_EFORMAT;
  }
  const int64_t n = h.n, npad = (n + 63) / 64 * 64;
  std::vector<uint64_t> codes;
  std::vector<float2> fac;
  std::vector<float> raw;
  uint64_t sum = 0xcbf29ce484222325ull;
  bool ok = true;
  auto get = [&](void* dst, size_t bytes) {
    if (!ok) return;
    ok = std::fread(dst, 1, bytes, f) == bytes;
    if (ok) sum = fnv1a(sum, dst, bytes);
  };
  try {
    idx->h_P.resize((size_t)idx->dp * idx->dp);
    idx->h_cent.resize((size_t)idx->nlist * idx->dim);
    idx->h_list_off.resize(idx->nlist + 1);
    idx->h_ids.resize(n);
    raw.resize((size_t)n * idx->dim);
    codes.resize((size_t)npad * idx->W);
    fac.resize(npad);
  } catch (...) {
    std::fclose(f);
    delete idx;
    return fail(RBQ_ENOMEM, "host allocation failed");
  }
  get(idx->h_P.data(), idx->h_P.size() * 8);
  get(idx->h_cent.data(), idx->h_cent.size() * 4);
  get(idx->h_list_off.data(), idx->h_list_off.size() * 8);
  get(idx->h_ids.data(), idx->h_ids.size() * 8);
  get(raw.data(), raw.size() * 4);
  get(codes.data(), codes.size() * 8);
  get(fac.data(), fac.size() * sizeof(float2));
  uint64_t stored = 0;
  if (ok) ok = std::fread(&stored, 8, 1, f) == 1;
  std::fclose(f);
  if (!ok) {
    delete idx;
    return fail(RBQ_EFORMAT, "%s: truncated file", path);
  }
  if (stored != sum) {
    delete idx;
    return fail(RBQ_EFORMAT, "%s: checksum mismatch", path);
  }
  bool sane = idx->h_list_off[0] == 0 && idx->h_list_off[idx->nlist] == n;
  for (int k = 0; sane && k < idx->nlist; ++k) sane = idx->h_list_off[k] <= idx->h_list_off[k + 1];
  if (!sane) {
    delete idx;
    return fail(RBQ_EFORMAT, "%s: inconsistent list offsets", path);
  }
  idx->n = n;
  hipStream_t st = nullptr;
  rbq_status rs = upload_model(idx, st);
  if (rs != RBQ_OK) {
    delete idx;
    return rs;
  }
  auto up = [&](DBuf& b, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = b.ensure(bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = up(idx->d_codes, codes.data(), codes.size() * 8);
  if (e == hipSuccess) e = up(idx->d_fac, fac.data(), fac.size() * sizeof(float2));
  if (e == hipSuccess) e = up(idx->d_raw, raw.data(), raw.size() * 4);
  if (e == hipSuccess) e = up(idx->d_ids, idx->h_ids.data(), idx->h_ids.size() * 8);
  if (e != hipSuccess) {
    delete idx;
    return fail(e == hipErrorOutOfMemory ? RBQ_ENOMEM : RBQ_EDEVICE, "upload failed: %s", hipGetErrorString(e));
  }
  rs = scan_factors(idx, nullptr);
  if (rs == RBQ_OK && idx->prm.metric != RBQ_METRIC_L2) {
    std::vector<int32_t> lof(n);
    for (int k = 0; k < idx->nlist; ++k)
      for (int64_t q = idx->h_list_off[k]; q < idx->h_list_off[k + 1]; ++q) lof[q] = k;
    TmpBuf listof;
    hipError_t e2 = listof.ensure((size_t)n * 4);
    if (e2 == hipSuccess) e2 = hipMemcpy(listof.p, lof.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    rs = e2 == hipSuccess ? ip_factors(idx, (const int32_t*)listof.p, nullptr)
                          : fail(RBQ_EDEVICE, "upload failed: %s", hipGetErrorString(e2));
  }
  if (rs != RBQ_OK) {
    delete idx;
    return rs;
  }
  account_bytes(idx);
  idx->built = true;
  *out = idx;
  return RBQ_OK;
}

// ------------------------------------------------------------------ debug exports
extern "C" rbq_status rbq_debug_export_codes(const rbq_index* cidx, uint64_t* codes, float* norm,
                                             float* ipo) {
  rbq_index* idx = const_cast<rbq_index*>(cidx);
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  std::lock_guard<std::mutex> lock(idx->mu);
  const int64_t n = idx->n, npad = (n + 63) / 64 * 64;
  const int W = idx->W;
  std::vector<uint64_t> c((size_t)npad * W);
  std::vector<float2> fac(npad);
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(c.data(), idx->d_codes.p, c.size() * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(fac.data(), idx->d_fac.p, fac.size() * sizeof(float2), hipMemcpyDeviceToHost));
  for (int64_t p = 0; p < n; ++p) {
    const int64_t id = idx->h_ids[p];
    if (codes)
      for (int w = 0; w < W; ++w) codes[(size_t)id * W + w] = c[((size_t)(p >> 6) * W + w) * 64 + (p & 63)];
    if (norm) norm[id] = fac[p].x;
    if (ipo) ipo[id] = fac[p].y;
  }
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_list_ids(const rbq_index* idx, int32_t list, int64_t* ids) {
  if (!idx || !ids) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (list < 0 || list >= idx->nlist) return fail(RBQ_EINVAL, "list out of range");
  for (int64_t p = idx->h_list_off[list]; p < idx->h_list_off[list + 1]; ++p)
    ids[p - idx->h_list_off[list]] = idx->h_ids[p];
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_rotate(rbq_index* idx, const float* queries, int64_t nq,
                                       float* out, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(out)) return fail(RBQ_EINVAL, "device pointers required");
  std::lock_guard<std::mutex> lock(idx->mu);
  return rotate_rows(idx, queries, idx->dim, nullptr, nullptr, nq, out, (hipStream_t)stream);
}

extern "C" rbq_status rbq_debug_centroid_dists(rbq_index* idx, const float* queries, int64_t nq,
                                               float* dists, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(dists)) return fail(RBQ_EINVAL, "device pointers required");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  rbq_status rs = ensure_workspace(idx, nq, 1, 1, kDefaultChunk, false);
  if (rs != RBQ_OK) return rs;
  rs = prepare_queries(idx, queries, nq, st, &queries);
  if (rs != RBQ_OK) return rs;
  HIPCHK(launch_centroid_dist(queries, nq, idx->dim, (const float*)idx->d_centT.p,
                              idx->probe_cnorm(), idx->nlist, (float*)idx->ws.cd.p, nullptr, st, idx->cent_hi(), idx->cent_lo()));
  HIPCHK(hipMemcpyAsync(dists, idx->ws.cd.p, (size_t)nq * idx->nlist * sizeof(float), hipMemcpyDeviceToDevice,
                        st));
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_probe(rbq_index* idx, const float* queries, int64_t nq,
                                      int32_t nprobe, int32_t* lists, float* dists, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nprobe < 1 || nprobe > std::min(idx->nlist, kMaxNprobe)) return fail(RBQ_EINVAL, "nprobe out of range");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(lists) || (dists && !is_device_ptr(dists)))
    return fail(RBQ_EINVAL, "device pointers required");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  rbq_status rs = ensure_workspace(idx, nq, nprobe, 1, kDefaultChunk, false);
  if (rs != RBQ_OK) return rs;
  rs = prepare_queries(idx, queries, nq, st, &queries);
  if (rs != RBQ_OK) return rs;
  HIPCHK(launch_centroid_dist(queries, nq, idx->dim, (const float*)idx->d_centT.p,
                              idx->probe_cnorm(), idx->nlist, (float*)idx->ws.cd.p,
                              (float*)idx->ws.cgmin.p, st, idx->cent_hi(), idx->cent_lo()));
  HIPCHK(launch_select_probe((const float*)idx->ws.cd.p, (const float*)idx->ws.cgmin.p, nq, idx->nlist, nprobe,
                             nullptr, lists,
                             dists, st));
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_quantize(rbq_index* idx, const float* queries, int64_t nq,
                                         const int32_t* lists, int32_t nprobe, int64_t qid_base,
                                         uint8_t* qu, float* scal, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nprobe < 1 || nprobe > kMaxNprobe) return fail(RBQ_EINVAL, "nprobe out of range");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(lists) || !is_device_ptr(qu) || !is_device_ptr(scal))
    return fail(RBQ_EINVAL, "device pointers required");
  if (qid_base < 0 || qid_base + nq > (1ll << 24)) return fail(RBQ_EINVAL, "query ids must stay below 2^24");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  rbq_status rs = ensure_workspace(idx, nq, nprobe, 1, kDefaultChunk, true);
  if (rs != RBQ_OK) return rs;
  rs = prepare_queries(idx, queries, nq, st, &queries);
  if (rs != RBQ_OK) return rs;
  rs = rotate_rows(idx, queries, idx->dim, nullptr, nullptr, nq, (float*)idx->ws.qrot.p, st);
  if (rs != RBQ_OK) return rs;
  HIPCHK(hipMemcpyAsync(idx->ws.probe.p, lists, (size_t)nq * nprobe * 4, hipMemcpyDeviceToDevice, st));
  SearchDev s = make_dev(idx, queries, nq, nprobe, 1, kDefaultChunk, nullptr, qid_base, true,
                         nullptr, nullptr);
  HIPCHK(launch_prep(s, false, st));
  HIPCHK(hipMemcpyAsync(qu, idx->ws.qu8.p, (size_t)nq * nprobe * idx->dp, hipMemcpyDeviceToDevice, st));
  if (s.qoff) HIPCHK(launch_xor_u8(qu, (int64_t)nq * nprobe * idx->dp, (uint8_t)s.qoff, st));   // back to 0..255
  HIPCHK(launch_pairs_to_scal(s, scal, st));
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_scan(rbq_index* idx, int32_t list, const uint8_t* qu,
                                     const float* scal, int32_t kernel, int32_t* ip, int32_t* pc,
                                     float* est, float* dist, float* lb, void* stream) {
  if (!idx || !scal) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (list < 0 || list >= idx->nlist) return fail(RBQ_EINVAL, "list out of range");
  if (kernel != RBQ_SCAN_POPCNT && kernel != RBQ_SCAN_MFMA && kernel != RBQ_SCAN_MFMA_FP4)
    return fail(RBQ_EINVAL, "kernel must be POPCNT, MFMA or MFMA_FP4");
  if (kernel == RBQ_SCAN_MFMA && !rbq::mfma_available()) return fail(RBQ_EUNSUPPORTED, "MFMA scan not available");
  if (kernel == RBQ_SCAN_MFMA_FP4 && idx->prm.bq > 4)
    return fail(RBQ_EUNSUPPORTED, "the FP8 x FP4 scan holds query values up to 15 exactly (B_q <= 4)");
  for (const void* p : {(const void*)qu, (const void*)ip, (const void*)pc, (const void*)est,
                        (const void*)dist, (const void*)lb})
    if (!is_device_ptr(p)) return fail(RBQ_EINVAL, "qu and outputs must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  rbq_status rs = ensure_workspace(idx, 1, 1, 1, kDefaultChunk, true);
  if (rs != RBQ_OK) return rs;
  Workspace& w = idx->ws;
  SearchDev s = make_dev(idx, nullptr, 1, 1, 1, kDefaultChunk, nullptr, 0, true, nullptr, nullptr);
  HIPCHK(launch_debug_pack(qu, idx->dp, idx->W, s.npl, s.qoff, scal[0], scal[1], scal[2], scal[3],
                           (PairRec*)w.pairs.p, (uint64_t*)w.planes.p, (int8_t*)w.qu8.p, (float*)w.pair_pt.p,
                           list, st));
  if (kernel == RBQ_SCAN_POPCNT) {
    // the list as main-phase work units of pair 0, for the production scan's export phase
    const int64_t beg = idx->h_list_off[list], end = idx->h_list_off[list + 1];
    std::vector<UnitDesc> units;
    for (int64_t p0 = beg; p0 < end; p0 += s.chunk) {
      UnitDesc u;
      std::memset(&u, 0, sizeof(u));
      u.start = p0;
      u.g = 0;
      u.count_slot = (int64_t)units.size();
      u.len = (int32_t)std::min<int64_t>(s.chunk, end - p0);
      units.push_back(u);
    }
    if (units.empty()) return RBQ_OK;
    HIPCHK(w.units1.ensure(units.size() * sizeof(UnitDesc)));
    HIPCHK(w.seg_count.ensure(units.size() * 4));
    const int64_t off_p1[2] = {0, (int64_t)units.size()};
    HIPCHK(hipMemcpyAsync(w.units1.p, units.data(), units.size() * sizeof(UnitDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s.off_p1, off_p1, sizeof(off_p1), hipMemcpyHostToDevice, st));
    s = make_dev(idx, nullptr, 1, 1, 1, kDefaultChunk, nullptr, 0, true, nullptr, nullptr);
    s.dbg_base = beg;
    s.dbg_ip = ip;
    s.dbg_pc = pc;
    s.dbg_est = est;
    s.dbg_dist = dist;
    s.dbg_lb = lb;
    HIPCHK(hipStreamSynchronize(st));   // the host tables above are stack memory
  }
  s.mfma_f4 = kernel == RBQ_SCAN_MFMA_FP4 ? 1 : 0;
  s.mf_rg = mfma_row_groups(idx->dp, s.mfma_f4 != 0, 0);
  HIPCHK(launch_debug_scan(s, (const PairRec*)w.pairs.p, (const uint64_t*)w.planes.p,
                           (const int8_t*)w.qu8.p, list, kernel, ip, pc, est, dist, lb, st));
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_seg_budget(int64_t bytes) {
  if (bytes < 0) return fail(RBQ_EINVAL, "bytes < 0");
  rbq::g_seg_budget_set(bytes);   // 0: back to the free-memory default
  return RBQ_OK;
}

extern "C" rbq_status rbq_debug_fail_alloc_after(int32_t n) {
  rbq::g_fail_alloc_after = n;
  return RBQ_OK;
}

// ------------------------------------------------------------------ profiling
void rbq::ProfState::clear() {
  for (hipEvent_t e : events)
    if (e) (void)hipEventDestroy(e);
  events.clear();
  searches = 0;
}

extern "C" rbq_status rbq_profile_enable(rbq_index* idx, int32_t on) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  std::lock_guard<std::mutex> lock(idx->mu);
  HIPCHK(hipDeviceSynchronize());
  if (on < 0 || on > RBQ_PROFILE_SCAN) return fail(RBQ_EINVAL, "profile level must be 0, 1 or 2");
  idx->prof.clear();
  idx->prof.on = on != 0;
  idx->prof.level = on;
  if (idx->prof.on) {
    HIPCHK(idx->prof.acc.ensure(16));
    HIPCHK(hipMemset(idx->prof.acc.p, 0, 16));
  }
  return RBQ_OK;
}

extern "C" rbq_status rbq_profile_read(rbq_index* idx, rbq_profile* out) {
  if (!idx || !out) return fail(RBQ_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(idx->mu);
  std::memset(out, 0, sizeof(*out));
  HIPCHK(hipDeviceSynchronize());
  ProfState& pf = idx->prof;
  out->searches = pf.searches;
  double* f[6] = {&out->ms_front, &out->ms_prep, &out->ms_scan0, &out->ms_tau, &out->ms_scan1,
                  &out->ms_finalize};
  for (size_t b = 0; b + 7 <= pf.events.size(); b += 7)
    for (int i = 0; i < 6; ++i) {
      if (!pf.events[b + i] || !pf.events[b + i + 1]) continue;
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, pf.events[b + i], pf.events[b + i + 1]));
      *f[i] += ms;
    }
  if (pf.acc.p) {
    long long acc[2];
    HIPCHK(hipMemcpy(acc, pf.acc.p, 16, hipMemcpyDeviceToHost));
    out->codes_scan0 = acc[0];
    out->codes_scan1 = acc[1];
  }
  return RBQ_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {
struct EventHolder {
  hipEvent_t e = nullptr;
  ~EventHolder() {
    if (e) (void)hipEventDestroy(e);
  }
};
}  // namespace

rbq::TuneEntry rbq_index::tuned_for(int64_t nq) const {
  rbq::TuneEntry d;
  if (tune.empty()) return d;
  for (const rbq::TuneEntry& t : tune)
    if (nq <= t.max_nq) return t;
  return tune.back();
}

extern "C" rbq_status rbq_autotune(rbq_index* idx, const float* queries, int64_t nq, int32_t k,
                                   int32_t nprobe, void* stream) {
  if (!idx || !queries) return fail(RBQ_EINVAL, "NULL argument");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nq < 1 || nq > (1ll << 24) || k < 1 || k > kMaxK || nprobe < 1 || nprobe > std::min(idx->nlist, kMaxNprobe))
    return fail(RBQ_EINVAL, "bad nq, k or nprobe");
  hipStream_t st = (hipStream_t)stream;
  TmpBuf dq, di, dd;
  const float* q = queries;
  if (!is_device_ptr(queries)) {
    HIPCHK(dq.ensure((size_t)nq * idx->dim * 4));
    HIPCHK(hipMemcpy(dq.p, queries, (size_t)nq * idx->dim * 4, hipMemcpyHostToDevice));
    q = (const float*)dq.p;
  }
  HIPCHK(di.ensure((size_t)nq * k * 8));
  HIPCHK(dd.ensure((size_t)nq * k * 4));
  EventHolder e0, e1;
  HIPCHK(hipEventCreate(&e0.e));
  HIPCHK(hipEventCreate(&e1.e));
  rbq_search_opts o;
  std::memset(&o, 0, sizeof(o));
  o.k = k;
  o.nprobe = nprobe;
  std::lock_guard<std::mutex> lock(idx->mu);
  if (idx->prof.on) return fail(RBQ_ESTATE, "profiling is enabled");
  // each trial is a whole rbq_search (validation done, sub-batches, the same
  // kernels): the best of three timed runs after one warm-up
  auto timed = [&](int64_t n, const TuneEntry& t, float* ms) -> rbq_status {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      HIPCHK(hipEventRecord(e0.e, st));
      rbq_status rs = search_locked(idx, q, n, o, (int64_t*)di.p, (float*)dd.p, nullptr, st, &t);
      if (rs != RBQ_OK) return rs;
      HIPCHK(hipEventRecord(e1.e, st));
      HIPCHK(hipEventSynchronize(e1.e));
      float v = 0.f;
      HIPCHK(hipEventElapsedTime(&v, e0.e, e1.e));
      if (rep > 0) best = std::min(best, v);
    }
    *ms = best;
    return RBQ_OK;
  };
  // batch-size buckets: powers of 8 up to the sample, and the sample itself
  std::vector<int64_t> sizes;
  for (int64_t m = 1; m < nq; m *= 8) sizes.push_back(m);
  sizes.push_back(nq);
  std::vector<TuneEntry> table;
  const int chunks[] = {256, 512, 1024, 2048};
  std::vector<int> kernels = {RBQ_SCAN_POPCNT};
  if (rbq::mfma_available()) kernels.push_back(RBQ_SCAN_MFMA);
  if (rbq::mfma_available() && idx->prm.bq <= 4) kernels.push_back(RBQ_SCAN_MFMA_FP4);
  for (int64_t m : sizes) {
    TuneEntry best;
    float best_ms = 1e30f;
    for (int c : chunks) {
      if (c > kMaxP0 + 1 - k) continue;
      for (int kern : kernels) {
        TuneEntry t;
        t.chunk = c;
        t.kernel = kern;
        t.fin_w = 0;
        float ms = 0.f;
        rbq_status rs = timed(m, t, &ms);
        if (rs != RBQ_OK) return rs;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
    // query rows per unit of the batched scan (16, 32 or 64 of them share each
    // expanded code fragment; fewer rows per unit leave more blocks per CU)
    if (best.kernel == RBQ_SCAN_MFMA || best.kernel == RBQ_SCAN_MFMA_FP4) {
      const bool f4 = best.kernel == RBQ_SCAN_MFMA_FP4;
      const int rg0 = mfma_row_groups(idx->dp, f4, 0);
      for (int rg : {1, 2, 4}) {
        if (mfma_row_groups(idx->dp, f4, rg) != rg || rg == rg0) continue;
        TuneEntry t = best;
        t.mf_rg = rg;
        float ms = 0.f;
        rbq_status rs = timed(m, t, &ms);
        if (rs != RBQ_OK) return rs;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
    // rerank waves per query (only small batches split a query's rerank)
    if (graph_rows(m) < 2048) {
      for (int w : {1, 2, 4, 8, 16, 32, 64}) {
        if (w > fin_waves(64, m, k)) break;
        TuneEntry t = best;
        t.fin_w = w;
        float ms = 0.f;
        rbq_status rs = timed(m, t, &ms);
        if (rs != RBQ_OK) return rs;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
    best.max_nq = m;
    best.ms = best_ms;
    table.push_back(best);
  }
  // each entry serves the batch sizes up to the geometric middle between its size and the next
  for (size_t i = 0; i + 1 < table.size(); ++i)
    table[i].max_nq = (int64_t)std::sqrt((double)table[i].max_nq * (double)table[i + 1].max_nq);
  table.back().max_nq = INT64_MAX;
  idx->tune = table;
  idx->graphs_clear();   // captured searches hold the old choices
  HIPCHK(hipStreamSynchronize(st));
  return RBQ_OK;
}

extern "C" rbq_status rbq_autotune_get(const rbq_index* idx, int32_t max_entries, rbq_tune_entry* entries,
                                       int32_t* count) {
  if (!idx || !count || (max_entries > 0 && !entries)) return fail(RBQ_EINVAL, "NULL argument");
  *count = (int32_t)idx->tune.size();
  for (int32_t i = 0; i < std::min<int32_t>(max_entries, *count); ++i) {
    const rbq::TuneEntry& t = idx->tune[i];
    entries[i].max_nq = t.max_nq;
    entries[i].chunk = t.chunk;
    entries[i].scan_kernel = t.kernel;
    entries[i].rerank_waves = t.fin_w;
    entries[i].ms = t.ms;
    entries[i].mfma_row_groups = t.mf_rg;
  }
  return RBQ_OK;
}
