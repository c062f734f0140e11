// Learned per-query nprobe: features, inference, GPU training (BF16 MFMA
// forward/backward, FP32 master weights, Adam) and the search hook.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rbq_mlp.hpp"
#include "rbq_runtime.hpp"

using namespace rbq;

namespace rbq {
rbq_status set_error(rbq_status st, const char* msg);
}

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

// Activations and gradients of one forward/backward over n rows.
struct Pass {
  float *A, *H, *Z, *dZ, *dH, *loss;
};

rbq_status forward(const float* X, int64_t n, const float* w, const Pass& p, const int32_t* y,
                   hipStream_t st) {
  const int N = (int)n;
  HIPCHK(launch_gemm_bf16(X, kMlpIn, 1, w + kMlpW1, kMlpHidden, 1, p.A, kMlpHidden, N, kMlpHidden,
                          kMlpIn, false, st));
  HIPCHK(launch_bias_relu(p.A, w + kMlpB1, p.H, n, kMlpHidden, st));
  HIPCHK(launch_gemm_bf16(p.H, kMlpHidden, 1, w + kMlpW2, kMlpOut, 1, p.Z, kMlpOut, N, kMlpOut,
                          kMlpHidden, false, st));
  HIPCHK(launch_softmax_ce(p.Z, w + kMlpB2, y, n, p.dZ, p.loss, st));
  return RBQ_OK;
}

rbq_status backward(const float* X, int64_t n, const float* w, const Pass& p, float* g, hipStream_t st) {
  const int N = (int)n;
  // dW2 = H^T dZ, db2 = column sums of dZ
  HIPCHK(launch_gemm_bf16(p.H, 1, kMlpHidden, p.dZ, kMlpOut, 1, g + kMlpW2, kMlpOut, kMlpHidden,
                          kMlpOut, N, false, st));
  HIPCHK(launch_colsum(p.dZ, n, kMlpOut, g + kMlpB2, st));
  // dH = dZ W2^T, masked by the ReLU
  HIPCHK(launch_gemm_bf16(p.dZ, kMlpOut, 1, w + kMlpW2, 1, kMlpOut, p.dH, kMlpHidden, N, kMlpHidden,
                          kMlpOut, false, st));
  HIPCHK(launch_relu_grad(p.dH, p.A, n * kMlpHidden, st));
  // dW1 = X^T dA, db1 = column sums of dA
  HIPCHK(launch_gemm_bf16(X, 1, kMlpIn, p.dH, kMlpHidden, 1, g + kMlpW1, kMlpHidden, kMlpIn,
                          kMlpHidden, N, false, st));
  HIPCHK(launch_colsum(p.dH, n, kMlpHidden, g + kMlpB1, st));
  return RBQ_OK;
}

size_t pass_floats(int64_t n) { return (size_t)n * (2 * kMlpHidden + 2 * kMlpOut + kMlpHidden) + 16; }

Pass carve(float* base, int64_t n) {
  Pass p;
  p.A = base;
  p.H = p.A + n * kMlpHidden;
  p.Z = p.H + n * kMlpHidden;
  p.dZ = p.Z + n * kMlpOut;
  p.dH = p.dZ + n * kMlpOut;
  p.loss = p.dH + n * kMlpHidden;
  return p;
}

// Glorot-uniform weights from a SplitMix64 counter stream, zero biases.
void init_weights(uint64_t seed, std::vector<float>& w) {
  w.assign(kMlpParams, 0.f);
  auto uni = [&](uint64_t i) {
    return (double)(host_splitmix64(seed ^ (0x4D4C500000000000ull + i)) >> 11) * (1.0 / 9007199254740992.0);
  };
  const double a1 = std::sqrt(6.0 / (kMlpIn + kMlpHidden)), a2 = std::sqrt(6.0 / (kMlpHidden + kMlpOut));
  for (int i = 0; i < kMlpIn * kMlpHidden; ++i) w[kMlpW1 + i] = (float)((2 * uni(i) - 1) * a1);
  for (int i = 0; i < kMlpHidden * kMlpOut; ++i) w[kMlpW2 + i] = (float)((2 * uni(1000000 + i) - 1) * a2);
}

// FP32 -> BF16, round to nearest even (the rounding the GEMM kernels apply
// when they stage operands).
uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace

// ------------------------------------------------------------------ search hook
namespace rbq {

// Uploads the current FP32 weights (m.host_w) and their BF16 fragment-order
// copy that the fused inference kernel reads.
rbq_status upload_model_weights(MlpState& m) {
  std::vector<uint16_t> frag(kMlpFragWords);
  for (int i = 0; i < kMlpIn; ++i)
    for (int j = 0; j < kMlpHidden; ++j)
      frag[mlp_fragment_index(1, i, j)] = bf16_rne(m.host_w[kMlpW1 + i * kMlpHidden + j]);
  for (int i = 0; i < kMlpHidden; ++i)
    for (int j = 0; j < kMlpOut; ++j)
      frag[mlp_fragment_index(2, i, j)] = bf16_rne(m.host_w[kMlpW2 + i * kMlpOut + j]);
  HIPCHK(m.w32.ensure((size_t)kMlpParams * 4));
  HIPCHK(m.wfrag.ensure(frag.size() * 2));
  HIPCHK(hipMemcpy(m.w32.p, m.host_w.data(), (size_t)kMlpParams * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(m.wfrag.p, frag.data(), frag.size() * 2, hipMemcpyHostToDevice));
  return RBQ_OK;
}

rbq_status features_into(rbq_index* idx, const float* queries, int64_t nq, int64_t qid_base,
                         float* feats, hipStream_t st) {
  const int nsel = std::min(kMlpNear, idx->nlist);
  rbq_status rs = ensure_workspace(idx, nq, nsel, 1, kDefaultChunk, false);
  if (rs != RBQ_OK) return rs;
  rs = front(idx, queries, nq, nsel, nullptr, st);
  if (rs != RBQ_OK) return rs;
  FeatDev f;
  f.stats = nullptr;
  f.feats = feats;
  f.probe_d = (const float*)idx->ws.probe_d.p;
  f.probe = (const int32_t*)idx->ws.probe.p;
  f.stride = nsel;
  f.navail = nsel;
  f.q = queries;
  f.qrot = (const float*)idx->ws.qrot.p;
  f.cent = (const float*)idx->d_cent.p;
  f.crot = (const float*)idx->d_crot.p;
  f.dim = idx->dim;
  f.dp = idx->dp;
  f.W = idx->W;
  f.nq = nq;
  f.qid_base = qid_base;
  f.seed = idx->prm.seed;
  HIPCHK(launch_features(f, st));
  return RBQ_OK;
}

rbq_status mlp_reserve(rbq_index* idx, int64_t rows) {
  HIPCHK(idx->mlp.act.ensure(pass_floats(rows) * 4));
  return RBQ_OK;
}

rbq_status predict_into(rbq_index* idx, const float* feats, int64_t nq, int nprobe_max,
                        int32_t* nprobe, float* logits, hipStream_t st) {
  MlpState& m = idx->mlp;
  HIPCHK(m.act.ensure(pass_floats(nq) * 4));
  const Pass p = carve((float*)m.act.p, nq);
  rbq_status rs = forward(feats, nq, (const float*)m.w32.p, p, nullptr, st);
  if (rs != RBQ_OK) return rs;
  if (logits) HIPCHK(hipMemcpyAsync(logits, p.Z, (size_t)nq * kMlpOut * 4, hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_policy(p.Z, nq, m.threshold, nprobe_max, nprobe, st));
  return RBQ_OK;
}

// Learned path of a search: one centroid scoring / probe selection with `stride`
// lists per query (>= 64 when the index has that many lists), then one fused
// launch computes each query's features from the nearest 64 of them, the MLP
// and the policy; the search reuses the same selection with the per-query
// nprobe. A query whose logits are not finite gets nprobe_max, the caller's
// fixed nprobe (flagged in ws.q_fb).
rbq_status learned_nprobe(rbq_index* idx, const float* queries, int64_t nq, int nprobe_max, int stride,
                          int64_t qid_base, hipStream_t st, const int32_t** out) {
  Workspace& w = idx->ws;
  HIPCHK(w.nprobe_q.ensure((size_t)nq * 4));
  HIPCHK(w.q_fb.ensure((size_t)nq * 4));
  HIPCHK(w.lstats.ensure((size_t)nq * kMlpStats * 4 * sizeof(float)));
  rbq_status rs = front(idx, queries, nq, stride, nullptr, st);
  if (rs != RBQ_OK) return rs;
  FeatDev f;
  f.stats = (float*)w.lstats.p;
  f.feats = nullptr;
  f.probe_d = (const float*)w.probe_d.p;
  f.probe = (const int32_t*)w.probe.p;
  f.stride = stride;
  f.navail = std::min(stride, kMlpNear);
  f.q = queries;
  f.qrot = (const float*)w.qrot.p;
  f.cent = (const float*)idx->d_cent.p;
  f.crot = (const float*)idx->d_crot.p;
  f.dim = idx->dim;
  f.dp = idx->dp;
  f.W = idx->W;
  f.nq = nq;
  f.qid_base = qid_base;
  f.seed = idx->prm.seed;
  HIPCHK(launch_list_stats(f, st));
  HIPCHK(launch_learned_front(f, (const uint16_t*)idx->mlp.wfrag.p, (const float*)idx->mlp.w32.p,
                              idx->mlp.threshold, nprobe_max, (int32_t*)w.nprobe_q.p, (int32_t*)w.q_fb.p, st));
  *out = (const int32_t*)w.nprobe_q.p;
  return RBQ_OK;
}

}  // namespace rbq

// ------------------------------------------------------------------ C ABI
extern "C" rbq_status rbq_nprobe_features(rbq_index* idx, const float* queries, int64_t nq,
                                          int64_t qid_base, float* feats, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(feats)) return fail(RBQ_EINVAL, "device pointers required");
  if (qid_base < 0 || qid_base + nq > (1ll << 24)) return fail(RBQ_EINVAL, "query ids must stay below 2^24");
  std::lock_guard<std::mutex> lock(idx->mu);
  return features_into(idx, queries, nq, qid_base, feats, (hipStream_t)stream);
}

extern "C" rbq_status rbq_nprobe_model_set(rbq_index* idx, const float* weights, float threshold) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!(threshold > 0.f && threshold <= 1.f)) return fail(RBQ_EINVAL, "threshold must be in (0, 1]");
  std::lock_guard<std::mutex> lock(idx->mu);
  idx->graphs_clear();   // captured searches hold the policy threshold
  MlpState& m = idx->mlp;
  if (!weights) {
    m.has_model = false;
    m.threshold = threshold;
    return RBQ_OK;
  }
  if (is_device_ptr(weights)) return fail(RBQ_EINVAL, "weights must be a host pointer");
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(weights[i])) return fail(RBQ_EINVAL, "weights contain non-finite values");
  m.host_w.assign(weights, weights + kMlpParams);
  rbq_status rs = upload_model_weights(m);
  if (rs != RBQ_OK) return rs;
  m.threshold = threshold;
  m.has_model = true;
  return RBQ_OK;
}

extern "C" rbq_status rbq_nprobe_model_get(const rbq_index* cidx, float* weights, float* threshold) {
  if (!cidx) return fail(RBQ_EINVAL, "index is NULL");
  rbq_index* idx = const_cast<rbq_index*>(cidx);
  std::lock_guard<std::mutex> lock(idx->mu);
  if (!idx->mlp.has_model) return fail(RBQ_ESTATE, "no model set");
  if (weights) std::memcpy(weights, idx->mlp.host_w.data(), (size_t)kMlpParams * 4);
  if (threshold) *threshold = idx->mlp.threshold;
  return RBQ_OK;
}

extern "C" rbq_status rbq_nprobe_predict(rbq_index* idx, const float* feats, int64_t nq,
                                         int32_t* nprobe, float* logits, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->mlp.has_model) return fail(RBQ_ESTATE, "no model set");
  if (nq < 0) return fail(RBQ_EINVAL, "nq < 0");
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(feats) || !is_device_ptr(nprobe) || (logits && !is_device_ptr(logits)))
    return fail(RBQ_EINVAL, "device pointers required");
  std::lock_guard<std::mutex> lock(idx->mu);
  const int cap = std::min(idx->nlist, 1 << 30);
  return predict_into(idx, feats, nq, std::min(cap, mlp_bucket_nprobe(kMlpOut - 1)), nprobe, logits,
                      (hipStream_t)stream);
}

extern "C" rbq_status rbq_mlp_loss_grad(const float* x, const int32_t* labels, int64_t n,
                                        const float* weights, float* grads, float* loss, void* stream) {
  if (!x || !labels || !weights || !grads || !loss) return fail(RBQ_EINVAL, "NULL argument");
  if (n < 1 || n > (1 << 24)) return fail(RBQ_EINVAL, "n out of range");
  if (!is_device_ptr(x) || !is_device_ptr(labels) || !is_device_ptr(weights) || !is_device_ptr(grads))
    return fail(RBQ_EINVAL, "x, labels, weights and grads must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  TmpBuf buf;
  HIPCHK(buf.ensure(pass_floats(n) * 4));
  const Pass p = carve((float*)buf.p, n);
  HIPCHK(hipMemsetAsync(p.loss, 0, 4, st));
  rbq_status rs = forward(x, n, weights, p, labels, st);
  if (rs == RBQ_OK) rs = backward(x, n, weights, p, grads, st);
  float ls = 0.f;
  if (rs == RBQ_OK) {
    HIPCHK(hipMemcpyAsync(&ls, p.loss, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *loss = ls / (float)n;
  }
  buf.release();
  return rs;
}

extern "C" rbq_status rbq_nprobe_model_train(rbq_index* idx, const float* feats, const int32_t* labels,
                                             int64_t n, const rbq_train_cfg* cfg, float* losses,
                                             void* stream) {
  if (!idx || !feats || !labels || !cfg) return fail(RBQ_EINVAL, "NULL argument");
  if (n < 1 || n > (1ll << 31) - 1) return fail(RBQ_EINVAL, "n out of range");
  if (cfg->epochs < 1 || cfg->batch < 1 || !(cfg->lr > 0.f)) return fail(RBQ_EINVAL, "bad training config");
  if (!is_device_ptr(feats) || !is_device_ptr(labels)) return fail(RBQ_EINVAL, "feats and labels must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  idx->graphs_clear();
  MlpState& m = idx->mlp;
  std::vector<float> w;
  init_weights(cfg->seed, w);
  HIPCHK(m.w32.ensure((size_t)kMlpParams * 4));
  HIPCHK(m.grad.ensure((size_t)kMlpParams * 4));
  HIPCHK(m.m.ensure((size_t)kMlpParams * 4));
  HIPCHK(m.v.ensure((size_t)kMlpParams * 4));
  HIPCHK(hipMemcpyAsync(m.w32.p, w.data(), (size_t)kMlpParams * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(m.m.p, 0, (size_t)kMlpParams * 4, st));
  HIPCHK(hipMemsetAsync(m.v.p, 0, (size_t)kMlpParams * 4, st));
  // Inputs are standardised per feature for training; the statistics are
  // folded into W1 and b1 afterwards, so the model consumes raw features.
  TmpBuf xs, stats;
  HIPCHK(xs.ensure((size_t)n * kMlpIn * 4));
  HIPCHK(stats.ensure((size_t)2 * kMlpIn * 4));
  float* mu = (float*)stats.p;
  float* isd = mu + kMlpIn;
  HIPCHK(launch_feat_stats(feats, n, kMlpIn, mu, isd, st));
  HIPCHK(launch_standardize(feats, n, kMlpIn, mu, isd, (float*)xs.p, st));
  feats = (const float*)xs.p;
  const int64_t B = std::min<int64_t>(cfg->batch, n);
  HIPCHK(m.act.ensure(pass_floats(B) * 4));
  const Pass p = carve((float*)m.act.p, B);
  TmpBuf xb, yb, perm;
  HIPCHK(xb.ensure((size_t)B * kMlpIn * 4));
  HIPCHK(yb.ensure((size_t)B * 4));
  HIPCHK(perm.ensure((size_t)n * 4));
  std::vector<int32_t> order(n);
  int step = 0;
  for (int e = 0; e < cfg->epochs; ++e) {
    for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {   // Fisher-Yates with a counter stream
      const uint64_t r = host_splitmix64(cfg->seed ^ (0x5348000000000000ull + ((uint64_t)e << 36) + (uint64_t)i));
      std::swap(order[i], order[r % (uint64_t)(i + 1)]);
    }
    HIPCHK(hipMemcpyAsync(perm.p, order.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(p.loss, 0, 4, st));
    for (int64_t b0 = 0; b0 < n; b0 += B) {
      const int64_t nb = std::min(B, n - b0);
      HIPCHK(launch_gather_rows(feats, labels, (const int32_t*)perm.p + b0, nb, kMlpIn, (float*)xb.p,
                                (int32_t*)yb.p, st));
      rbq_status rs = forward((const float*)xb.p, nb, (const float*)m.w32.p, p, (const int32_t*)yb.p, st);
      if (rs != RBQ_OK) return rs;
      rs = backward((const float*)xb.p, nb, (const float*)m.w32.p, p, (float*)m.grad.p, st);
      if (rs != RBQ_OK) return rs;
      HIPCHK(launch_adam((float*)m.w32.p, (const float*)m.grad.p, (float*)m.m.p, (float*)m.v.p,
                         kMlpParams, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, ++step, st));
    }
    float ls = 0.f;
    HIPCHK(hipMemcpyAsync(&ls, p.loss, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (losses) losses[e] = ls / (float)n;
  }
  m.host_w.resize(kMlpParams);
  HIPCHK(hipMemcpy(m.host_w.data(), m.w32.p, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost));
  {
    // fold the standardisation: x' = (x - mu) * isd  =>  W1[i][j] *= isd_i,
    // b1[j] -= sum_i mu_i * isd_i * W1[i][j]
    std::vector<float> hs(2 * kMlpIn);
    HIPCHK(hipMemcpy(hs.data(), stats.p, hs.size() * 4, hipMemcpyDeviceToHost));
    for (int j = 0; j < kMlpHidden; ++j) {
      double shift = 0.0;
      for (int i = 0; i < kMlpIn; ++i) {
        float& wij = m.host_w[kMlpW1 + i * kMlpHidden + j];
        wij *= hs[kMlpIn + i];
        shift += (double)hs[i] * wij;
      }
      m.host_w[kMlpB1 + j] -= (float)shift;
    }
  }
  for (float v : m.host_w)
    if (!std::isfinite(v)) {
      m.has_model = false;
      return fail(RBQ_EDEVICE, "training diverged (non-finite weights); model disabled");
    }
  rbq_status rs = upload_model_weights(m);
  if (rs != RBQ_OK) return rs;
  m.has_model = true;
  return RBQ_OK;
}

extern "C" rbq_status rbq_nprobe_bucket_table(int32_t* nprobe) {
  if (!nprobe) return fail(RBQ_EINVAL, "NULL argument");
  for (int j = 0; j < kMlpOut; ++j) nprobe[j] = mlp_bucket_nprobe(j);
  return RBQ_OK;
}

extern "C" rbq_status rbq_nprobe_labels(rbq_index* idx, const float* queries, int64_t nq, const int64_t* nn_ids,
                                        int32_t k, int32_t* labels, int32_t* need, void* stream) {
  if (!idx) return fail(RBQ_EINVAL, "index is NULL");
  if (!idx->built) return fail(RBQ_ESTATE, "index not built");
  if (nq < 0 || k < 1 || k > kMaxK) return fail(RBQ_EINVAL, "nq < 0 or k outside [1, %d]", kMaxK);
  if (nq == 0) return RBQ_OK;
  if (!is_device_ptr(queries) || !is_device_ptr(nn_ids) || !is_device_ptr(labels) || (need && !is_device_ptr(need)))
    return fail(RBQ_EINVAL, "queries, nn_ids, labels and need must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(idx->mu);
  if (!idx->d_id2list.p) {
    std::vector<int32_t> m(idx->n);
    for (int l = 0; l < idx->nlist; ++l)
      for (int64_t p = idx->h_list_off[l]; p < idx->h_list_off[l + 1]; ++p) m[idx->h_ids[p]] = l;
    HIPCHK(idx->d_id2list.ensure((size_t)idx->n * 4));
    HIPCHK(hipMemcpy(idx->d_id2list.p, m.data(), (size_t)idx->n * 4, hipMemcpyHostToDevice));
  }
  // centroid distances in sub-batches of at most 256 MiB
  const int64_t rows = std::max<int64_t>(16, std::min<int64_t>(nq, (256ll << 20) / ((int64_t)idx->nlist * 4)));
  rbq_status rs = ensure_workspace(idx, std::min(rows, nq), 1, 1, kDefaultChunk, false);
  if (rs != RBQ_OK) return rs;
  TmpBuf tmp;
  int32_t* nd = need;
  if (!nd) {
    HIPCHK(tmp.ensure((size_t)nq * 4));
    nd = (int32_t*)tmp.p;
  }
  for (int64_t q0 = 0; q0 < nq; q0 += rows) {
    const int64_t m = std::min(rows, nq - q0);
    const float* qs = queries + q0 * idx->dim;
    rs = prepare_queries(idx, qs, m, st, &qs);   // the cosine metric ranks lists for unit queries
    if (rs != RBQ_OK) return rs;
    HIPCHK(launch_centroid_dist(qs, m, idx->dim, (const float*)idx->d_centT.p, idx->probe_cnorm(), idx->nlist,
                                (float*)idx->ws.cd.p, nullptr, st, idx->cent_hi(), idx->cent_lo()));
    HIPCHK(launch_probe_need((const float*)idx->ws.cd.p, m, idx->nlist, nn_ids + q0 * k, k,
                             (const int32_t*)idx->d_id2list.p, idx->n, nd + q0, st));
  }
  HIPCHK(launch_bucket_labels(nd, nq, labels, st));
  if (tmp.p) HIPCHK(hipStreamSynchronize(st));   // tmp is freed on return
  return RBQ_OK;
}
