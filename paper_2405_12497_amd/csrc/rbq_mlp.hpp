// Learned per-query nprobe: shapes, bucket table, launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace rbq {

constexpr int kMlpIn = 96, kMlpHidden = 128, kMlpOut = 32;
constexpr int kMlpNear = 64;   // nearest centroid distances in the features
constexpr int kMlpStats = 8;   // nearest lists whose quantiser statistics are used
constexpr int kMlpW1 = 0, kMlpB1 = kMlpIn * kMlpHidden, kMlpW2 = kMlpB1 + kMlpHidden,
              kMlpB2 = kMlpW2 + kMlpHidden * kMlpOut, kMlpParams = kMlpB2 + kMlpOut;

// nprobe of bucket j: b_0 = 4, b_j = max(b_{j-1} + 1, round(4 * 2^(7j/31))).
__host__ __device__ inline int mlp_bucket_nprobe(int j) {
  int b = 4;
  for (int i = 1; i <= j; ++i) {
    const int v = (int)floor(4.0 * exp2(7.0 * i / 31.0) + 0.5);
    b = v > b + 1 ? v : b + 1;
  }
  return b;
}

struct FeatDev {
  float* feats;            // nq x 96
  const float* probe_d;    // nq x stride (nearest first)
  const int32_t* probe;    // nq x stride
  int stride, navail;
  const float* q;          // nq x dim
  const float* qrot;       // nq x dp
  const float* cent;       // nlist x dim
  const float* crot;       // nlist x dp
  int dim, dp, W;
  int64_t nq, qid_base;
  uint64_t seed;
  float* stats;            // nq x 8 x 4: {b, v_l, v_r, E[S_q] / (15 dp)} of the 8 nearest lists
};

hipError_t launch_features(const FeatDev& f, hipStream_t st);
// The quantiser statistics of each query's 8 nearest lists into f.stats, one
// wave per (query, list); launch_learned_front reads them.
hipError_t launch_list_stats(const FeatDev& f, hipStream_t st);
hipError_t launch_gemm_bf16(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                            int64_t sbn, float* C, int64_t ldc, int M, int N, int K, bool accumulate,
                            hipStream_t st);
hipError_t launch_bias_relu(float* A, const float* bias, float* H, int64_t rows, int cols, hipStream_t st);
hipError_t launch_softmax_ce(float* Z, const float* b2, const int32_t* y, int64_t n, float* dZ,
                             float* loss_sum, hipStream_t st);
hipError_t launch_relu_grad(float* dH, const float* A, int64_t total, hipStream_t st);
hipError_t launch_colsum(const float* X, int64_t rows, int cols, float* out, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t st);
hipError_t launch_gather_rows(const float* X, const int32_t* y, const int32_t* idx, int64_t n, int cols,
                              float* Xo, int32_t* yo, hipStream_t st);
hipError_t launch_feat_stats(const float* X, int64_t rows, int cols, float* mu, float* inv_sd, hipStream_t st);
hipError_t launch_standardize(const float* X, int64_t rows, int cols, const float* mu, const float* inv_sd,
                              float* Y, hipStream_t st);
// Fused learned-nprobe step after the probe selection: features, MLP and
// policy of every query in one launch. wfrag: the weights in fragment order
// (kMlpFragWords uint16, see mlp_fragment_index); w32: the FP32 weights
// (biases read from it); fallback: per query 1 when the logits were not finite.
constexpr int kMlpFragWords = (kMlpHidden / 16) * (kMlpIn / 32) * 64 * 8 + (kMlpOut / 16) * (kMlpHidden / 32) * 64 * 8;
hipError_t launch_learned_front(const FeatDev& f, const uint16_t* wfrag, const float* w32, float thr,
                                int nprobe_max, int32_t* nprobe, int32_t* fallback, hipStream_t st);
// Position in the fragment array of weight (i, j) of layer 1 (W1[i][j], i < 96
// inputs, j < 128 hidden) or layer 2 (W2[i][j], i < 128, j < 32): the B operand
// of v_mfma_f32_16x16x32_bf16 for output tile j / 16 and K step i / 32, whose
// lane (j % 16) + 16 ((i % 32) / 8) holds element (i % 32) % 8.
inline int mlp_fragment_index(int layer, int i, int j) {
  const int lane = (j % 16) + 16 * ((i % 32) / 8), e = (i % 32) % 8;
  if (layer == 1) return (((j / 16) * (kMlpIn / 32) + i / 32) * 64 + lane) * 8 + e;
  const int base = (kMlpHidden / 16) * (kMlpIn / 32) * 64 * 8;
  return base + (((j / 16) * (kMlpHidden / 32) + i / 32) * 64 + lane) * 8 + e;
}
hipError_t launch_bucket_labels(const int32_t* need, int64_t n, int32_t* labels, hipStream_t st);
hipError_t launch_policy(const float* Z, int64_t n, float thr, int nprobe_max, int32_t* out, hipStream_t st);

}  // namespace rbq
