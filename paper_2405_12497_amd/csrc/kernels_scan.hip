// Query phase on the GPU: per-(query, list) quantisation, the bit-plane
// popcount scan with the estimator epilogue, and the error-bound rerank.
//
// Work layout. Every probed (query, list) pair is cut into chunks of at most
// `chunk` codes; a chunk is one entry of a phase's unit table, which the waves
// of the persistent grid take in static round-robin. A query's chunks, in
// probe order, are numbered 0..nch-1 and its probed codes 0..ncode-1 ("query
// code space"). Each chunk owns the
// slots of its codes in a per-query candidate segment, so results land at
// positions fixed by (query, list, chunk), independent of scheduling.
//
// Rerank (Sec. 4). A code whose distance lower bound exceeds tau, the k-th
// smallest exact distance known, cannot be among the k nearest and is dropped;
// the others get their exact distance. tau must never be below the true k-th
// distance; it only controls how much is reranked:
//   phase 0: the first chunks of each query (at least k codes, nearest list
//            first) are scanned and all their codes kept as candidates;
//   tau:     the k of them with the smallest estimated distance get exact
//            distances; the k-th of those bounds the true k-th distance;
//   phase 1: the remaining chunks keep only codes with lb <= tau;
//   final:   candidates are reranked in probe order with tau tightened after
//            every round (the running k-th exact distance), giving the top-k.
#include <algorithm>

#include "rbq_internal.hpp"
#include "scan_code.hpp"
#include "wave_select.hpp"
#include "rbq_runtime.hpp"

namespace rbq {
namespace {

// <x_bar, q_bar> = k1 <x_b, q_u> + k2 popcount(x_b) + k0 with k1 = 2 Delta / sqrt(D),
// k2 = 2 v_l / sqrt(D) and k0 = -(Delta / sqrt(D)) sum(q_u) - sqrt(D) v_l
// (Sec. 3.3.1-3.3.2), in FP64; rd = sqrt(D) and ird = 1 / rd come from the host.
__device__ __forceinline__ void pair_coeffs(double vl, double delta, int sq, double rd, double ird,
                                            PairRec& r) {
  const double dr = delta * ird;
  r.k1 = (float)(2.0 * dr);
  r.k2 = (float)(2.0 * vl * ird);
  r.k0 = (float)(-dr * (double)sq - rd * vl);
}

// v_l = rmin / b and Delta = range / ((2^B_q - 1) b) of a pair, in FP64 (0 when b = 0).
__device__ __forceinline__ void pair_scalars(float rmin, float range, float b, int qmax, double& vl,
                                             double& delta) {
  vl = 0.0;
  delta = 0.0;
  if (b > 0.f) {
    const double ib = 1.0 / (double)b;
    vl = (double)rmin * ib;
    delta = (double)range * ib / (double)qmax;
  }
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

// Per (query, list) pair, Section 3.3.1: residual r = q_rot - c_rot (the
// rotated-space form of P^T (q_r - c)), b = ||r|| (= ||q_r - c|| since P is
// orthogonal), v_l / v_r = min / max of r / b, Delta = (v_r - v_l) / (2^B_q - 1)
// and the randomized rounding q_u[i] = min(2^B_q - 1, floor((r_i/b - v_l)/Delta + u_i)),
// written as s.npl bit planes (and as int8 q_u - s.qoff for the MFMA scan), plus the pair's
// estimator constants. prep_pair does this for pair g = (query q, list) from
// the residual rv (this lane's coordinates t * 64 + lane, WS >= W words, a
// compile-time bound) and the query's norm qn.
template <int WS, int NPL>
__device__ __forceinline__ void prep_pair(const SearchDev& s, int64_t g, int64_t q, int list, const float* rv,
                                          float qn) {
  const int lane = lane_id();
  const int W = s.W;
  PairRec rec;
  float rmin = rv[0], rmax = rv[0], ss = 0.f;
#pragma unroll
  for (int t = 0; t < WS; ++t) {
    if (t < W) {
      rmin = fminf(rmin, rv[t]);
      rmax = fmaxf(rmax, rv[t]);
      ss = fmaf(rv[t], rv[t], ss);
    }
  }
  float b = uniform_f32(sqrtf(wave_sum(ss)));
  // Near a centroid the rotated residual is dominated by the rotation's
  // rounding (~1e-6 (||q|| + ||c||)): take b from the raw vectors there, so
  // that b is exactly 0 when the query coincides with the centroid.
  const float scale_qc = uniform_f32(qn + sqrtf(s.cnorm[list]));
  if (b <= 1e-4f * scale_qc) {
    const float* qr = s.q + q * s.dim;
    const float* c = s.cent + (int64_t)list * s.dim;
    float acc = 0.f;
    for (int i = lane; i < s.dim; i += kWave) {
      const float d = qr[i] - c[i];
      acc = fmaf(d, d, acc);
    }
    b = uniform_f32(sqrtf(wave_sum(acc)));
  }
  rmin = wave_min(rmin);
  rmax = wave_max(rmax);
  const float range = rmax - rmin;
  const bool live = (b > 0.f) && (range > 0.f);
  const float scale = live ? (float)s.qmax / range : 0.f;
  const uint64_t qid = (uint64_t)(s.qid_base + q);
  int sq = 0;
  const int npl = NPL > 0 ? NPL : s.npl;   // bit planes (B_q), compile-time when given
  uint64_t* pl = s.planes + g * npl * W;
  int8_t* q8 = s.qu8 ? s.qu8 + g * s.dp : nullptr;
  // with the MFMA scan, only the pairs whose first chunk is a bootstrap chunk
  // (scanned by the popcount phase 0) need bit planes
  const int64_t r = g - q * s.nprobe;
  const bool planes =
      !s.boot_planes_only || uniform_i32(s.pair_choff[q * (s.nprobe + 1) + r]) < uniform_i32(s.q_p0[q]);
  float u_next = 0.f;   // word t + 1's uniform, drawn with word t's (t even)
#pragma unroll
  for (int t = 0; t < WS; ++t) {
    if (t < W) {
      const int i = t * kWave + lane;
      float u;
      if ((t & 1) == 0) {
        rounding_u2(s.seed, qid, (uint32_t)list, (uint32_t)i, u, u_next);
      } else {
        u = u_next;
      }
      // a pair that is not live has scale 0, so x = 0 and floor(u) = 0
      const float x = (rv[t] - rmin) * scale;
      const int qu = min(s.qmax, (int)floorf(x + u));
      sq += qu;
      if (q8) q8[(uint32_t)i] = (int8_t)(qu - s.qoff);
      if (!planes) continue;
      if constexpr (NPL > 0) {   // all ballots first, then one branch for the stores
        uint64_t w[NPL > 0 ? NPL : 1];
#pragma unroll
        for (int jb = 0; jb < NPL; ++jb) w[jb] = __ballot((qu >> jb) & 1);
        if (lane == 0) {
#pragma unroll
          for (int jb = 0; jb < NPL; ++jb) pl[jb * W + t] = w[jb];
        }
      } else {
        for (int jb = 0; jb < npl; ++jb) {
          const uint64_t w = __ballot((qu >> jb) & 1);
          if (lane == 0) pl[jb * W + t] = w;
        }
      }
    }
  }
  sq = wave_sum_i(sq);
  if (s.metric != 0) {   // inner product: the pair's constant M_q - <q_r, c> from the raw vectors
    const float* qr = s.q + q * s.dim;
    const float* c = s.cent + (int64_t)list * s.dim;
    float acc = 0.f;
    for (int i = lane; i < s.dim; i += kWave) acc = fmaf(qr[i], c[i], acc);
    const float gdot = wave_sum(acc);
    if (lane == 0) s.pair_pt[g] = s.q_m[q] - gdot;
  }
  if (lane == 0) {
    double vl, delta;
    pair_scalars(rmin, range, b, s.qmax, vl, delta);
    pair_coeffs(vl, delta, sq, s.rd, s.ird, rec);
    rec.b = b;
    rec.vl = (float)vl;
    rec.delta = (float)delta;
    rec.sq = sq;
    rec.list = list;
    s.pairs[g] = rec;
  }
}

// One wave per PPW consecutive pairs, residuals held in registers (each
// coordinate loaded once).
template <int WS, int PPW, int NPL>
__global__ __launch_bounds__(kThreads) void k_prep_reg(SearchDev s) {
  const int lane = lane_id();
  const int W = s.W;
  const int64_t npairs = s.nq * s.nprobe;
  // one query's pairs are consecutive: a contiguous run of blocks per XCD
  // reads the query's rotated vector into one L2
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t g0 = uniform_i64((blk * kWaves + (threadIdx.x >> 6)) * PPW);
  if (g0 >= npairs) return;
  float rv[PPW][WS];
  float qq[PPW];
  int list[PPW];
  bool act[PPW];
  // index loads first, then every coordinate load unconditionally (clamped
  // rows and words), so all of them are in flight together
  int64_t qj[PPW];
  int32_t pl_raw[PPW], npq_raw[PPW];
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
    const int64_t g = min(g0 + j, npairs - 1);
    qj[j] = g / s.nprobe;
    pl_raw[j] = s.probe[g];
    npq_raw[j] = s.nprobe_q ? s.nprobe_q[qj[j]] : s.nprobe;
  }
  bool any = false;
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
    const int64_t g = g0 + j;
    const int r = (int)(min(g, npairs - 1) - qj[j] * s.nprobe);
    const int P = min(max(npq_raw[j], 1), s.nprobe);
    list[j] = uniform_i32((g < npairs && r < P) ? pl_raw[j] : -1);
    act[j] = list[j] >= 0;
    any = any || act[j];
  }
  if (!any) {   // probe slots past the query's nprobe: empty records, no coordinate reads
    if (lane < PPW && g0 + lane < npairs) {
      PairRec rec;
      rec.k1 = rec.k2 = rec.k0 = rec.b = rec.vl = rec.delta = 0.f;
      rec.sq = 0;
      rec.list = -1;
      s.pairs[g0 + lane] = rec;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
    qq[j] = 0.f;
    const float* qrot = s.qrot + qj[j] * s.dp;
    const float* crot = s.crot + (int64_t)max(list[j], 0) * s.dp;
    // all words' reads issued before any is used (used one by one, each
    // would wait for its own round trip)
    float xs[WS], cs[WS];
#pragma unroll
    for (int t = 0; t < WS; ++t) {
      const int tt = min(t, W - 1);
      // wave-uniform row bases, 32-bit lane offsets (scalar-base loads)
      const uint32_t off = 4u * (uint32_t)(tt * kWave + lane);
      xs[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(qrot) + off);
      cs[t] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(crot) + off);
    }
#pragma unroll
    for (int t = 0; t < WS; ++t) {
      keep_loaded(xs[t]);
      keep_loaded(cs[t]);
    }
#pragma unroll
    for (int t = 0; t < WS; ++t) {
      const bool in = t < W;
      rv[j][t] = in ? xs[t] - cs[t] : 0.f;
      qq[j] = in ? fmaf(xs[t], xs[t], qq[j]) : qq[j];
    }
  }
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
    const int64_t g = g0 + j;
    if (g >= npairs) break;
    if (!act[j]) {
      PairRec rec;
      if (lane == 0) {
        rec.k1 = rec.k2 = rec.k0 = rec.b = rec.vl = rec.delta = 0.f;
        rec.sq = 0;
        rec.list = -1;
        s.pairs[g] = rec;
      }
      continue;
    }
    prep_pair<WS, NPL>(s, g, g / s.nprobe, list[j], rv[j], sqrtf(wave_sum(qq[j])));
  }
}

// Row-local (16-lane DPP row) integer reductions; every lane of the row gets
// the result.
__device__ __forceinline__ uint32_t row_or_u32(uint32_t v) {
  int x = (int)v;
  x |= dpp_i32<kDppXor1>(x);
  x |= dpp_i32<kDppXor2>(x);
  x |= dpp_i32<kDppHalfMirror>(x);
  x |= dpp_i32<kDppMirror>(x);
  return (uint32_t)x;
}
__device__ __forceinline__ int row_sum_i32(int x) {
  x += dpp_i32<kDppXor1>(x);
  x += dpp_i32<kDppXor2>(x);
  x += dpp_i32<kDppHalfMirror>(x);
  x += dpp_i32<kDppMirror>(x);
  return x;
}
__device__ __forceinline__ float row_sum_f32(float v) {
  return row_reduce(v, [](float a, float b) { return a + b; });
}

// Quarter-wave form of the same per-pair quantisation for W <= 4 (D <= 256):
// the 16 lanes of a DPP row own one pair (lane l of the row holds coordinates
// 64 t + l + 16 j, j < 4, of every word t), so a pair's reductions are four
// row-local DPP steps, its plane words are row-local ORs, and one wave
// quantises four pairs at once. The per-coordinate arithmetic (residual,
// scale, randomized rounding) is that of k_prep_reg; only the summation
// order of ||r||^2 differs. Every lane stays active around the DPP steps:
// per-row conditions are applied as values, not branches.
// QU8: also store the int8 codes q_u (the MFMA scan's operand). blk: the
// block's index among the quantisation blocks of its launch.
template <int W, bool QU8>
__device__ __forceinline__ void prep_q_body(const SearchDev& s, int64_t blk) {
  const int lane = lane_id(), row = lane >> 4, l = lane & 15;
  const int64_t npairs = s.nq * s.nprobe;
  const int64_t g0 = uniform_i64((blk * kWaves + (threadIdx.x >> 6)) * 4);
  if (g0 >= npairs) return;   // whole waves
  const int64_t g = g0 + row;
  const bool valid = g < npairs;
  const int64_t gc = min(g, npairs - 1);
  const int64_t q = gc / s.nprobe;
  const int r = (int)(gc - q * s.nprobe);
  const int npq = s.nprobe_q ? s.nprobe_q[q] : s.nprobe;
  const int pl_raw = s.probe[gc];
  const int P = min(max(npq, 1), s.nprobe);
  const int list = (valid && r < P) ? pl_raw : -1;
  const bool act = list >= 0;
  const float* qrot = s.qrot + q * s.dp;
  const float* crot = s.crot + (int64_t)max(list, 0) * s.dp;
  const float cn = s.cnorm[max(list, 0)];
  float rv[W][4];
  float rmin = __builtin_inff(), rmax = -__builtin_inff(), ss = 0.f, qq = 0.f;
#pragma unroll
  for (int t = 0; t < W; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = t * kWave + l + 16 * j;
      const float x = qrot[i];
      rv[t][j] = x - crot[i];
      ss = fmaf(rv[t][j], rv[t][j], ss);
      qq = fmaf(x, x, qq);
      rmin = fminf(rmin, rv[t][j]);
      rmax = fmaxf(rmax, rv[t][j]);
    }
  ss = row_sum_f32(ss);
  qq = row_sum_f32(qq);
  rmin = row_reduce(rmin, [](float a, float b) { return fminf(a, b); });
  rmax = row_reduce(rmax, [](float a, float b) { return fmaxf(a, b); });
  float b = sqrtf(ss);
  // near a centroid: b from the raw vectors (see k_prep_reg)
  const bool degen = act && b <= 1e-4f * (sqrtf(qq) + sqrtf(cn));
  if (__ballot(degen)) {
    float acc = 0.f;
    if (degen) {
      const float* qr = s.q + q * s.dim;
      const float* c = s.cent + (int64_t)list * s.dim;
      for (int i = l; i < s.dim; i += 16) {
        const float d = qr[i] - c[i];
        acc = fmaf(d, d, acc);
      }
    }
    acc = row_sum_f32(acc);
    if (degen) b = sqrtf(acc);
  }
  const float range = rmax - rmin;
  const bool live = act && (b > 0.f) && (range > 0.f);
  const float scale = live ? (float)s.qmax / range : 0.f;   // B_q <= 4 on this path (s.npl == 4)
  const uint64_t qid = (uint64_t)(s.qid_base + q);
  int8_t* q8 = QU8 ? s.qu8 + gc * s.dp : nullptr;
  int sq = 0;
  uint64_t myword = 0;   // lane l < 4 W of the row: plane word l (= plane jb * W + word t)
  float u_next[4] = {0.f, 0.f, 0.f, 0.f};   // word t + 1's uniforms, drawn with word t's (t even)
#pragma unroll
  for (int t = 0; t < W; ++t) {
    int qu[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = t * kWave + l + 16 * j;
      float u;
      if ((t & 1) == 0) {
        rounding_u2(s.seed, qid, (uint32_t)max(list, 0), (uint32_t)i, u, u_next[j]);
      } else {
        u = u_next[j];
      }
      // a pair that is not live has scale 0, so x = 0 and floor(u) = 0
      const float x = (rv[t][j] - rmin) * scale;
      qu[j] = min(s.qmax, (int)floorf(x + u));
      sq += qu[j];
      if (QU8 && act) q8[i] = (int8_t)(qu[j] - s.qoff);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const uint32_t lo = (((uint32_t)qu[0] >> jb) & 1u) << l | (((uint32_t)qu[1] >> jb) & 1u) << (l + 16);
      const uint32_t hi = (((uint32_t)qu[2] >> jb) & 1u) << l | (((uint32_t)qu[3] >> jb) & 1u) << (l + 16);
      const uint64_t w = ((uint64_t)row_or_u32(hi) << 32) | row_or_u32(lo);
      if (l == jb * W + t) myword = w;
    }
  }
  sq = row_sum_i32(sq);
  if (s.metric != 0) {   // inner product: the pair's constant M_q - <q_r, c> (every lane takes part)
    const float* qr = s.q + q * s.dim;
    const float* c = s.cent + (int64_t)max(list, 0) * s.dim;
    float acc = 0.f;
    for (int i = l; i < s.dim; i += 16) acc = fmaf(qr[i], c[i], acc);
    acc = row_sum_f32(acc);
    if (act && l == 0) s.pair_pt[g] = s.q_m[q] - acc;
  }
  if (act && l < 4 * W) s.planes[g * 4 * W + l] = myword;
  if (valid && l == 0) {
    PairRec rec;
    if (!act) {
      rec.k1 = rec.k2 = rec.k0 = rec.b = rec.vl = rec.delta = 0.f;
      rec.sq = 0;
      rec.list = -1;
    } else {
      double vl, delta;
      pair_scalars(rmin, range, b, s.qmax, vl, delta);
      pair_coeffs(vl, delta, sq, s.rd, s.ird, rec);
      rec.b = b;
      rec.vl = (float)vl;
      rec.delta = (float)delta;
      rec.sq = sq;
      rec.list = list;
    }
    s.pairs[g] = rec;
  }
}

template <int W, bool QU8>
__global__ __launch_bounds__(kThreads) void k_prep_q(SearchDev s) {
  prep_q_body<W, QU8>(s, blockIdx.x);
}

// ------------------------------------------------------------------ planning
// One wave per query: chunk and code prefixes over its probed pairs (64 ranks
// per step, shuffle scans), and the bootstrap: whole chunks in probe order up
// to the first chunk at which the covered codes reach s.boot.
__global__ __launch_bounds__(kThreads) void k_plan(SearchDev s) {
  const int64_t q = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (q >= s.nq) return;   // whole waves
  const int lane = lane_id();
  int P = s.nprobe;
  if (s.nprobe_q) P = uniform_i32(min(max(s.nprobe_q[q], 1), s.nprobe));
  int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
  int32_t* codeoff = s.pair_codeoff + q * (s.nprobe + 1);
  int32_t ch = 0, code = 0, p0 = -1, n0 = 0;   // wave-uniform running values
  for (int r0 = 0; r0 < s.nprobe; r0 += kWave) {
    const int r = r0 + lane;
    int n = 0, nc = 0;
    const int list = (r < P) ? s.probe[q * s.nprobe + r] : -1;
    if (list >= 0) {
      n = s.list_off[list + 1] - s.list_off[list];
      nc = (n + s.chunk - 1) / s.chunk;
    }
    int in = n, ic = nc;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int yn = __shfl_up(in, o, kWave), yc = __shfl_up(ic, o, kWave);
      if (lane >= o) {
        in += yn;
        ic += yc;
      }
    }
    const int exn = code + in - n, exc = ch + ic - nc;
    if (r < s.nprobe) {
      choff[r] = exc;
      codeoff[r] = exn;
    }
    if (p0 < 0) {
      const uint64_t m = __ballot(r < s.nprobe && exn + n >= s.boot);
      if (m) {
        const int l = __ffsll((long long)m) - 1;   // first rank whose codes reach boot
        const int exn_l = __shfl(exn, l, kWave), exc_l = __shfl(exc, l, kWave), n_l = __shfl(n, l, kWave);
        const int cstar = (s.boot - exn_l + s.chunk - 1) / s.chunk - 1;
        p0 = uniform_i32(exc_l + cstar + 1);
        n0 = uniform_i32(exn_l + min((cstar + 1) * s.chunk, n_l));
      }
    }
    code = uniform_i32(code + __shfl(in, kWave - 1, kWave));
    ch = uniform_i32(ch + __shfl(ic, kWave - 1, kWave));
  }
  if (p0 < 0) {   // fewer than boot codes probed: everything is bootstrap
    p0 = ch;
    n0 = code;
  }
  if (lane == 0) {
    choff[s.nprobe] = ch;
    codeoff[s.nprobe] = code;
    s.q_nch[q] = ch;
    s.q_p0[q] = p0;
    s.q_n0[q] = n0;
    s.q_ncode[q] = code;
  }
}

// k_plan for a wide probe (nprobe > kPlanWaveMax), one block per query:
// thread t takes a contiguous run of ranks, the block scans the runs' chunk
// and code counts, and the first rank whose codes reach s.boot (block
// minimum) fixes the bootstrap. Same outputs as k_plan.
constexpr int kPlanWaveMax = 1024;
constexpr int kPlanThreads = 1024;
constexpr int kPlanPer = 16;   // ranks per thread
static_assert(kMaxNprobe <= kPlanThreads * kPlanPer, "k_plan_block covers every rank");

// The query's list sizes are gathered once by rank-strided threads (reads of
// the probe row coalesced) into LDS, each thread then scans its contiguous run
// from LDS (rows padded by one word per 16 so the runs fall in distinct
// banks), and the offsets go back out rank-strided: the one CU running the
// block does not serve 64 cache lines per load and store.
__host__ __device__ inline int plan_pad(int r) { return r + (r >> 4); }
constexpr size_t kPlanLdsBytes = 2 * (size_t)(kMaxNprobe + kMaxNprobe / 16 + 1) * sizeof(int32_t);

__global__ __launch_bounds__(kPlanThreads) void k_plan_block(SearchDev s) {
  extern __shared__ int32_t plan_lds[];
  __shared__ int32_t wsum[kPlanThreads / kWave][2];
  __shared__ int32_t sh_rstar, sh_p0, sh_n0;
  const int64_t q = blockIdx.x;
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  int P = s.nprobe;
  if (s.nprobe_q) P = min(max(s.nprobe_q[q], 1), s.nprobe);
  const int np = s.nprobe;
  int32_t* lco = plan_lds;                      // sizes, then code offsets
  int32_t* lch = plan_lds + plan_pad(np) + 1;   // chunk offsets
  int32_t* choff = s.pair_choff + q * (np + 1);
  int32_t* codeoff = s.pair_codeoff + q * (np + 1);
  {
    // rank t + kPlanThreads i: clamped reads all in flight, then masks
    int lid[kPlanPer];
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) lid[i] = s.probe[q * np + min(t + kPlanThreads * i, np - 1)];
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) keep_loaded(lid[i]);
    int lo[kPlanPer], hi[kPlanPer];
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) {
      const int l = max(lid[i], 0);
      lo[i] = s.list_off[l];
      hi[i] = s.list_off[l + 1];
    }
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) {
      const int r = t + kPlanThreads * i;
      if (r < np) lco[plan_pad(r)] = (r < P && lid[i] >= 0) ? hi[i] - lo[i] : 0;
    }
  }
  if (t == 0) sh_rstar = INT32_MAX;
  __syncthreads();
  const int per = (np + kPlanThreads - 1) / kPlanThreads;
  const int r0 = min(t * per, np), r1 = min(r0 + per, np);
  int ln[kPlanPer];
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) ln[i] = r0 + i < r1 ? lco[plan_pad(r0 + i)] : 0;
  int sn = 0, sc = 0;
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    sn += ln[i];
    sc += (ln[i] + s.chunk - 1) / s.chunk;
  }
  // block exclusive scan of (sc, sn)
  int ic = sc, in = sn;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int yc = __shfl_up(ic, o, kWave), yn = __shfl_up(in, o, kWave);
    if (lane >= o) {
      ic += yc;
      in += yn;
    }
  }
  if (lane == kWave - 1) {
    wsum[wave][0] = ic;
    wsum[wave][1] = in;
  }
  __syncthreads();
  int bc = 0, bn = 0, tc = 0, tn = 0;
  for (int w = 0; w < kPlanThreads / kWave; ++w) {
    bc += w < wave ? wsum[w][0] : 0;
    bn += w < wave ? wsum[w][1] : 0;
    tc += wsum[w][0];
    tn += wsum[w][1];
  }
  int exc = bc + ic - sc, exn = bn + in - sn;
  int first = INT32_MAX, f_exc = 0, f_exn = 0, f_n = 0;
#pragma unroll
  for (int i = 0; i < kPlanPer; ++i) {
    const int r = r0 + i, n = ln[i], nc = (n + s.chunk - 1) / s.chunk;
    if (r < r1) {
      lch[plan_pad(r)] = exc;
      lco[plan_pad(r)] = exn;   // its own size was read above
      // the first rank reaching boot codes is the one rank whose exclusive
      // count is below boot and inclusive count is not (counts only grow)
      if (exn < s.boot && exn + n >= s.boot) {
        first = r;
        f_exc = exc;
        f_exn = exn;
        f_n = n;
      }
    }
    exc += nc;
    exn += n;
  }
  if (first != INT32_MAX) {   // a single thread
    sh_rstar = first;
    const int cstar = (s.boot - f_exn + s.chunk - 1) / s.chunk - 1;
    sh_p0 = f_exc + cstar + 1;
    sh_n0 = f_exn + min((cstar + 1) * s.chunk, f_n);
  }
  __syncthreads();
  for (int r = t; r < np; r += kPlanThreads) {
    choff[r] = lch[plan_pad(r)];
    codeoff[r] = lco[plan_pad(r)];
  }
  if (t == 0) {
    const bool boot_all = sh_rstar == INT32_MAX;   // fewer than boot codes probed: all bootstrap
    choff[np] = tc;
    codeoff[np] = tn;
    s.q_nch[q] = tc;
    s.q_p0[q] = boot_all ? tc : sh_p0;
    s.q_n0[q] = boot_all ? tn : sh_n0;
    s.q_ncode[q] = tn;
  }
}

// Exclusive prefix sums over queries of five per-query counts (chunks,
// bootstrap chunks, other chunks, codes, bootstrap codes), in two launches
// over blocks of kOffQ queries (thread t: queries 4t..4t+3 of the block):
// k_offsets_sum writes each block's five sums; k_offsets_scan adds the sums
// of the blocks before it and scans its own queries (shuffle scan in each
// wave, then the four wave totals).
constexpr int kOffThreads = kOffQ / 4;

__device__ __forceinline__ void off_counts(const SearchDev& s, int64_t q, int64_t (&v)[5]) {
  // clamped loads, then masks (loads under a branch would each wait at its join)
  const bool in = q < s.nq;
  const int64_t qc = min(q, s.nq - 1);
  const int64_t nch = s.q_nch[qc], p0 = s.q_p0[qc], ncode = s.q_ncode[qc], n0 = s.q_n0[qc];
  v[0] = in ? nch : 0;
  v[1] = in ? p0 : 0;
  v[2] = in ? nch - p0 : 0;
  v[3] = in ? ncode : 0;
  v[4] = in ? n0 : 0;
}

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kOffThreads) void k_offsets_sum(SearchDev s) {
  __shared__ int64_t wtot[kOffThreads / kWave][5];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  if (blockIdx.x == 0 && t == 0) {
    s.counters[0] = 0;
    s.counters[1] = 0;
  }
  const int64_t q0 = (int64_t)blockIdx.x * kOffQ + (int64_t)t * 4;
  int64_t sum[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int64_t v[5];
    off_counts(s, q0 + u, v);
#pragma unroll
    for (int a = 0; a < 5; ++a) sum[a] += v[a];
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    int64_t x = sum[a];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    if (lane == 0) wtot[wave][a] = x;
  }
  __syncthreads();
  if (t < 5) {
    int64_t x = 0;
    for (int w = 0; w < kOffThreads / kWave; ++w) x += wtot[w][t];
    s.blk_sums[(int64_t)blockIdx.x * 5 + t] = x;
  }
}

__global__ __launch_bounds__(kOffThreads) void k_offsets_scan(SearchDev s) {
  __shared__ int64_t wtot[kOffThreads / kWave][5];
  __shared__ int64_t carry[5];
  const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
  constexpr int kNW = kOffThreads / kWave;
  // carry: the sums of the blocks before this one
  {
    int64_t c[5] = {0, 0, 0, 0, 0};
    for (int b = t; b < (int)blockIdx.x; b += kOffThreads)
#pragma unroll
      for (int a = 0; a < 5; ++a) c[a] += s.blk_sums[(int64_t)b * 5 + a];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      int64_t x = c[a];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
      if (lane == 0) wtot[wave][a] = x;
    }
    __syncthreads();
    if (t < 5) {
      int64_t x = 0;
      for (int w = 0; w < kNW; ++w) x += wtot[w][t];
      carry[t] = x;
    }
    __syncthreads();
  }
  const int64_t q0 = (int64_t)blockIdx.x * kOffQ + (int64_t)t * 4;
  int64_t v[4][5];
#pragma unroll
  for (int u = 0; u < 4; ++u) off_counts(s, q0 + u, v[u]);
  int64_t sum[5], inc[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    sum[a] = v[0][a] + v[1][a] + v[2][a] + v[3][a];
    inc[a] = wave_incl_scan_i64(sum[a]);
  }
  __syncthreads();   // the carry reduction's wtot reads are done
  if (lane == kWave - 1)
#pragma unroll
    for (int a = 0; a < 5; ++a) wtot[wave][a] = inc[a];
  __syncthreads();
  int64_t* outs[5] = {s.off_ch, s.off_p0, s.off_p1, s.off_seg, s.off_n0};
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    int64_t before = carry[a], total = carry[a];
#pragma unroll
    for (int w = 0; w < kNW; ++w) {
      before += (w < wave) ? wtot[w][a] : 0;
      total += wtot[w][a];
    }
    int64_t run = before + inc[a] - sum[a];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (q0 + u < s.nq) outs[a][q0 + u] = run;
      run += v[u][a];
    }
    if (blockIdx.x == gridDim.x - 1 && t == 0) outs[a][s.nq] = total;
  }
}

// A lane per probe rank: the descriptors of its chunks,
// bootstrap ones to units0 (at off_p0[q]) and, for the popcount main phase,
// the others to units1 (at off_p1[q]); and each chunk's first query-code
// index, for finalize.
// One wave per (query, 64 probe ranks): the descriptors of those ranks' chunks.
__device__ __forceinline__ void units_body(const SearchDev& s, int64_t blk) {
  const int nrb = (s.nprobe + kWave - 1) / kWave;
  const int64_t w = blk * kWaves + (threadIdx.x >> 6);
  if (w >= s.nq * (int64_t)nrb) return;   // whole waves
  const int64_t q = w / nrb;
  const int lane = lane_id();
  const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
  const int32_t* codeoff = s.pair_codeoff + q * (s.nprobe + 1);
  const int p0 = s.q_p0[q];
  const int64_t b0 = s.off_p0[q], b1 = s.off_p1[q];
  const int64_t seg0 = s.off_seg[q], n00 = s.off_n0[q], ch0 = s.off_ch[q];
  {
    const int r = (int)(w % nrb) * kWave + lane;
    if (r >= s.nprobe) return;
    const int c0 = choff[r], nc = choff[r + 1] - c0;
    if (nc == 0) return;
    const int64_t g = q * s.nprobe + r;
    const int list = s.probe[g];   // a rank with chunks is an active one
    const int64_t lbeg = s.list_off[list];
    const int n = s.list_off[list + 1] - s.list_off[list];
    for (int c = 0; c < nc; ++c) {
      const int j = c0 + c;
      UnitDesc d;
      d.start = lbeg + (int64_t)c * s.chunk;
      d.len = min(s.chunk, n - c * s.chunk);
      d.g = g;
      d.qcode = (int64_t)codeoff[r] + (int64_t)c * s.chunk;
      d.seg = seg0 + d.qcode;
      d.p0slot = n00 + d.qcode;
      d.count_slot = ch0 + j;
      d.q = (int32_t)q;
      d.pad = 0;
      s.chunk_qcode[ch0 + j] = (int32_t)d.qcode;
      // with the batched scan (boot_planes_only) the main phase takes its
      // work from the pairs grouped by list, so only bootstrap units are built
      if (j < p0) {
        s.units0[b0 + j] = d;
      } else if (!s.boot_planes_only) {
        s.units1[b1 + (j - p0)] = d;
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_units(SearchDev s) { units_body(s, blockIdx.x); }

// The unit descriptors and the per-pair quantisation are independent (both
// follow the offsets): one launch, the units' blocks first, so each fills the
// other's idle issue slots.
template <int W, bool QU8>
__global__ __launch_bounds__(kThreads) void k_prep_units(SearchDev s, int64_t nunit_blocks) {
  if ((int64_t)blockIdx.x < nunit_blocks)
    units_body(s, blockIdx.x);
  else
    prep_q_body<W, QU8>(s, (int64_t)blockIdx.x - nunit_blocks);
}

// ------------------------------------------------------------------ exact distance
// Squared distances of up to NC raw vectors (list-order positions pos[j],
// -1 = none) to the query, by a group of 8 consecutive lanes: lane `sub`
// accumulates the columns sub, sub + 8, ... (float4 columns when rows are
// 16-byte aligned) in order, then the group reduces by xor-shuffles 4, 2, 1.
// U columns per lane are loaded per round trip, for all NC vectors together
// (columns past the row read its last one and add 0), so a pass costs
// ceil(D / (32 U)) round trips; the order of the additions does not depend on
// U. Every exact distance on the device comes from this routine, so equal
// vectors get equal bits.
constexpr int kLpc = 8;

// One column's contribution: (a - b)^2 for squared L2, a b for the inner
// product (whose searched "distance" is M_q minus the sum, clamped at 0).
template <bool IP>
__device__ __forceinline__ void acc1(float& acc, float a, float b) {
  if constexpr (IP) {
    acc = fmaf(a, b, acc);
  } else {
    const float d = a - b;
    acc = fmaf(d, d, acc);
  }
}
template <bool IP>
__device__ __forceinline__ void acc4(float& acc, const float4& a, const float4& b) {
  acc1<IP>(acc, a.x, b.x);
  acc1<IP>(acc, a.y, b.y);
  acc1<IP>(acc, a.z, b.z);
  acc1<IP>(acc, a.w, b.w);
}

template <int NC, int U = 1, bool IP = false>
__device__ __forceinline__ void group_dists(const float* __restrict__ raw, const int32_t (&pos)[NC], int dim,
                                            const float* __restrict__ qv, int sub, float (&out)[NC], float mq = 0.f) {
  float acc[NC];
  int64_t base[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    acc[j] = 0.f;
    base[j] = (int64_t)(pos[j] >= 0 ? pos[j] : 0) * dim;   // absent entries read row 0
  }
  if constexpr (U == 1) {
    if ((dim & 3) == 0) {
      const float4* q4 = reinterpret_cast<const float4*>(qv);
      for (int i = sub; i < (dim >> 2); i += kLpc) {
        const float4 b = q4[i];
        float4 a[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) a[j] = reinterpret_cast<const float4*>(raw + base[j])[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          acc4<IP>(acc[j], a[j], b);
        }
      }
    } else {
      for (int i = sub; i < dim; i += kLpc) {
        const float b = qv[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          acc1<IP>(acc[j], raw[base[j] + i], b);
        }
      }
    }
  } else if ((dim & 3) == 0) {
    const int n4 = dim >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(qv);
    for (int i0 = 0; i0 < n4; i0 += U * kLpc) {
      float4 b[U], a[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u * kLpc + sub, n4 - 1);
        b[u] = q4[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) a[u][j] = reinterpret_cast<const float4*>(raw + base[j])[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = i0 + u * kLpc + sub < n4;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float4 z = {0.f, 0.f, 0.f, 0.f};
          acc4<IP>(acc[j], live ? a[u][j] : (IP ? z : b[u]), b[u]);
        }
      }
    }
  } else {
    for (int i0 = 0; i0 < dim; i0 += U * kLpc) {
      float b[U], a[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u * kLpc + sub, dim - 1);
        b[u] = qv[i];
#pragma unroll
        for (int j = 0; j < NC; ++j) a[u][j] = raw[base[j] + i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = i0 + u * kLpc + sub < dim;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          acc1<IP>(acc[j], live ? a[u][j] : (IP ? 0.f : b[u]), b[u]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    float v = acc[j];
    v += __shfl_xor(v, 4, kWave);
    v += __shfl_xor(v, 2, kWave);
    v += __shfl_xor(v, 1, kWave);
    out[j] = IP ? fmaxf(mq - v, 0.f) : v;
  }
}

// Exact-distance shape of tau and finalize: narrow rows (D <= 256) take passes
// of 64 vectors with one column per lane per round trip; wide rows passes of
// 32 vectors with four columns per lane per round trip (the same bytes in
// flight, a quarter of the round trips).
template <bool WIDE>
struct DistShape {
  static constexpr int kMaxNC = WIDE ? 4 : 8;
  static constexpr int kU = WIDE ? 4 : 1;
};
inline bool dist_wide(int dim) { return dim > 256; }

// Low word of an id (ids are below 2^31): a 4-byte load instead of 8.
__device__ __forceinline__ uint32_t id_lo32(const int64_t* ids, int64_t i) {
  return reinterpret_cast<const uint32_t*>(ids)[2 * i];
}

// Float bits mapped to unsigned integers that order like the floats.
__device__ __forceinline__ uint32_t sortable_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------ bootstrap tau
// One wave per query (four per block, no block barriers). The m = min(n0,
// 4k, kMaxK) bootstrap codes with the smallest estimated distance (ties by
// bootstrap order) get their exact distance, by 8 groups of 8 lanes; the k
// best of them by (distance, id) seed the top-k and tau = the k-th. The others
// cannot enter the top-k (k better ones are known), so all m segment entries
// are marked done (pos = -1).
// With W > 1 (small batches, large k), W waves share a query: each makes the
// same selection, reranks its share [m w / W, m (w + 1) / W) of it and writes
// those exact keys to tpart (stride min(kMaxK, 4k) per query); k_tau_merge
// sorts them and writes the seeds and tau.
template <bool WIDE>
__global__ __launch_bounds__(kThreads) void k_tau(SearchDev s, int W, uint64_t* __restrict__ tpart) {
  using DS = DistShape<WIDE>;
  __shared__ uint64_t selw[kWaves][kWSelCap];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t wid = (int64_t)blockIdx.x * kWaves + wave;
  if (wid >= s.nq * W) return;   // whole waves
  const int64_t q = wid / W;
  const int wsub = (int)(wid - q * W);
  uint64_t* sel = selw[wave];
  const int n0 = uniform_i32(s.q_n0[q]);
  const int64_t b0 = uniform_i64(s.off_n0[q]);
  const int mstride = min(kMaxK, 4 * s.k);
  const int m = min(n0, mstride);
  const int lo = (int)((int64_t)m * wsub / W), hi = (int)((int64_t)m * (wsub + 1) / W);
  if (wsub == 0 && lane == 0) s.q_boot[q] = m;   // exact distances of the bootstrap rerank
  if (m > 0) {
    const EstEnt* est = s.p0buf + b0;
    wave_smallest<8, kMaxP0 / kWave>([&](int i) { return __float_as_uint(est[i].dist); },
                                     [](uint32_t v) { return sortable_bits(__uint_as_float(v)); }, n0, m, sel);
    const int64_t seg0 = uniform_i64(s.off_seg[q]);
    const float* qv = s.q + q * s.dim;
    const int grp = lane / kLpc, sub = lane % kLpc;
    constexpr int kGroups = kWave / kLpc;
    // passes over the wave's share [lo, hi): entry base + grp + 8 j, j < NC (a
    // bootstrap entry's index is its slot in the query's segment)
    auto run = [&](int base, auto nc_tag) {
      constexpr int NC = decltype(nc_tag)::value;
      int32_t slot[NC], pos[NC];
      // clamped reads, then masks: reads under per-entry branches would each
      // wait at the branch's join
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int i = base + grp + j * kGroups;
        slot[j] = (int32_t)(uint32_t)(sel[min(i, hi - 1)] & 0xffffffffu);
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) pos[j] = est[slot[j]].pos;
#pragma unroll
      for (int j = 0; j < NC; ++j) keep_loaded(pos[j]);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const bool in = base + grp + j * kGroups < hi;
        slot[j] = in ? slot[j] : -1;
        pos[j] = in ? pos[j] : -1;
      }
      // the ids travel with the raw vectors (one round trip for both)
      uint32_t id[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) id[j] = id_lo32(s.ids, max(pos[j], 0));
      float d[NC];
      if (s.metric != 0) {
        group_dists<NC, DS::kU, true>(s.raw, pos, s.dim, qv, sub, d, uniform_f32(s.q_m[q]));
      } else {
        group_dists<NC, DS::kU, false>(s.raw, pos, s.dim, qv, sub, d);
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) keep_loaded(id[j]);
      wave_lds_sync();   // every lane has read its sel entries
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int i = base + grp + j * kGroups;
        // exact distances are >= 0, so their bits order like the values; ids < 2^31
        const uint64_t v = ((uint64_t)__float_as_uint(d[j]) << 32) | id[j];
        if (sub == 0 && i < hi) {
          s.seg[seg0 + slot[j]].pos = -1;
          sel[i] = v;
        }
      }
      wave_lds_sync();
    };
    for (int base = lo; base < hi; base += kGroups * DS::kMaxNC) {
      const int per = (min(hi - base, kGroups * DS::kMaxNC) + kGroups - 1) / kGroups;
      if (per <= 1) run(base, IntC<1>{});
      else if (per <= 2) run(base, IntC<2>{});
      else if (per <= 4 || DS::kMaxNC == 4) run(base, IntC<4>{});
      else run(base, IntC<DS::kMaxNC>{});
    }
    if (W > 1) {
      for (int i = lo + lane; i < hi; i += kWave) tpart[q * mstride + i] = sel[i];
      return;
    }
    wave_sort_sel(sel, m);
  } else if (W > 1) {
    return;   // the merge writes the empty seeds
  }
  for (int i = lane; i < s.k; i += kWave) {
    SeedEnt e;
    const bool live = i < min(m, s.k);
    const uint64_t v = live ? sel[i] : 0;
    e.dist = live ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
    e.id = live ? (int32_t)(uint32_t)(v & 0xffffffffu) : -1;
    s.seedk[q * s.k + i] = e;
  }
  if (lane == 0) s.tau[q] = (m >= s.k) ? __uint_as_float((uint32_t)(sel[s.k - 1] >> 32)) : __builtin_inff();
}

// The seeds and tau of a query whose bootstrap rerank was shared by several
// waves: its m exact keys from tpart, sorted.
__global__ __launch_bounds__(kThreads) void k_tau_merge(SearchDev s, const uint64_t* __restrict__ tpart) {
  __shared__ uint64_t selw[kWaves][kMaxK];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWaves + wave;
  if (q >= s.nq) return;   // whole waves
  uint64_t* sel = selw[wave];
  const int mstride = min(kMaxK, 4 * s.k);
  const int m = min(uniform_i32(s.q_n0[q]), mstride);
  for (int i = lane; i < m; i += kWave) sel[i] = tpart[q * mstride + i];
  if (m > 0) wave_sort_sel(sel, m);
  for (int i = lane; i < s.k; i += kWave) {
    SeedEnt e;
    const bool live = i < min(m, s.k);
    const uint64_t v = live ? sel[i] : 0;
    e.dist = live ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
    e.id = live ? (int32_t)(uint32_t)(v & 0xffffffffu) : -1;
    s.seedk[q * s.k + i] = e;
  }
  if (lane == 0) s.tau[q] = (m >= s.k) ? __uint_as_float((uint32_t)(sel[s.k - 1] >> 32)) : __builtin_inff();
}

// The reported value of a result: the exact squared distance (+inf pads), or
// for the inner-product metrics the inner product M_q - d (-inf pads).
__device__ __forceinline__ float out_value(const SearchDev& s, float mq, bool live, float d) {
  if (s.metric != 0) return live ? mq - d : -__builtin_inff();
  return live ? d : __builtin_inff();
}

// ------------------------------------------------------------------ finalize (S7)
// One wave per query (four per block, no block barriers). The top-k starts
// from the bootstrap seeds (tau = their k-th exact distance). The query's live
// candidate entries with bound <= tau are gathered chunk by chunk into a window
// of kFinWin entries, and a window is reranked in rounds: a round takes the
// entries whose bound is at or below a cut read from a sorted sample of the
// window's bounds (about 64 of them; all when at most 64 are left), computes
// their exact distances (groups of 8 lanes: the routine every exact distance
// uses), merges them into the top-k and lowers tau to the k-th exact distance.
// The window keeps only the entries above the cut whose bound is still <= tau.
// Top-k entries are (distance bits << 32 | id) keys: distances are >= 0 and
// ids < 2^31, so the keys order by (distance, id).
constexpr int kFinWin = 512;
constexpr int kFinRoundMax = 128;
constexpr int kFinGather = 4;   // gather batches of 64 entries loaded together
constexpr int kFinSplitWaves = 2048;   // batches below this many queries split each query's rerank
constexpr int kFinSplitMax = 64;       // ... over at most this many waves

__device__ __forceinline__ int fin_lds_words(int k) { return kFinWin + kFinRoundMax + k; }

// With W > 1 (small batches), W waves share a query: wave w takes the
// query's chunks w, w + W, ... and keeps its own tau (the k-th exact distance
// among the seeds and its own reranked candidates, never below the query's
// true k-th distance), so each wave's top-k contains every true top-k member
// of its chunks whose bound holds; it writes that top-k to part and
// k_fin_merge keeps the k best distinct keys of the W lists (the seeds appear
// in all of them).
template <bool WIDE>
__global__ __launch_bounds__(kThreads, WIDE ? 3 : 4) void k_finalize(SearchDev s, int W, uint64_t* __restrict__ part,
                                                          int32_t* __restrict__ pst) {
  using DS = DistShape<WIDE>;
  extern __shared__ uint64_t fin_lds[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  if (s.prof_acc && blockIdx.x == 0 && threadIdx.x == 0) {   // codes estimated by each scan phase
    atomicAdd(&s.prof_acc[0], (unsigned long long)s.off_n0[s.nq]);
    atomicAdd(&s.prof_acc[1], (unsigned long long)(s.off_seg[s.nq] - s.off_n0[s.nq]));
  }
  const int64_t wid = (int64_t)blockIdx.x * kWaves + wave;
  if (wid >= s.nq * W) return;   // whole waves
  const int64_t qi = wid / W;
  const int64_t q = s.q_order ? (int64_t)uniform_i32(s.q_order[qi]) : qi;
  const int wsub = (int)(wid - qi * W);
  const int K = s.k;
  uint64_t* win = fin_lds + (size_t)wave * fin_lds_words(K);
  uint64_t* rnd = win + kFinWin;
  uint64_t* top = rnd + kFinRoundMax;
  // seeds: the valid ones first, in (distance, id) order
  int cnt = 0;
  for (int i0 = 0; i0 < K; i0 += kWave) {
    const int i = i0 + lane;
    // one 8-byte load per seed {dist, id}
    const uint64_t raw = reinterpret_cast<const uint64_t*>(s.seedk)[q * K + min(i, K - 1)];
    const float dist = __uint_as_float((uint32_t)raw);
    const int32_t id = (int32_t)(uint32_t)(raw >> 32);
    const bool v = i < K && id >= 0;
    if (i < K) top[i] = v ? ((uint64_t)__float_as_uint(dist) << 32) | (uint32_t)id : ~0ull;
    cnt += __popcll(__ballot(v));
  }
  wave_lds_sync();
  float tau = uniform_f32(cnt == K ? __uint_as_float((uint32_t)(top[K - 1] >> 32)) : __builtin_inff());
  const int seeds = cnt;
  int reranked = cnt, ncand = 0, nk = 0;
  const float* qv = s.q + q * s.dim;
  const int grp = lane / kLpc, sub = lane % kLpc;
  constexpr int kGroups = kWave / kLpc;

  // rnd[0..n): (distance << 32 | id) of a round. Entries below the current
  // k-th (all of them while fewer than K are known) are compacted to the
  // front; each element of the union of top and those takes its rank: a top
  // element its index plus the entrants below it, an entrant the top elements
  // below it (binary search) plus the entrants below it.
  auto merge = [&](int n) {
    const uint64_t kth = cnt == K ? top[K - 1] : ~0ull;
    int m = 0;
    for (int i0 = 0; i0 < n; i0 += kWave) {
      const int i = i0 + lane;
      const uint64_t x = rnd[min(i, n - 1)];
      const bool in = i < n && x < kth;
      const uint64_t b = __ballot(in);
      if (in) rnd[m + __popcll(b & lanemask_lt())] = x;
      m += __popcll(b);
    }
    if (m == 0) return;
    wave_lds_sync();
    constexpr int kPer = (kMaxK + kFinRoundMax + kWave - 1) / kWave;
    const int mtot = cnt + m;
    uint64_t ev[kPer];
    int er[kPer];
#pragma unroll
    for (int h = 0; h < kPer; ++h) {
      const int e = lane + h * kWave;
      er[h] = K;
      ev[h] = ~0ull;
      if (e < mtot) {
        const bool t = e < cnt;
        ev[h] = t ? top[e] : rnd[e - cnt];
        int r = e;
        if (!t) {
          int lo = 0, hi = cnt;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (top[mid] < ev[h]) lo = mid + 1; else hi = mid;
          }
          r = lo;
        }
        for (int u = 0; u < m; ++u) r += rnd[u] < ev[h];
        er[h] = r;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int h = 0; h < kPer; ++h)
      if (er[h] < K) top[er[h]] = ev[h];
    cnt = min(mtot, K);
    wave_lds_sync();
    if (cnt == K) tau = uniform_f32(fminf(tau, __uint_as_float((uint32_t)(top[K - 1] >> 32))));
  };

  // exact distances of rnd[0..n) ((sortable bound << 32 | position) entries),
  // in passes of 64: entry base + grp + 8 j, j < NC; each entry becomes
  // (distance << 32 | id)
  auto rerank = [&](int n) {
    auto pass = [&](int base, auto nc_tag) {
      constexpr int NC = decltype(nc_tag)::value;
      int32_t pos[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int i = base + grp + j * kGroups;
        pos[j] = (int32_t)(uint32_t)(rnd[min(i, n - 1)] & 0xffffffffu);
        pos[j] = i < n ? pos[j] : -1;
      }
      // the ids travel with the raw vectors (one round trip for both)
      uint32_t id[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) id[j] = id_lo32(s.ids, max(pos[j], 0));
      float d[NC];
      if (s.metric != 0) {
        group_dists<NC, DS::kU, true>(s.raw, pos, s.dim, qv, sub, d, uniform_f32(s.q_m[q]));
      } else {
        group_dists<NC, DS::kU, false>(s.raw, pos, s.dim, qv, sub, d);
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) keep_loaded(id[j]);
      wave_lds_sync();   // every lane has read its entries
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int i = base + grp + j * kGroups;
        const uint64_t v = ((uint64_t)__float_as_uint(d[j]) << 32) | id[j];
        if (sub == 0 && i < n) rnd[i] = v;
      }
      wave_lds_sync();
    };
    for (int base = 0; base < n; base += kGroups * DS::kMaxNC) {
      const int per = (min(n - base, kGroups * DS::kMaxNC) + kGroups - 1) / kGroups;
      if (per <= 1) pass(base, IntC<1>{});
      else if (per <= 2) pass(base, IntC<2>{});
      else if (per <= 4 || DS::kMaxNC == 4) pass(base, IntC<4>{});
      else pass(base, IntC<DS::kMaxNC>{});
    }
  };

  auto process_window = [&]() {
    while (nk > 0) {
      uint32_t cut = 0xFFFFFFFFu;
      if (nk > kWave) {
        uint32_t sv[1] = {(uint32_t)(win[(int)(((int64_t)lane * nk) >> 6)] >> 32)};
        wave_bitonic<1>(sv);
        const int sidx = max(0, kWave * kWave / nk - 1);   // about (sidx + 1) nk / 64 entries <= cut
        cut = (uint32_t)__builtin_amdgcn_readlane((int)sv[0], sidx);
      }
      // entries with bound <= tau: those <= cut to the round (at most
      // kFinRoundMax; the rest stay), the others stay in the window
      const uint32_t tkey = sortable_bits(tau);
      int nr = 0, keep = 0;
      for (int i0 = 0; i0 < nk; i0 += kWave) {
        const int i = i0 + lane;
        const uint64_t x = win[min(i, nk - 1)];
        const uint32_t k = (uint32_t)(x >> 32);
        const bool live = i < nk && k <= tkey;
        const bool to_r = live && k <= cut;
        const uint64_t br = __ballot(to_r);
        const int ar = nr + __popcll(br & lanemask_lt());
        const bool take = to_r && ar < kFinRoundMax;
        const bool stay = live && !take;
        const uint64_t bs = __ballot(stay);
        if (take) rnd[ar] = x;
        if (stay) win[keep + __popcll(bs & lanemask_lt())] = x;
        nr = min(nr + __popcll(br), kFinRoundMax);
        keep += __popcll(bs);
      }
      nk = keep;
      if (nr == 0) break;   // no live entry at or below the cut: none is live at all
      wave_lds_sync();
      reranked += nr;
      rerank(nr);
      merge(nr);
    }
    nk = 0;
  };

  // gather: the wave's chunks (wsub, wsub + W, ...) in groups of 64 (lane j:
  // its chunk j0 + j), entries by a shuffle scan of the chunk counts
  const int nch = uniform_i32(s.q_nch[q]);
  const int nchw = nch > wsub ? (nch - wsub + W - 1) / W : 0;
  const int64_t seg0 = uniform_i64(s.off_seg[q]);
  const int64_t ch0 = uniform_i64(s.off_ch[q]);
  for (int j0 = 0; j0 < nchw; j0 += kWave) {
    const int j = j0 + lane;
    const int jc = wsub + min(j, nchw - 1) * W;   // nchw >= 1 inside the loop
    int64_t base = seg0 + s.chunk_qcode[ch0 + jc];
    int cj = s.seg_count[ch0 + jc];
    base = j < nchw ? base : 0;
    cj = j < nchw ? cj : 0;
    int incl = cj;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int pre = incl - cj;
    const int Tg = __builtin_amdgcn_readlane(incl, kWave - 1);
    ncand += Tg;
    const int64_t base0 = uniform_i64(base);   // chunk j0 (Tg > 0 implies it exists)
    // kFinGather batches of 64 entries at a time: their chunks are located
    // first, then all their segment loads are issued together
    int ccur = 0;
    for (int e0 = 0; e0 < Tg; e0 += kFinGather * kWave) {
      if (nk + kFinGather * kWave > kFinWin) process_window();
      int64_t at[kFinGather];
      bool in[kFinGather];
#pragma unroll
      for (int g = 0; g < kFinGather; ++g) {
        const int eb = e0 + g * kWave, idx = eb + lane;
        int myc = ccur;
        for (int c = ccur + 1; c < kWave; ++c) {   // chunks starting inside this batch
          const int pc = __builtin_amdgcn_readlane(pre, c);
          if (pc > eb + kWave - 1) break;
          if (idx >= pc) myc = c;
        }
        const int64_t mybase = __shfl(base, myc, kWave);
        const int mypre = __shfl(pre, myc, kWave);
        in[g] = idx < Tg;
        at[g] = in[g] ? mybase + (idx - mypre) : base0;
        ccur = __builtin_amdgcn_readlane(myc, kWave - 1);
      }
      Cand cd[kFinGather];
#pragma unroll
      for (int g = 0; g < kFinGather; ++g) cd[g] = s.seg[at[g]];
#pragma unroll
      for (int g = 0; g < kFinGather; ++g) {
        const bool keep = in[g] && cd[g].pos >= 0 && cd[g].lb <= tau;
        const uint64_t b = __ballot(keep);
        if (keep)
          win[nk + __popcll(b & lanemask_lt())] = ((uint64_t)sortable_bits(cd[g].lb) << 32) | (uint32_t)cd[g].pos;
        nk += __popcll(b);
      }
    }
  }
  process_window();
  if (W == 1) {
    const float mq = s.metric != 0 ? s.q_m[q] : 0.f;
    for (int i = lane; i < K; i += kWave) {
      const uint64_t v = top[i];
      const bool live = i < cnt;
      s.out_ids[q * K + i] = live ? (int64_t)(uint32_t)(v & 0xffffffffu) : (int64_t)-1;
      s.out_d[q * K + i] = out_value(s, mq, live, __uint_as_float((uint32_t)(v >> 32)));
    }
    if (lane == 0) {
      s.q_rerank[q] = reranked - seeds;   // the seeds' distances were computed by the bootstrap rerank
      s.q_cand[q] = ncand;
    }
  } else {
    const int64_t slot = q * W + wsub;   // the merge reads query q's W partial results
    for (int i = lane; i < K; i += kWave) part[slot * K + i] = i < cnt ? top[i] : ~0ull;
    if (lane == 0) {
      pst[slot * 2] = reranked - seeds;
      pst[slot * 2 + 1] = ncand;
    }
  }
}

// Merge of a query's W partial top-k lists (W K <= kFinMergeCap keys): the k best
// distinct (distance, id) keys, and the statistics: every wave's own reranks
// (the seeds were reranked by the bootstrap) and every wave's candidates. fin_merge_out takes the
// keys sorted in sel[0..n); one wave.
__device__ __forceinline__ void fin_merge_out(const SearchDev& s, int64_t q, int W, const uint64_t* sel, int n,
                                              const int32_t* __restrict__ pst) {
  const int lane = lane_id();
  const int K = s.k;
  const float mq = s.metric != 0 ? s.q_m[q] : 0.f;
  int out = 0;
  for (int i0 = 0; i0 < n && out < K; i0 += kWave) {
    const int i = i0 + lane;
    const uint64_t x = sel[min(i, n - 1)], prev = sel[max(min(i, n - 1) - 1, 0)];
    const bool keep = i < n && x != ~0ull && (i == 0 || x != prev);
    const uint64_t b = __ballot(keep);
    const int at = out + __popcll(b & lanemask_lt());
    if (keep && at < K) {
      s.out_ids[q * K + at] = (int64_t)(uint32_t)(x & 0xffffffffu);
      s.out_d[q * K + at] = out_value(s, mq, true, __uint_as_float((uint32_t)(x >> 32)));
    }
    out += __popcll(b);
  }
  for (int i = min(out, K) + lane; i < K; i += kWave) {
    s.out_ids[q * K + i] = -1;
    s.out_d[q * K + i] = out_value(s, mq, false, 0.f);
  }
  int rer = 0, cand = 0;
  for (int w = lane; w < W; w += kWave) {
    rer += pst[(q * W + w) * 2];
    cand += pst[(q * W + w) * 2 + 1];
  }
  rer = wave_sum_i(rer);
  cand = wave_sum_i(cand);
  if (lane == 0) {
    s.q_rerank[q] = rer;
    s.q_cand[q] = cand;
  }
}

// At most kMergeWaveMax keys per query: one wave per query, sorted in
// registers.
constexpr int kMergeWaveMax = 256;
__global__ __launch_bounds__(kThreads) void k_fin_merge(SearchDev s, int W, const uint64_t* __restrict__ part,
                                                        const int32_t* __restrict__ pst) {
  __shared__ uint64_t selw[kWaves][kMergeWaveMax];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWaves + wave;
  if (q >= s.nq) return;   // whole waves
  const int n = W * s.k;
  uint64_t* sel = selw[wave];
  for (int i = lane; i < n; i += kWave) sel[i] = part[q * n + i];
  wave_sort_sel(sel, n);
  fin_merge_out(s, q, W, sel, n, pst);
}

// More keys (up to kFinMergeCap): one block per query sorts them in LDS.
constexpr int kMergeThreads = 512;
__global__ __launch_bounds__(kMergeThreads) void k_fin_merge_block(SearchDev s, int W,
                                                                   const uint64_t* __restrict__ part,
                                                                   const int32_t* __restrict__ pst) {
  __shared__ uint64_t sel[kFinMergeCap];
  const int64_t q = blockIdx.x;
  const int n = W * s.k;
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += kMergeThreads) sel[i] = i < n ? part[q * n + i] : ~0ull;
  __syncthreads();
  bitonic_sort_u64(sel, n2);
  if (threadIdx.x < kWave) fin_merge_out(s, q, W, sel, n, pst);
}

// ------------------------------------------------------------------ debug
__global__ void k_debug_pack(const uint8_t* __restrict__ qu, int dp, int W, int npl, int qoff, float b, float vl,
                             float delta, float pt, PairRec* rec, uint64_t* planes, int8_t* qu8, float* pair_pt,
                             int32_t list, double rd, double ird) {
  // one wave
  const int lane = lane_id();
  if (lane == 0 && pair_pt) pair_pt[0] = pt;
  int sq = 0;
  for (int t = 0; t < W; ++t) {
    const int i = t * kWave + lane;
    const int v = qu[i];
    sq += v;
    if (qu8) qu8[i] = (int8_t)(v - qoff);
    for (int j = 0; j < npl; ++j) {
      const uint64_t w = __ballot((v >> j) & 1);
      if (lane == 0) planes[j * W + t] = w;
    }
  }
  sq = wave_sum_i(sq);
  if (lane == 0) {
    PairRec r;
    pair_coeffs((double)vl, (double)delta, sq, rd, ird, r);
    r.b = b;
    r.vl = vl;
    r.delta = delta;
    r.sq = sq;
    r.list = list;
    *rec = r;
  }
}



}  // namespace

template <int W>
void launch_prep_q(const SearchDev& s, int64_t unit_blocks, int64_t prep_blocks, hipStream_t st) {
  const dim3 grid((unsigned)(unit_blocks + prep_blocks));
  if (unit_blocks > 0) {
    if (s.qu8)
      hipLaunchKernelGGL((k_prep_units<W, true>), grid, dim3(kThreads), 0, st, s, unit_blocks);
    else
      hipLaunchKernelGGL((k_prep_units<W, false>), grid, dim3(kThreads), 0, st, s, unit_blocks);
  } else {
    if (s.qu8)
      hipLaunchKernelGGL((k_prep_q<W, true>), grid, dim3(kThreads), 0, st, s);
    else
      hipLaunchKernelGGL((k_prep_q<W, false>), grid, dim3(kThreads), 0, st, s);
  }
}

// The per-pair quantisation, and with `units` also the unit descriptors
// (which need the plan and the query offsets): for W <= 4 in one launch.
hipError_t launch_prep(const SearchDev& s, bool units, hipStream_t st) {
  const int64_t npairs = s.nq * s.nprobe;
  if (npairs <= 0) return hipSuccess;
  auto grid = [&](int ppw) { return dim3((unsigned)((npairs + ppw * kWaves - 1) / (ppw * kWaves))); };
  const int64_t qblocks = (npairs + 4 * kWaves - 1) / (4 * kWaves);
  const int64_t nrb = (s.nprobe + kWave - 1) / kWave;
  const int64_t ublocks = units ? (s.nq * nrb + kWaves - 1) / kWaves : 0;
  if (s.W <= 0 || s.W > 64) return hipErrorInvalidValue;
  if (s.npl == 8 && s.W <= 4) {   // the quarter-wave form holds 4 W plane words per row: B_q <= 4 only
    hipLaunchKernelGGL((k_prep_reg<4, 2, 8>), grid(2), dim3(kThreads), 0, st, s);
    if (units) hipLaunchKernelGGL(k_units, dim3((unsigned)ublocks), dim3(kThreads), 0, st, s);
    return hipGetLastError();
  }
  // wide rows: one pair per wave (two up to W = 8), the register bound WS exact
  // for D = 768 and 960, and B_q = 4 planes compile-time
  const bool p4 = s.npl == 4;
#define RBQ_PREP(WS_, PPW_)                                                                          \
  do {                                                                                              \
    if (p4)                                                                                         \
      hipLaunchKernelGGL((k_prep_reg<WS_, PPW_, 4>), grid(PPW_), dim3(kThreads), 0, st, s);         \
    else                                                                                            \
      hipLaunchKernelGGL((k_prep_reg<WS_, PPW_, 0>), grid(PPW_), dim3(kThreads), 0, st, s);         \
  } while (0)
  switch (s.W) {
    case 1: launch_prep_q<1>(s, ublocks, qblocks, st); return hipGetLastError();
    case 2: launch_prep_q<2>(s, ublocks, qblocks, st); return hipGetLastError();
    case 3: launch_prep_q<3>(s, ublocks, qblocks, st); return hipGetLastError();
    case 4: launch_prep_q<4>(s, ublocks, qblocks, st); return hipGetLastError();
    case 12: RBQ_PREP(12, 1); break;
    case 15: RBQ_PREP(15, 1); break;
    default:
      if (s.W <= 8) {
        RBQ_PREP(8, 2);
      } else if (s.W <= 16) {
        RBQ_PREP(16, 1);
      } else if (s.W <= 32) {
        RBQ_PREP(32, 1);
      } else {
        RBQ_PREP(64, 1);
      }
  }
#undef RBQ_PREP
  if (units) hipLaunchKernelGGL(k_units, dim3((unsigned)ublocks), dim3(kThreads), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_plan(const SearchDev& s, hipStream_t st) {
  if (s.nq <= 0) return hipSuccess;
  if (s.nprobe > kPlanWaveMax) {
    static bool attr_done = false;
    if (!attr_done) {
      (void)hipFuncSetAttribute((const void*)k_plan_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kPlanLdsBytes);
      attr_done = true;
    }
    const size_t shm = 2 * ((size_t)plan_pad(s.nprobe) + 1) * sizeof(int32_t);
    hipLaunchKernelGGL(k_plan_block, dim3((unsigned)s.nq), dim3(kPlanThreads), shm, st, s);
  } else {
    const dim3 gq((unsigned)((s.nq + kWaves - 1) / kWaves));
    hipLaunchKernelGGL(k_plan, gq, dim3(kThreads), 0, st, s);
  }
  const dim3 gb((unsigned)((s.nq + kOffQ - 1) / kOffQ));
  hipLaunchKernelGGL(k_offsets_sum, gb, dim3(kOffThreads), 0, st, s);
  hipLaunchKernelGGL(k_offsets_scan, gb, dim3(kOffThreads), 0, st, s);
  return hipGetLastError();
}


int tau_split(int fin_w, int k) {
  const int m = std::min(kMaxK, 4 * k);
  return std::max(1, std::min(fin_w, m / 32));   // at least 32 entries per wave
}

hipError_t launch_tau_split(const SearchDev& s, int W, uint64_t* tpart, hipStream_t st) {
  if (s.nq <= 0) return hipSuccess;
  if (W < 1 || (W > 1 && !tpart)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((s.nq * W + kWaves - 1) / kWaves));
  if (dist_wide(s.dim))
    hipLaunchKernelGGL(k_tau<true>, grid, dim3(kThreads), 0, st, s, W, tpart);
  else
    hipLaunchKernelGGL(k_tau<false>, grid, dim3(kThreads), 0, st, s, W, tpart);
  if (W > 1)
    hipLaunchKernelGGL(k_tau_merge, dim3((unsigned)((s.nq + kWaves - 1) / kWaves)), dim3(kThreads), 0, st, s,
                       tpart);
  return hipGetLastError();
}

hipError_t launch_tau(const SearchDev& s, hipStream_t st) { return launch_tau_split(s, 1, nullptr, st); }

int finalize_split(int64_t nq, int k) {
  if (nq <= 0 || nq >= kFinSplitWaves) return 1;
  int w = (int)((kFinSplitWaves + nq - 1) / nq);
  w = std::min(w, kFinSplitMax);
  w = std::min(w, kFinMergeCap / std::max(k, 1));
  return std::max(w, 1);
}

namespace {
constexpr int kOrderBins = 64;

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {   // a kernel, not a memset: capturable
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__device__ __forceinline__ int order_bin(int npq, int nprobe) {
  return min(kOrderBins - 1, (int)((int64_t)min(max(npq, 1), nprobe) * kOrderBins / (nprobe + 1)));
}

__global__ void k_order_hist(const int32_t* __restrict__ npq, int64_t nq, int nprobe, int32_t* hist) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) atomicAdd(&hist[order_bin(npq[q], nprobe)], 1);
}

// One wave: hist[b] -> the first slot of bin b, bins in descending order.
__global__ void k_order_scan(int32_t* hist) {
  const int lane = threadIdx.x;   // kOrderBins == kWave
  const int b = kOrderBins - 1 - lane;   // lane 0 holds the heaviest bin
  const int c = hist[b];
  int inc = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  hist[kOrderBins + b] = inc - c;
}

__global__ void k_order_scatter(const int32_t* __restrict__ npq, int64_t nq, int nprobe, int32_t* hist,
                                int32_t* __restrict__ order) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) order[atomicAdd(&hist[kOrderBins + order_bin(npq[q], nprobe)], 1)] = (int32_t)q;
}
}  // namespace

hipError_t launch_query_order(const int32_t* nprobe_q, int64_t nq, int nprobe, int32_t* hist, int32_t* order,
                              hipStream_t st) {
  static_assert(kOrderBins == kWave, "one lane per bin");
  if (nq <= 0) return hipSuccess;
  const unsigned g = (unsigned)((nq + 255) / 256);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(2 * kOrderBins), 0, st, hist, (int64_t)(2 * kOrderBins));
  hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, st, nprobe_q, nq, nprobe, hist);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kWave), 0, st, hist);
  hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, st, nprobe_q, nq, nprobe, hist, order);
  return hipGetLastError();
}

hipError_t launch_finalize_split(const SearchDev& s, int W, uint64_t* part, int32_t* pst, hipStream_t st) {
  if (s.nq <= 0) return hipSuccess;
  if (W < 1 || (W > 1 && (!part || !pst || W * s.k > kFinMergeCap))) return hipErrorInvalidValue;
  const size_t shm = (size_t)kWaves * (kFinWin + kFinRoundMax + s.k) * sizeof(uint64_t);
  const dim3 grid((unsigned)((s.nq * W + kWaves - 1) / kWaves));
  if (dist_wide(s.dim))
    hipLaunchKernelGGL(k_finalize<true>, grid, dim3(kThreads), shm, st, s, W, part, pst);
  else
    hipLaunchKernelGGL(k_finalize<false>, grid, dim3(kThreads), shm, st, s, W, part, pst);
  if (W > 1 && W * s.k > kMergeWaveMax)
    hipLaunchKernelGGL(k_fin_merge_block, dim3((unsigned)s.nq), dim3(kMergeThreads), 0, st, s, W, part, pst);
  else if (W > 1)
    hipLaunchKernelGGL(k_fin_merge, dim3((unsigned)((s.nq + kWaves - 1) / kWaves)), dim3(kThreads), 0, st, s, W,
                       part, pst);
  return hipGetLastError();
}

hipError_t launch_finalize(const SearchDev& s, hipStream_t st) {
  return launch_finalize_split(s, 1, nullptr, nullptr, st);
}

hipError_t launch_debug_pack(const uint8_t* qu, int dp, int W, int npl, int qoff, float b, float vl, float delta,
                             float pt, PairRec* rec, uint64_t* planes, int8_t* qu8, float* pair_pt, int32_t list,
                             hipStream_t st) {
  const double rd = std::sqrt((double)dp);
  hipLaunchKernelGGL(k_debug_pack, dim3(1), dim3(kWave), 0, st, qu, dp, W, npl, qoff, b, vl, delta, pt, rec,
                     planes, qu8, pair_pt, list, rd, 1.0 / rd);
  return hipGetLastError();
}

hipError_t launch_debug_scan(const SearchDev& s, const PairRec* rec, const uint64_t* planes,
                             const int8_t* qu8, int32_t list, int kernel, int32_t* ip,
                             int32_t* pc, float* est, float* dist, float* lb, hipStream_t st) {
  int n = 0;
  {
    int32_t off[2];
    hipError_t e = hipMemcpy(off, s.list_off + list, sizeof(off), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    n = off[1] - off[0];
  }
  if (n == 0) return hipSuccess;
  if (kernel == 2 || kernel == 3)   // int8 or FP8 x FP4 (s.mfma_f4)
    return launch_debug_mfma(s, rec, qu8, list, (n + s.chunk - 1) / s.chunk, ip, pc, est, dist, lb, st);
  // the production popcount scan, phase 2, over the unit table the caller
  // prepared in s.units1 (s.off_p1[s.nq] units of pair 0)
  (void)planes;
  const int units = (n + s.chunk - 1) / s.chunk;   // one wave each
  const int grid = std::max(1, (units + 3) / 4);
  return launch_scan_popcnt(s, 2, grid, st);
}

}  // namespace rbq

namespace rbq {
namespace {
__global__ void k_pairs_to_scal(const PairRec* __restrict__ pairs, int64_t n, float* __restrict__ scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PairRec r = pairs[i];
  scal[i * 4 + 0] = r.b;
  scal[i * 4 + 1] = r.vl;
  scal[i * 4 + 2] = r.delta;
  scal[i * 4 + 3] = (float)r.sq;
}
}  // namespace
hipError_t launch_pairs_to_scal(const SearchDev& s, float* scal, hipStream_t st) {
  const int64_t n = s.nq * s.nprobe;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pairs_to_scal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.pairs, n, scal);
  return hipGetLastError();
}
}  // namespace rbq


