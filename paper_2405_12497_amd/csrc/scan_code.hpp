// Device helpers shared by the popcount scan and the parity-export scan:
// bit-plane inner products, the estimator epilogue and work-unit decoding.
#ifndef RBQ_SCAN_CODE_HPP
#define RBQ_SCAN_CODE_HPP

#include <type_traits>

#include "rbq_internal.hpp"

namespace rbq {
namespace {

// ------------------------------------------------------------------ scan arithmetic (S4 + S6)
// Integer <x_b, q_u> = sum_j 2^j popcount(x_b AND plane_j) and popcount(x_b)
// (Sec. 3.3.2), with NPL bit planes: 4 for B_q <= 4 (the planes j >= B_q are
// zero), 8 for B_q = 5..8.
// Planes<WS, NPL>: the pair's planes in registers (1 <= WS <= 4 words, W == WS).
template <int WS, int NPL>
struct Planes {
  uint64_t w[NPL][WS];
  __device__ __forceinline__ uint64_t get(int j, int t) const { return w[j][t]; }
};
// PlanesLds<WS>: the planes in LDS ([NPL][W]), W == WS > 4 known at compile
// time, or runtime W when WS == 0.
template <int WS>
struct PlanesLds {
  const uint64_t* p;
  int Wr;
  __device__ __forceinline__ uint64_t get(int j, int t) const { return p[j * (WS > 0 ? WS : Wr) + t]; }
};
template <int WS, int NPL>
using PlanesFor = typename std::conditional<(WS >= 1 && WS <= 4), Planes<WS, NPL>, PlanesLds<WS>>::type;

// Word 0 of the code at list-order position p; word t is row[64 * t]
// (interleaved layout: word w of 64 consecutive codes is one 512-byte row).
// Word offsets are 32-bit: the index keeps npad * W below 2^32.
__device__ __forceinline__ const uint64_t* code_row(const uint64_t* __restrict__ codes, int32_t p, int W) {
  return codes + ((uint32_t)(p >> 6) * (uint32_t)(W * 64) + (uint32_t)(p & 63));
}

template <int WS, int NPL, typename PL>
__device__ __forceinline__ void code_ip(const uint64_t* __restrict__ row, int W, const PL& pl, int& ip,
                                        int& pc) {
  const int Wn = WS > 0 ? WS : W;
  int sj[NPL];
#pragma unroll
  for (int j = 0; j < NPL; ++j) sj[j] = 0;
  int c = 0;
#pragma unroll
  for (int t = 0; t < Wn; ++t) {
    const uint64_t x = row[64 * t];
    c += __popcll(x);
#pragma unroll
    for (int j = 0; j < NPL; ++j) sj[j] += __popcll(x & pl.get(j, t));
  }
  int v = 0;
#pragma unroll
  for (int j = 0; j < NPL; ++j) v += sj[j] << j;
  ip = v;
  pc = c;
}

// est = <x_bar, q_bar>/<o_bar,o> (Theorem 3.2); Eq. (2) gives the distance;
// the lower bound plugs est + half-width into Eq. (2).
// Scan factors of a code, precomputed in FP64 from (a, <o_bar,o>) when the
// index is built or loaded: G = a / <o_bar,o> and H = a sqrt(1 - <o_bar,o>^2)
// / <o_bar,o>, so that a^2 = G^2 - H^2. With the pair's b and
// x = <x_bar, q_bar> (Sec. 3.3.2 decomposition):
//   dist = a^2 + b^2 - 2 b G x       (Eq. (2) with est = x / <o_bar,o>, Theorem 3.2)
//   lb   = dist - 2 b (eps0 / sqrt(D - 1)) H   (2ab times the half-width of Theorem 3.2)
// The per-pair constants are b^2, -2b and -2b eps0 / sqrt(D - 1). Every scan
// uses this form, so all of them give identical bits.
// Inner product (RBQ_METRIC_IP / COSINE): the searched "distance" is
// M_q - <o_r, q_r> with <o_r, q_r> = a b <o, q> + <o_r - c, c> + <q_r, c>
// (the conclusion's identity), so
//   dist = (M_q - <q_r, c>) - <o_r - c, c> - b G x,   lb = dist - b (eps0 / sqrt(D - 1)) H:
// per-pair constants M_q - <q_r, c> (from the quantiser), -b, -b eps0 / sqrt(D - 1),
// and the per-code term -<o_r - c, c> in place of a^2.
// Per-pair constants of the scan's estimator (Theorem 3.2 through the scan
// factors G, H): with x the estimate of <o_bar, q> from (ip, pc) (k1 ip +
// k2 pc + k0) and coef its coefficient in the distance, y = coef x =
// a1 ip + a2 pc + a0 (coef folded into k1, k2, k0), the distance estimate is
// G y + ct + pt and its lower bound adds coefh H. The bound test compares the
// bound without the pair term pt against tau - pt.
struct PairTerms {
  float a1, a2, a0;   // coef k1, coef k2, coef k0
  float pt, coefh;    // pair term, coefficient of H
};
__device__ __forceinline__ PairTerms pair_terms_from(const PairRec& r, float coef, float hwk, float pt) {
  PairTerms t;
  t.a1 = coef * r.k1;
  t.a2 = coef * r.k2;
  t.a0 = coef * r.k0;
  t.pt = pt;
  t.coefh = coef * hwk;
  return t;
}
// L2: -2 ||q_r - c|| <o_bar, q> and pair term ||q_r - c||^2.
__device__ __forceinline__ PairTerms pair_terms(const PairRec& r, float hwk) {
  return pair_terms_from(r, -2.f * r.b, hwk, r.b * r.b);
}
// inner product: -||q_r - c|| <o_bar, q> and pair term M_q - <q_r, c>.
__device__ __forceinline__ PairTerms pair_terms_ip(const PairRec& r, float hwk, float pair_term) {
  return pair_terms_from(r, -r.b, hwk, pair_term);
}
// The per-code term: a^2 = G^2 - H^2 (L2), or -<o_r - c, c> (inner product).
__device__ __forceinline__ float code_term_l2(float2 sf) { return fmaf(sf.x, sf.x, -sf.y * sf.y); }
// y from the integer inner product and popcount.
__device__ __forceinline__ float est_y(const PairTerms& t, int ip, int pc) {
  return fmaf(t.a1, (float)ip, fmaf(t.a2, (float)pc, t.a0));
}
// Distance estimate and lower bound, both without the pair term pt.
__device__ __forceinline__ void est_dl(const PairTerms& t, float2 sf, float ct, float y, float& d0, float& l0) {
  d0 = fmaf(sf.x, y, ct);
  l0 = fmaf(t.coefh, sf.y, d0);
}
// Distance estimate and lower bound (the bootstrap and parity exports).
__device__ __forceinline__ void estimate(const PairTerms& t, float2 sf, float ct, int ip, int pc, float& dist,
                                         float& lb) {
  float d0, l0;
  est_dl(t, sf, ct, est_y(t, ip, pc), d0, l0);
  dist = d0 + t.pt;
  lb = l0 + t.pt;
}
// The estimate itself, from the stored (a, <o_bar,o>) (the parity exports).
__device__ __forceinline__ float estimate_est(const PairRec& r, float ipo, int ip, int pc) {
  const float xq = fmaf(r.k1, (float)ip, fmaf(r.k2, (float)pc, r.k0));
  return xq / ipo;
}

// A unit descriptor read with a wave-uniform address, made wave-uniform.
__device__ __forceinline__ UnitDesc load_unit(const UnitDesc* __restrict__ tab, int64_t u) {
  const UnitDesc d = tab[u];
  UnitDesc w;
  w.start = uniform_i64(d.start);
  w.g = uniform_i64(d.g);
  w.seg = uniform_i64(d.seg);
  w.qcode = uniform_i64(d.qcode);
  w.p0slot = uniform_i64(d.p0slot);
  w.count_slot = uniform_i64(d.count_slot);
  w.len = uniform_i32(d.len);
  w.q = uniform_i32(d.q);
  w.pad = 0;
  return w;
}

}  // namespace
}  // namespace rbq

#endif  // RBQ_SCAN_CODE_HPP
