// Device helpers shared by the popcount scan and the parity-export scan:
// bit-plane inner products, the estimator epilogue and work-unit decoding.
#ifndef RBQ_SCAN_CODE_HPP
#define RBQ_SCAN_CODE_HPP

#include "rbq_internal.hpp"

namespace rbq {
namespace {

// ------------------------------------------------------------------ scan arithmetic (S4 + S6)
// Integer <x_b, q_u> = sum_j 2^j popcount(x_b AND plane_j) and popcount(x_b)
// for the code at position p. WS > 0: planes held in registers (W == WS).
template <int WS>
struct Planes {
  uint64_t w[4][WS];
  __device__ __forceinline__ void load(const uint64_t* src, int) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int t = 0; t < WS; ++t) w[j][t] = src[j * WS + t];
  }
  __device__ __forceinline__ uint64_t get(int j, int t) const { return w[j][t]; }
};
template <>
struct Planes<0> {
  const uint64_t* p;   // LDS copy, [4][W]
  int W;
  __device__ __forceinline__ uint64_t get(int j, int t) const { return p[j * W + t]; }
};

template <int WS>
__device__ __forceinline__ void code_ip(const uint64_t* __restrict__ codes, int64_t p, int W,
                                        const Planes<WS>& pl, int& ip, int& pc) {
  const int Wn = WS > 0 ? WS : W;
  int s0 = 0, s1 = 0, s2 = 0, s3 = 0, c = 0;
#pragma unroll
  for (int t = 0; t < Wn; ++t) {
    const uint64_t x = codes[code_word_index(p, t, W)];
    c += __popcll(x);
    s0 += __popcll(x & pl.get(0, t));
    s1 += __popcll(x & pl.get(1, t));
    s2 += __popcll(x & pl.get(2, t));
    s3 += __popcll(x & pl.get(3, t));
  }
  ip = s0 + 2 * s1 + 4 * s2 + 8 * s3;
  pc = c;
}

// est = <x_bar, q_bar>/<o_bar,o> (Theorem 3.2); Eq. (2) gives the distance;
// the lower bound plugs est + half-width into Eq. (2).
__device__ __forceinline__ void estimate(const PairRec& r, float2 f, int ip, int pc, float hwk,
                                         float& est, float& dist, float& lb) {
  const float a = f.x, ipo = f.y;
  const float xq = fmaf(r.k1, (float)ip, fmaf(r.k2, (float)pc, r.k0));
  const float inv = __builtin_amdgcn_rcpf(ipo);
  est = xq * inv;
  const float ab2 = 2.f * a * r.b;
  const float base = fmaf(a, a, r.b * r.b);
  dist = fmaf(-ab2, est, base);
  const float hw = sqrtf(fmaxf(fmaf(-ipo, ipo, 1.f), 0.f)) * inv * hwk;
  lb = fmaf(-ab2, hw, dist);
}

struct Unit {
  int64_t q;
  int r, c;
  int64_t g;            // pair index
  int64_t start, end;   // code positions
  int64_t codeoff;      // query code-space offset of the chunk start
  int64_t count_slot;   // seg_count index
};

__device__ __forceinline__ Unit load_unit(const SearchDev& s, uint64_t e) {
  Unit w;
  w.q = uniform_i64((int64_t)(e >> 40));
  w.r = uniform_i32((int)((e >> 24) & 0xFFFFu));
  w.c = uniform_i32((int)(e & 0xFFFFFFu));
  w.g = w.q * s.nprobe + w.r;
  const int list = uniform_i32(s.pairs[w.g].list);
  const int32_t* choff = s.pair_choff + w.q * (s.nprobe + 1);
  const int32_t* codeoff = s.pair_codeoff + w.q * (s.nprobe + 1);
  const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
  w.start = lbeg + (int64_t)w.c * s.chunk;
  w.end = lend < w.start + s.chunk ? lend : w.start + s.chunk;
  w.codeoff = uniform_i64((int64_t)codeoff[w.r] + (int64_t)w.c * s.chunk);
  w.count_slot = uniform_i64(s.off_ch[w.q] + choff[w.r] + w.c);
  return w;
}

}  // namespace
}  // namespace rbq

#endif  // RBQ_SCAN_CODE_HPP
