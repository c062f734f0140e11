// Persistent bit-plane popcount scan (S4 + S6) with the rerank filter of
// phase 1: every probed code's integer <x_b, q_u> and popcount, the unbiased
// estimate, its distance lower bound, and the candidate segment it lands in.
#include "rbq_internal.hpp"
#include "scan_code.hpp"

namespace rbq {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

// Scan of one chunk: UN blocks of 64 codes per iteration, one code per lane
// per block, all loads of an iteration issued before the arithmetic.
template <int WS, int UN>
__device__ __forceinline__ int scan_chunk(const SearchDev& s, int phase, const Unit& w,
                                          const PairRec& rec, const Planes<WS>& pl, float tau,
                                          float hwk) {
  const int lane = lane_id();
  const int64_t seg_base = s.off_seg[w.q] + w.codeoff;
  const int64_t p0base = phase == 0 ? s.off_n0[w.q] + w.codeoff : 0;
  int count = 0;
  for (int64_t b0 = w.start; b0 < w.end; b0 += 64 * UN) {
    int64_t p[UN];
    bool valid[UN];
    float2 f[UN];
    int ip[UN], pc[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      valid[u] = b0 + 64 * u + lane < w.end;
      p[u] = valid[u] ? b0 + 64 * u + lane : w.start;   // masked lanes read an in-bounds code
      f[u] = s.fac[p[u]];
    }
    if constexpr (WS > 0) {
      uint64_t x[UN][WS];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int t = 0; t < WS; ++t) x[u][t] = s.codes[code_word_index(p[u], t, WS)];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        int s0 = 0, s1 = 0, s2 = 0, s3 = 0, c = 0;
#pragma unroll
        for (int t = 0; t < WS; ++t) {
          c += __popcll(x[u][t]);
          s0 += __popcll(x[u][t] & pl.get(0, t));
          s1 += __popcll(x[u][t] & pl.get(1, t));
          s2 += __popcll(x[u][t] & pl.get(2, t));
          s3 += __popcll(x[u][t] & pl.get(3, t));
        }
        ip[u] = s0 + 2 * s1 + 4 * s2 + 8 * s3;
        pc[u] = c;
      }
    } else {
#pragma unroll
      for (int u = 0; u < UN; ++u) code_ip<WS>(s.codes, p[u], s.W, pl, ip[u], pc[u]);
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      float est, dist, lb;
      estimate(rec, f[u], ip[u], pc[u], hwk, est, dist, lb);
      lb = valid[u] ? lb : __builtin_inff();
      const int64_t off = p[u] - w.start;
      if (phase == 0) {
        if (valid[u]) {
          Cand cd;
          cd.pos = (int32_t)p[u];
          cd.lb = lb;
          s.seg[seg_base + off] = cd;
          EstEnt e;
          e.dist = dist;
          e.slot = (int32_t)(w.codeoff + off);
          s.p0buf[p0base + off] = e;
        }
      } else {
        const bool pass = valid[u] && (lb <= tau);
        const uint64_t m = __ballot(pass);
        if (pass) {
          Cand cd;
          cd.pos = (int32_t)p[u];
          cd.lb = lb;
          s.seg[seg_base + count + __popcll(m & lanemask_lt())] = cd;
        }
        count += __popcll(m);
      }
    }
  }
  return phase == 0 ? (int)(w.end - w.start) : count;
}

// Persistent scan: wave i of the grid takes units i, i + nwaves, ... of the
// phase's unit table (units are chunks of at most `chunk` codes, so a static
// round-robin balances them; no atomics and no per-unit searches).
template <int WS, int UN>
__global__ __launch_bounds__(kThreads) void k_scan_popcnt(SearchDev s, int phase) {
  __shared__ uint64_t lds_planes[kWaves][4 * (kMaxCodeBits / 64)];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t total = uniform_i64((phase == 0 ? s.off_p0 : s.off_p1)[s.nq]);
  const uint64_t* tab = phase == 0 ? s.units0 : s.units1;
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  for (int64_t u = uniform_i64((int64_t)blockIdx.x * kWaves + wave); u < total; u += nw) {
    const Unit w = load_unit(s, tab[u]);
    const PairRec rec = s.pairs[w.g];
    const uint64_t* src = s.planes + w.g * 4 * s.W;
    Planes<WS> pl;
    if constexpr (WS > 0) {
      pl.load(src, s.W);
    } else {
      uint64_t* dst = lds_planes[wave];
      for (int i = lane; i < 4 * s.W; i += kWave) dst[i] = src[i];
      pl.p = dst;
      pl.W = s.W;
    }
    const float tau = phase == 0 ? __builtin_inff() : uniform_f32(s.tau[w.q]);
    const int count = scan_chunk<WS, UN>(s, phase, w, rec, pl, tau, hwk);
    if (lane == 0) s.seg_count[w.count_slot] = count;
  }
}

template <int WS, int UN>
void launch_scan_ws(const SearchDev& s, int phase, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_scan_popcnt<WS, UN>), dim3(grid), dim3(kThreads), 0, st, s, phase);
}

}  // namespace

hipError_t launch_scan_popcnt(const SearchDev& s, int phase, int grid, hipStream_t st) {
  switch (s.W) {
    case 1: launch_scan_ws<1, 4>(s, phase, grid, st); break;
    case 2: launch_scan_ws<2, 4>(s, phase, grid, st); break;
    case 3: launch_scan_ws<3, 4>(s, phase, grid, st); break;
    case 4: launch_scan_ws<4, 2>(s, phase, grid, st); break;
    default: launch_scan_ws<0, 2>(s, phase, grid, st); break;
  }
  return hipGetLastError();
}

}  // namespace rbq
