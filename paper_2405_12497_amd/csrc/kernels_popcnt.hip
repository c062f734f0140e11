// Persistent bit-plane popcount scan (S4 + S6) with the rerank filter of
// phase 1: every probed code's integer <x_b, q_u> and popcount, the unbiased
// estimate, its distance lower bound, and the candidate segment it lands in.
#include "rbq_internal.hpp"
#include "scan_code.hpp"

namespace rbq {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

// Codes [b0, b0 + 64 UN) of a unit, one per lane per 64-code block: all
// loads issued before the arithmetic, then the estimate and lower bound of
// each code. PHASE 0 (bootstrap) keeps every code: its candidate entry and
// its estimated distance go to the unit's segment and bootstrap slots.
// PHASE 1 keeps the codes with lb <= tau, compacted into the segment.
// PHASE 2 (parity export) writes every code's ip, popcount, estimate,
// distance and bound to the debug arrays at its offset from s.dbg_base.
template <int WS, int UN, int PHASE, int NPL, typename PL>
__device__ __forceinline__ void scan_step(const SearchDev& s, const UnitDesc& w, int32_t b0, int32_t wend,
                                          const PairRec& rec, const PairTerms& pt, const PL& pl, float tau, int& count) {
  const int lane = lane_id();
  const int32_t start = (int32_t)w.start;
  const int W = WS > 0 ? WS : s.W;
  int32_t p[UN];
  bool valid[UN];
  float2 f[UN];
  float ct[UN];
  int ip[UN], pc[UN];
  const uint64_t* row[UN];
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    valid[u] = b0 + 64 * u + lane < wend;
    p[u] = valid[u] ? b0 + 64 * u + lane : start;   // masked lanes read an in-bounds code
    f[u] = s.sfac[p[u]];
    row[u] = code_row(s.codes, p[u], W);
  }
  if (s.metric != 0) {   // inner product: the per-code term -<o_r - c, c>
#pragma unroll
    for (int u = 0; u < UN; ++u) ct[u] = -s.fip[p[u]];
  } else {
#pragma unroll
    for (int u = 0; u < UN; ++u) ct[u] = code_term_l2(f[u]);
  }
  if constexpr (WS > 0) {
    uint64_t x[UN][WS];
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int t = 0; t < WS; ++t) x[u][t] = row[u][64 * t];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      int sj[NPL];
#pragma unroll
      for (int j = 0; j < NPL; ++j) sj[j] = 0;
      int c = 0;
#pragma unroll
      for (int t = 0; t < WS; ++t) {
        c += __popcll(x[u][t]);
#pragma unroll
        for (int j = 0; j < NPL; ++j) sj[j] += __popcll(x[u][t] & pl.get(j, t));
      }
      int v = 0;
#pragma unroll
      for (int j = 0; j < NPL; ++j) v += sj[j] << j;
      ip[u] = v;
      pc[u] = c;
    }
  } else {
#pragma unroll
    for (int u = 0; u < UN; ++u) code_ip<0, NPL>(row[u], W, pl, ip[u], pc[u]);
  }
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    float d0, l0;
    est_dl(pt, f[u], ct[u], est_y(pt, ip[u], pc[u]), d0, l0);
    const float dist = d0 + pt.pt, lb = l0 + pt.pt;
    const int32_t off = p[u] - start;
    if constexpr (PHASE == 0) {
      if (valid[u]) {
        Cand cd;
        cd.pos = p[u];
        cd.lb = lb;
        s.seg[w.seg + off] = cd;
        EstEnt e;
        e.dist = dist;
        e.pos = p[u];
        s.p0buf[w.p0slot + off] = e;
      }
    } else if constexpr (PHASE == 2) {
      if (valid[u]) {
        const int64_t o = (int64_t)p[u] - s.dbg_base;
        s.dbg_ip[o] = ip[u];
        s.dbg_pc[o] = pc[u];
        s.dbg_est[o] = estimate_est(rec, s.fac[p[u]].y, ip[u], pc[u]);
        s.dbg_dist[o] = dist;
        s.dbg_lb[o] = lb;
      }
    } else {
      const bool pass = valid[u] && (l0 <= tau);   // tau here is tau - pt
      const uint64_t m = __ballot(pass);
      if (pass) {
        Cand cd;
        cd.pos = p[u];
        cd.lb = lb;
        s.seg[w.seg + count + __popcll(m & lanemask_lt())] = cd;
      }
      count += __popcll(m);
    }
  }
}

// One unit: steps of UN blocks of 64 codes while they are full, then single
// blocks for the rest (short lists do not pay for a mostly masked wide step).
template <int WS, int UN, int PHASE, int NPL, typename PL>
__device__ __forceinline__ int scan_unit(const SearchDev& s, const UnitDesc& w, const PairRec& rec, const PL& pl,
                                         float tau, float hwk) {
  const PairTerms pt = s.metric != 0 ? pair_terms_ip(rec, hwk, uniform_f32(s.pair_pt[w.g])) : pair_terms(rec, hwk);
  tau -= pt.pt;   // the bound test takes lb - pt against tau - pt
  const int32_t start = (int32_t)w.start, wend = (int32_t)(w.start + w.len);
  int count = 0;
  int32_t b0 = start;
  for (; b0 + 64 * UN <= wend; b0 += 64 * UN) {
    // LDS planes are re-read every step (shared by its UN codes) rather than
    // hoisted into 8W registers, which would cut the occupancy
    if constexpr (!(WS >= 1 && WS <= 4)) asm volatile("" ::: "memory");
    scan_step<WS, UN, PHASE, NPL>(s, w, b0, wend, rec, pt, pl, tau, count);
  }
  for (; b0 < wend; b0 += 64) scan_step<WS, 1, PHASE, NPL>(s, w, b0, wend, rec, pt, pl, tau, count);
  return PHASE == 0 ? w.len : PHASE == 1 ? count : 0;
}

// Persistent scan: wave i of the grid takes units i, i + nwaves, ... of the
// phase's unit table (units are chunks of at most `chunk` codes, so a static
// round-robin balances them; no atomics and no per-unit searches). The unit
// loop is pipelined: while a unit is scanned, the descriptor two units ahead
// and the pair record and bit planes (one word per lane) of the next unit are
// already being loaded.
template <int WS, int UN, int PHASE, int NPL>
__global__ __launch_bounds__(kThreads) void k_scan_popcnt(SearchDev s) {
  __shared__ uint64_t lds_planes[kWaves][NPL * (kMaxCodeBits / 64)];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t total = uniform_i64((PHASE == 0 ? s.off_p0 : s.off_p1)[s.nq]);
  const UnitDesc* tab = PHASE == 0 ? s.units0 : s.units1;   // phase 2 runs the main-phase table
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  const int nplw = NPL * s.W;                     // plane words of a pair
  // plane words per lane: NPL W words spread over the wave
  constexpr int kPlPerLane = WS > 0 ? (NPL * WS + kWave - 1) / kWave : kMaxCodeBits / 64 * NPL / kWave;
  int64_t u = uniform_i64((int64_t)blockIdx.x * kWaves + wave);
  UnitDesc w, wn;
  PairRec rec;
  uint64_t plv[kPlPerLane];
  auto fetch_pair = [&](const UnitDesc& d, PairRec& r, uint64_t (&v)[kPlPerLane]) {
    r = s.pairs[d.g];
    const uint64_t* src = s.planes + d.g * nplw;
#pragma unroll
    for (int i = 0; i < kPlPerLane; ++i) {
      const int k = lane + i * kWave;
      v[i] = k < nplw ? src[k] : 0ull;
    }
  };
  if (u < total) {
    w = load_unit(tab, u);
    fetch_pair(w, rec, plv);
  }
  if (u + nw < total) wn = load_unit(tab, u + nw);
  while (u < total) {
    const int64_t u1 = u + nw, u2 = u + 2 * nw;
    UnitDesc wnn;
    if (u2 < total) wnn = load_unit(tab, u2);
    PairRec recn;
    uint64_t plvn[kPlPerLane];
    if (u1 < total) fetch_pair(wn, recn, plvn);
    PlanesFor<WS, NPL> pl;
    if constexpr (WS >= 1 && WS <= 4) {
#pragma unroll
      for (int j = 0; j < NPL; ++j)
#pragma unroll
        for (int t = 0; t < WS; ++t) {
          const int k = j * WS + t;   // word k sits in lane k % 64 of register k / 64
          const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)plv[k / kWave], k % kWave);
          const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(plv[k / kWave] >> 32), k % kWave);
          pl.w[j][t] = ((uint64_t)hi << 32) | lo;
        }
    } else {
      uint64_t* dst = lds_planes[wave];
#pragma unroll
      for (int i = 0; i < kPlPerLane; ++i) {
        const int k = lane + i * kWave;
        if (k < nplw) dst[k] = plv[i];
      }
      pl.p = dst;
      pl.Wr = s.W;
    }
    const float tau = PHASE == 1 ? uniform_f32(s.tau[w.q]) : __builtin_inff();
    const int count = scan_unit<WS, UN, PHASE, NPL>(s, w, rec, pl, tau, hwk);
    if (lane == 0) s.seg_count[w.count_slot] = count;
    u = u1;
    w = wn;
    wn = wnn;
    rec = recn;
#pragma unroll
    for (int i = 0; i < kPlPerLane; ++i) plv[i] = plvn[i];
  }
}

template <int WS, int UN, int NPL>
void launch_scan_np(const SearchDev& s, int phase, int grid, hipStream_t st) {
  if (phase == 0) {
    hipLaunchKernelGGL((k_scan_popcnt<WS, UN, 0, NPL>), dim3(grid), dim3(kThreads), 0, st, s);
  } else if (phase == 1) {
    hipLaunchKernelGGL((k_scan_popcnt<WS, UN, 1, NPL>), dim3(grid), dim3(kThreads), 0, st, s);
  } else {
    hipLaunchKernelGGL((k_scan_popcnt<WS, UN, 2, NPL>), dim3(grid), dim3(kThreads), 0, st, s);
  }
}
template <int WS, int UN>
void launch_scan_ws(const SearchDev& s, int phase, int grid, hipStream_t st) {
  if (s.npl == 8) {
    launch_scan_np<WS, UN, 8>(s, phase, grid, st);
  } else {
    launch_scan_np<WS, UN, 4>(s, phase, grid, st);
  }
}

}  // namespace

namespace {
template <int WS, int UN, int NPL>
int blocks_per_cu_np() {
  static int nb = 0;
  if (nb == 0) {
    int v0 = 0, v1 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v0, (const void*)k_scan_popcnt<WS, UN, 0, NPL>, kThreads, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&v1, (const void*)k_scan_popcnt<WS, UN, 1, NPL>, kThreads, 0) !=
            hipSuccess)
      v0 = v1 = 1;
    nb = std::max(1, std::min(v0, v1));
  }
  return nb;
}
template <int WS, int UN>
int blocks_per_cu_ws(int npl) {
  return npl == 8 ? blocks_per_cu_np<WS, UN, 8>() : blocks_per_cu_np<WS, UN, 4>();
}
}  // namespace

// Resident blocks per CU of the scan instantiation used for W words and npl planes (the
// smaller of its two phases): the persistent grid is sized to what fits, so
// that the static round-robin of units never waits for a second wave
// generation.
int scan_popcnt_blocks_per_cu(int W, int npl) {
  switch (W) {
    case 1: return blocks_per_cu_ws<1, 4>(npl);
    case 2: return blocks_per_cu_ws<2, 4>(npl);
    case 3: return blocks_per_cu_ws<3, 4>(npl);
    case 4: return blocks_per_cu_ws<4, 4>(npl);
    case 12: return blocks_per_cu_ws<12, 4>(npl);
    case 15: return blocks_per_cu_ws<15, 2>(npl);
    default: return blocks_per_cu_ws<0, 2>(npl);
  }
}

hipError_t launch_scan_popcnt(const SearchDev& s, int phase, int grid, hipStream_t st) {
  switch (s.W) {
    case 1: launch_scan_ws<1, 4>(s, phase, grid, st); break;
    case 2: launch_scan_ws<2, 4>(s, phase, grid, st); break;
    case 3: launch_scan_ws<3, 4>(s, phase, grid, st); break;
    case 4: launch_scan_ws<4, 4>(s, phase, grid, st); break;
    case 12: launch_scan_ws<12, 4>(s, phase, grid, st); break;   // D = 768
    case 15: launch_scan_ws<15, 2>(s, phase, grid, st); break;   // D = 960
    default: launch_scan_ws<0, 2>(s, phase, grid, st); break;
  }
  return hipGetLastError();
}

}  // namespace rbq
