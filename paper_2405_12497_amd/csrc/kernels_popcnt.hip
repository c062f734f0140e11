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
template <int WS, int UN, typename PL>
__device__ __forceinline__ int scan_chunk(const SearchDev& s, int phase, const UnitDesc& w,
                                          const PairRec& rec, const PL& pl, float tau, float hwk) {
  const int lane = lane_id();
  const int64_t seg_base = w.seg;
  const int64_t p0base = w.p0slot;
  const int32_t start = (int32_t)w.start, wend = (int32_t)(w.start + w.len);
  const int W = WS > 0 ? WS : s.W;
  int count = 0;
  for (int32_t b0 = start; b0 < wend; b0 += 64 * UN) {
    // LDS planes are re-read every iteration (shared by its UN codes) rather
    // than hoisted into 8W registers, which would cut the occupancy
    if constexpr (!(WS >= 1 && WS <= 4)) asm volatile("" ::: "memory");
    int32_t p[UN];
    bool valid[UN];
    float2 f[UN];
    int ip[UN], pc[UN];
    const uint64_t* row[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      valid[u] = b0 + 64 * u + lane < wend;
      p[u] = valid[u] ? b0 + 64 * u + lane : start;   // masked lanes read an in-bounds code
      f[u] = s.fac[p[u]];
      row[u] = code_row(s.codes, p[u], W);
    }
    if constexpr (WS > 0) {
      uint64_t x[UN][WS];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int t = 0; t < WS; ++t) x[u][t] = row[u][64 * t];
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
      for (int u = 0; u < UN; ++u) code_ip<0>(row[u], W, pl, ip[u], pc[u]);
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      float est, dist, lb;
      estimate(rec, f[u], ip[u], pc[u], hwk, est, dist, lb);
      lb = valid[u] ? lb : __builtin_inff();
      const int32_t off = p[u] - start;
      if (phase == 0) {
        if (valid[u]) {
          Cand cd;
          cd.pos = p[u];
          cd.lb = lb;
          s.seg[seg_base + off] = cd;
          EstEnt e;
          e.dist = dist;
          e.slot = (int32_t)(w.qcode + off);
          s.p0buf[p0base + off] = e;
        }
      } else {
        const bool pass = valid[u] && (lb <= tau);
        const uint64_t m = __ballot(pass);
        if (pass) {
          Cand cd;
          cd.pos = p[u];
          cd.lb = lb;
          s.seg[seg_base + count + __popcll(m & lanemask_lt())] = cd;
        }
        count += __popcll(m);
      }
    }
  }
  return phase == 0 ? w.len : count;
}

// Persistent scan: wave i of the grid takes units i, i + nwaves, ... of the
// phase's unit table (units are chunks of at most `chunk` codes, so a static
// round-robin balances them; no atomics and no per-unit searches).
template <int WS, int UN>
__global__ __launch_bounds__(kThreads) void k_scan_popcnt(SearchDev s, int phase) {
  __shared__ uint64_t lds_planes[kWaves][4 * (kMaxCodeBits / 64)];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t total = uniform_i64((phase == 0 ? s.off_p0 : s.off_p1)[s.nq]);
  const UnitDesc* tab = phase == 0 ? s.units0 : s.units1;
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t nw = (int64_t)gridDim.x * kWaves;
  int64_t u = uniform_i64((int64_t)blockIdx.x * kWaves + wave);
  UnitDesc w;
  if (u < total) w = load_unit(tab, u);
  while (u < total) {
    // the next unit's descriptor is requested before this unit's scan
    const int64_t un = u + nw;
    UnitDesc wn;
    if (un < total) wn = load_unit(tab, un);
    const PairRec rec = s.pairs[w.g];
    const uint64_t* src = s.planes + w.g * 4 * s.W;
    PlanesFor<WS> pl;
    if constexpr (WS >= 1 && WS <= 4) {
      pl.load(src);
    } else {
      uint64_t* dst = lds_planes[wave];
      for (int i = lane; i < 4 * s.W; i += kWave) dst[i] = src[i];
      pl.p = dst;
      pl.Wr = s.W;
    }
    const float tau = phase == 0 ? __builtin_inff() : uniform_f32(s.tau[w.q]);
    const int count = scan_chunk<WS, UN>(s, phase, w, rec, pl, tau, hwk);
    if (lane == 0) s.seg_count[w.count_slot] = count;
    u = un;
    w = wn;
  }
}

template <int WS, int UN>
void launch_scan_ws(const SearchDev& s, int phase, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_scan_popcnt<WS, UN>), dim3(grid), dim3(kThreads), 0, st, s, phase);
}

}  // namespace

namespace {
template <int WS, int UN>
int blocks_per_cu_ws() {
  static int nb = 0;
  if (nb == 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)k_scan_popcnt<WS, UN>, kThreads, 0) !=
            hipSuccess ||
        v < 1)
      v = 1;
    nb = v;
  }
  return nb;
}
}  // namespace

// Resident blocks per CU of the scan instantiation used for W words: the
// persistent grid is sized to exactly what fits, so that the static
// round-robin of units never waits for a second wave generation.
int scan_popcnt_blocks_per_cu(int W) {
  switch (W) {
    case 1: return blocks_per_cu_ws<1, 4>();
    case 2: return blocks_per_cu_ws<2, 4>();
    case 3: return blocks_per_cu_ws<3, 4>();
    case 4: return blocks_per_cu_ws<4, 2>();
    case 12: return blocks_per_cu_ws<12, 2>();
    case 15: return blocks_per_cu_ws<15, 2>();
    default: return blocks_per_cu_ws<0, 2>();
  }
}

hipError_t launch_scan_popcnt(const SearchDev& s, int phase, int grid, hipStream_t st) {
  switch (s.W) {
    case 1: launch_scan_ws<1, 4>(s, phase, grid, st); break;
    case 2: launch_scan_ws<2, 4>(s, phase, grid, st); break;
    case 3: launch_scan_ws<3, 4>(s, phase, grid, st); break;
    case 4: launch_scan_ws<4, 2>(s, phase, grid, st); break;
    case 12: launch_scan_ws<12, 2>(s, phase, grid, st); break;   // D = 768
    case 15: launch_scan_ws<15, 2>(s, phase, grid, st); break;   // D = 960
    default: launch_scan_ws<0, 2>(s, phase, grid, st); break;
  }
  return hipGetLastError();
}

}  // namespace rbq
