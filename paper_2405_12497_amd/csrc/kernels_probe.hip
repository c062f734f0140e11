// IVF probing (Sec. 4): per query, the nprobe lists with the smallest squared
// centroid distance, nearest first, ties to the lower list id.
#include "rbq_internal.hpp"
#include "wave_select.hpp"

namespace rbq {
namespace {

constexpr int kSelThreads = 256;
constexpr int kSelCap = 2048;   // nprobe handled with the keys in LDS; above: k_select_probe_large

// keys: distances as uint32 (non-negative floats order like their bit patterns),
// read from the distance row in global memory (no LDS copy of the row, so
// several queries' blocks share a CU). Sampled cut, then the exact radix
// selection when the cut does not isolate between P and kSelCap keys.
__device__ __forceinline__ uint32_t probe_key(const float* row, int k) { return __float_as_uint(fmaxf(row[k], 0.f)); }

__global__ __launch_bounds__(kSelThreads) void k_select_probe(const float* __restrict__ D,
                                                              int nlist, int nprobe,
                                                              const int32_t* __restrict__ nprobe_q,
                                                              int32_t* __restrict__ lists,
                                                              float* __restrict__ dists) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t sel[kSelCap];
  __shared__ uint32_t samp[256];
  __shared__ uint32_t sh_prefix, sh_rank, sh_nless, sh_nk;
  __shared__ uint32_t tie_scan[kSelThreads];
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & 63;
  int P = nprobe;
  if (nprobe_q) P = uniform_i32(min(max(nprobe_q[q], 1), nprobe));
  P = min(P, nlist);
  const float* row = D + q * (int64_t)nlist;
  // Sampled threshold: sort 256 evenly spaced keys and cut at a sample rank
  // expected to leave about 1.5 P + 32 keys at or below it. If that many keys
  // are kept (and they fit), sorting only them gives the answer; otherwise the
  // exact radix selection below runs.
  if (nlist >= 1024) {
    const int stride = nlist / 256;
    samp[threadIdx.x] = probe_key(row, threadIdx.x * stride);
    if (threadIdx.x == 0) sh_nk = 0;
    __syncthreads();
    for (int size = 2; size <= 256; size <<= 1)
      for (int st = size >> 1; st > 0; st >>= 1) {
        if (threadIdx.x < 128) {
          const int i = threadIdx.x;
          const int lo = 2 * i - (i & (st - 1)), hi = lo + st;
          const bool up = (lo & size) == 0;
          const uint32_t x = samp[lo], y = samp[hi];
          if ((x > y) == up) {
            samp[lo] = y;
            samp[hi] = x;
          }
        }
        __syncthreads();
      }
    const int sidx = min(255, (int)((1.5f * P + 32.f) * 256.f / (float)nlist) + 1);
    const uint32_t cut = (uint32_t)uniform_i32((int)samp[sidx]);
    // compaction of the keys <= cut in any order (the sort below orders them):
    // one LDS atomic per wave and step, four keys per thread in flight
    constexpr int kU = 4;
    for (int k0 = 0; k0 < nlist; k0 += kSelThreads * kU) {
      uint32_t kv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) kv[u] = probe_key(row, min(k0 + u * kSelThreads + (int)threadIdx.x, nlist - 1));
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int k = k0 + u * kSelThreads + threadIdx.x;
        const bool keep = k < nlist && kv[u] <= cut;
        const uint64_t m = __ballot(keep);
        if (m == 0ull) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&sh_nk, (uint32_t)__popcll(m));
        base = (uint32_t)__shfl((int)base, 0, kWave);
        const uint32_t idx = base + (uint32_t)__popcll(m & lanemask_lt());
        if (keep && idx < (uint32_t)kSelCap) sel[idx] = ((uint64_t)kv[u] << 32) | (uint32_t)k;
      }
    }
    __syncthreads();
    const int nk = uniform_i32((int)sh_nk);
    if (nk >= P && nk <= kSelCap) {
      int n2 = 1;
      while (n2 < nk) n2 <<= 1;
      for (int i = nk + threadIdx.x; i < n2; i += blockDim.x) sel[i] = ~0ull;
      __syncthreads();
      bitonic_sort_u64(sel, n2);
      for (int i = threadIdx.x; i < nprobe; i += blockDim.x) {
        if (i < P) {
          lists[q * nprobe + i] = (int32_t)(uint32_t)(sel[i] & 0xffffffffu);
          if (dists) dists[q * nprobe + i] = __uint_as_float((uint32_t)(sel[i] >> 32));
        } else {
          lists[q * nprobe + i] = -1;
          if (dists) dists[q * nprobe + i] = __builtin_inff();
        }
      }
      return;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sh_prefix = 0;
    sh_rank = P;
  }
  __syncthreads();
  uint32_t mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint32_t prefix = (uint32_t)uniform_i32((int)sh_prefix);
    for (int k = threadIdx.x; k < nlist; k += blockDim.x) {
      const uint32_t key = probe_key(row, k);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t rank = sh_rank, cum = 0;
      int b = 0;
      for (; b < 256; ++b) {
        if (cum + hist[b] >= rank) break;
        cum += hist[b];
      }
      sh_rank = rank - cum;
      sh_prefix = prefix | ((uint32_t)b << shift);
    }
    mask |= 255u << shift;
    __syncthreads();
  }
  const uint32_t thr = (uint32_t)uniform_i32((int)sh_prefix);   // key of the P-th smallest
  const uint32_t need = (uint32_t)uniform_i32((int)sh_rank);    // how many keys equal to thr to take
  if (threadIdx.x == 0) sh_nless = 0;
  __syncthreads();
  // keys strictly below the threshold (P - need of them), any order
  for (int k = threadIdx.x; k < nlist; k += blockDim.x) {
    const uint32_t key = probe_key(row, k);
    if (key < thr) {
      const uint32_t at = atomicAdd(&sh_nless, 1u);
      sel[at] = ((uint64_t)key << 32) | (uint32_t)k;
    }
  }
  // ties: the first `need` in list-id order; thread t scans a contiguous range
  const int per = (nlist + blockDim.x - 1) / blockDim.x;
  const int kb = threadIdx.x * per, ke = min(nlist, kb + per);
  uint32_t mine = 0;
  for (int k = kb; k < ke; ++k) mine += (probe_key(row, k) == thr);
  tie_scan[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      const uint32_t c = tie_scan[t];
      tie_scan[t] = run;
      run += c;
    }
  }
  __syncthreads();
  const uint32_t nless = (uint32_t)P - need;
  uint32_t rank = tie_scan[threadIdx.x];
  for (int k = kb; k < ke && rank < need; ++k) {
    if (probe_key(row, k) == thr) {
      sel[nless + rank] = ((uint64_t)thr << 32) | (uint32_t)k;
      ++rank;
    }
  }
  __syncthreads();
  int n2 = 1;
  while (n2 < P) n2 <<= 1;
  for (int i = P + threadIdx.x; i < n2; i += blockDim.x) sel[i] = ~0ull;
  __syncthreads();
  bitonic_sort_u64(sel, n2);
  for (int i = threadIdx.x; i < nprobe; i += blockDim.x) {
    if (i < P) {
      lists[q * nprobe + i] = (int32_t)(uint32_t)(sel[i] & 0xffffffffu);
      if (dists) dists[q * nprobe + i] = __uint_as_float((uint32_t)(sel[i] >> 32));
    } else {
      lists[q * nprobe + i] = -1;
      if (dists) dists[q * nprobe + i] = __builtin_inff();
    }
  }
}

// nprobe above kSelCap: the same exact selection with the keys read from the
// distance row in global memory and the selected (key, list) pairs sorted in
// dynamic LDS (next power of two of nprobe entries).
constexpr int kSelLargeThreads = 1024;   // the LDS sort of thousands of keys takes the whole block

__global__ __launch_bounds__(kSelLargeThreads) void k_select_probe_large(const float* __restrict__ D, int nlist,
                                                                         int nprobe,
                                                                         const int32_t* __restrict__ nprobe_q,
                                                                         int32_t* __restrict__ lists,
                                                                         float* __restrict__ dists) {
  extern __shared__ uint64_t selbig[];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sh_prefix, sh_rank, sh_nless;
  __shared__ uint32_t tie_scan[kSelLargeThreads];
  const int64_t q = blockIdx.x;
  int P = nprobe;
  if (nprobe_q) P = uniform_i32(min(max(nprobe_q[q], 1), nprobe));
  P = min(P, nlist);
  const float* row = D + q * (int64_t)nlist;
  auto key_of = [&](int k) { return __float_as_uint(fmaxf(row[k], 0.f)); };
  if (threadIdx.x == 0) {
    sh_prefix = 0;
    sh_rank = P;
  }
  __syncthreads();
  uint32_t mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t prefix = (uint32_t)uniform_i32((int)sh_prefix);
    for (int k = threadIdx.x; k < nlist; k += blockDim.x) {
      const uint32_t key = key_of(k);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t rank = sh_rank, cum = 0;
      int b = 0;
      for (; b < 256; ++b) {
        if (cum + hist[b] >= rank) break;
        cum += hist[b];
      }
      sh_rank = rank - cum;
      sh_prefix = prefix | ((uint32_t)b << shift);
    }
    mask |= 255u << shift;
    __syncthreads();
  }
  const uint32_t thr = (uint32_t)uniform_i32((int)sh_prefix);
  const uint32_t need = (uint32_t)uniform_i32((int)sh_rank);
  if (threadIdx.x == 0) sh_nless = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nlist; k += blockDim.x) {
    const uint32_t key = key_of(k);
    if (key < thr) selbig[atomicAdd(&sh_nless, 1u)] = ((uint64_t)key << 32) | (uint32_t)k;
  }
  const int per = (nlist + blockDim.x - 1) / blockDim.x;
  const int kb = threadIdx.x * per, ke = min(nlist, kb + per);
  uint32_t mine = 0;
  for (int k = kb; k < ke; ++k) mine += (key_of(k) == thr);
  tie_scan[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      const uint32_t c = tie_scan[t];
      tie_scan[t] = run;
      run += c;
    }
  }
  __syncthreads();
  const uint32_t nless = (uint32_t)P - need;
  uint32_t rank = tie_scan[threadIdx.x];
  for (int k = kb; k < ke && rank < need; ++k) {
    if (key_of(k) == thr) {
      selbig[nless + rank] = ((uint64_t)thr << 32) | (uint32_t)k;
      ++rank;
    }
  }
  __syncthreads();
  int n2 = 1;
  while (n2 < P) n2 <<= 1;
  for (int i = P + threadIdx.x; i < n2; i += blockDim.x) selbig[i] = ~0ull;
  __syncthreads();
  bitonic_sort_u64(selbig, n2);
  for (int i = threadIdx.x; i < nprobe; i += blockDim.x) {
    if (i < P) {
      lists[q * nprobe + i] = (int32_t)(uint32_t)(selbig[i] & 0xffffffffu);
      if (dists) dists[q * nprobe + i] = __uint_as_float((uint32_t)(selbig[i] >> 32));
    } else {
      lists[q * nprobe + i] = -1;
      if (dists) dists[q * nprobe + i] = __builtin_inff();
    }
  }
}

// ------------------------------------------------------------------ rank select
// Few queries with a large nprobe: the selection as ranks, spread over many
// blocks instead of one block per query. A list's rank in its query's row is
// the number of lists whose key (distance bits, then list id) is smaller; the
// lists of rank < P land in slot rank. Block (b, q) ranks lists
// 16 b .. 16 b + 15 of query q: each of its 512 threads holds KP keys of the
// row (lists t + 512 r) in registers and counts those below each of the 16
// keys, and the counts are summed over the block. nlist^2 compares per query.
constexpr int kRankThreads = 512, kRankElems = 16;

template <int KP>
__global__ __launch_bounds__(kRankThreads) void k_select_probe_rank(const float* __restrict__ D, int nlist,
                                                                    int nprobe,
                                                                    const int32_t* __restrict__ nprobe_q,
                                                                    int32_t* __restrict__ lists,
                                                                    float* __restrict__ dists) {
  __shared__ int part[kRankThreads / kWave][kRankElems];
  const int64_t q = blockIdx.y;
  const int i0 = blockIdx.x * kRankElems;
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  int P = nprobe;
  if (nprobe_q) P = uniform_i32(min(max(nprobe_q[q], 1), nprobe));
  P = min(P, nlist);
  const float* row = D + q * (int64_t)nlist;
  auto key_of = [&](int k) {
    return ((uint64_t)__float_as_uint(fmaxf(row[k], 0.f)) << 32) | (uint32_t)k;
  };
  uint64_t kj[KP];
#pragma unroll
  for (int r = 0; r < KP; ++r) {
    const int j = tid + kRankThreads * r;
    kj[r] = key_of(min(j, nlist - 1));
  }
#pragma unroll
  for (int r = 0; r < KP; ++r) kj[r] = tid + kRankThreads * r < nlist ? kj[r] : ~0ull;
  int cnt[kRankElems];
#pragma unroll
  for (int e = 0; e < kRankElems; ++e) {
    const uint64_t ki = key_of(min(i0 + e, nlist - 1));   // the same for every lane
    int c = 0;
#pragma unroll
    for (int r = 0; r < KP; ++r) c += kj[r] < ki ? 1 : 0;
    cnt[e] = c;
  }
#pragma unroll
  for (int e = 0; e < kRankElems; ++e) {
    const int c = wave_sum_i(cnt[e]);
    if (lane == 0) part[wave][e] = c;
  }
  __syncthreads();
  if (tid < kRankElems && i0 + tid < nlist) {
    int rank = 0;
#pragma unroll
    for (int w = 0; w < kRankThreads / kWave; ++w) rank += part[w][tid];
    if (rank < P) {
      const int i = i0 + tid;
      lists[q * nprobe + rank] = i;
      if (dists) dists[q * nprobe + rank] = fmaxf(row[i], 0.f);
    }
  }
  if (blockIdx.x == 0) {
    for (int i = P + tid; i < nprobe; i += kRankThreads) {
      lists[q * nprobe + i] = -1;
      if (dists) dists[q * nprobe + i] = __builtin_inff();
    }
  }
}

// The rank selection's cost bound: at most 16 queries and nq * nlist^2 <= 2^31.
bool rank_select(int64_t nq, int nlist) {
  return nq <= 16 && nlist <= kRankThreads * 32 && (double)nq * nlist * nlist <= 2147483648.0;
}

// ------------------------------------------------------------------ wave select
// One wave per query for nprobe <= kWSelMaxP: the wave selection over the
// query's distance row (keys: distance bits, non-negative floats ordering like
// their bit patterns; ties to the lower list id), no block barriers.
constexpr int kWSelMaxP = 256;
constexpr int kWSelWaves = kSelThreads / kWave;

__global__ __launch_bounds__(kSelThreads) void k_select_probe_wave(const float* __restrict__ D, int64_t nq,
                                                                   int nlist, int nprobe,
                                                                   const int32_t* __restrict__ nprobe_q,
                                                                   int32_t* __restrict__ lists,
                                                                   float* __restrict__ dists) {
  __shared__ uint64_t selw[kWSelWaves][kWSelCap];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWSelWaves + wave;
  if (q >= nq) return;   // whole waves
  uint64_t* sel = selw[wave];
  int P = nprobe;
  if (nprobe_q) P = uniform_i32(min(max(nprobe_q[q], 1), nprobe));
  P = min(P, nlist);
  const float* row = D + q * (int64_t)nlist;
  wave_smallest<16, 64>([&](int i) { return __float_as_uint(row[i]); },
                        [](uint32_t v) { return __float_as_uint(fmaxf(__uint_as_float(v), 0.f)); }, nlist, P,
                        sel);
  for (int i = lane; i < nprobe; i += kWave) {
    const bool live = i < P;
    const uint64_t v = sel[min(i, P - 1)];
    lists[q * nprobe + i] = live ? (int32_t)(uint32_t)(v & 0xffffffffu) : -1;
    if (dists) dists[q * nprobe + i] = live ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
  }
}

// ------------------------------------------------------------------ grouped wave select
// nprobe <= 64 with the row's group minima (the minimum of each group of 16
// lists, written by the centroid-distance kernel; group g holds lists
// 64 (g / 4) + 4 (g % 4) + 16 j + e, j, e < 4). Lane l holds the minima of
// groups l, l + 64, ...; the cut is the P-th smallest of the 64 lane minima,
// so at least P group minima (P distinct distances) are at or below it. Only a
// group whose minimum is at or below the cut can hold a distance at or below
// it: those groups' 16 distances are read (16 lanes per group), the ones at or
// below the cut are compacted and sorted, and the first P are the answer (the
// P smallest are all at or below the cut). More than kGrpSelCap kept
// distances (many equal ones) fall back to the full-row wave selection.
constexpr int kGrpSelCap = kWSelCap / 2;   // sel entries; the group list uses the upper half
constexpr int kGrpMaxG = 1024;             // groups per row (nlist <= 16384)
constexpr int kGrpMaxP = kWave;

template <int R>
__global__ __launch_bounds__(kSelThreads) void k_select_probe_grp(const float* __restrict__ D,
                                                                  const float* __restrict__ GM, int64_t nq,
                                                                  int nlist, int nprobe,
                                                                  const int32_t* __restrict__ nprobe_q,
                                                                  int32_t* __restrict__ lists,
                                                                  float* __restrict__ dists) {
  __shared__ uint64_t selw[kWSelWaves][kWSelCap];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t q = (int64_t)blockIdx.x * kWSelWaves + wave;
  if (q >= nq) return;   // whole waves
  uint64_t* sel = selw[wave];
  int32_t* grp = reinterpret_cast<int32_t*>(sel + kGrpSelCap);   // kGrpMaxG entries
  int P = nprobe;
  if (nprobe_q) P = uniform_i32(min(max(nprobe_q[q], 1), nprobe));
  P = min(P, nlist);
  const int G = ((nlist + 63) >> 6) * 4;
  const float* row = D + q * (int64_t)nlist;
  const float* gm = GM + q * (int64_t)G;
  auto key = [](float v) { return __float_as_uint(fmaxf(v, 0.f)); };
  uint32_t gk[R];   // all R loads in flight at once (indices past G read group G - 1)
#pragma unroll
  for (int j = 0; j < R; ++j) gk[j] = __float_as_uint(gm[min(j * kWave + lane, G - 1)]);
#pragma unroll
  for (int j = 0; j < R; ++j) keep_loaded(gk[j]);
#pragma unroll
  for (int j = 0; j < R; ++j) gk[j] = (j * kWave + lane < G) ? key(__uint_as_float(gk[j])) : 0xFFFFFFFFu;
  uint32_t lm[1] = {gk[0]};
#pragma unroll
  for (int j = 1; j < R; ++j) lm[0] = min(lm[0], gk[j]);
  wave_bitonic<1>(lm);
  const uint32_t cut = (uint32_t)__builtin_amdgcn_readlane((int)lm[0], P - 1);
  // the groups whose minimum is at or below the cut
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < R; ++j) cnt += gk[j] <= cut;
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int ng = __builtin_amdgcn_readlane(incl, kWave - 1);
  {
    int at = incl - cnt;
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (gk[j] <= cut) grp[at++] = j * kWave + lane;
  }
  wave_lds_sync();
  // their distances, 16 groups per round (4 per load, 16 lanes each)
  const int sub = lane & 15, gl = lane >> 4;
  int total = 0;
  for (int b0 = 0; b0 < ng; b0 += 16) {
    float rv[4];
    int col[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gi = b0 + u * 4 + gl;
      const int g = grp[min(gi, ng - 1)];
      col[u] = (g >> 2) * 64 + (g & 3) * 4 + (sub >> 2) * 16 + (sub & 3);
      rv[u] = row[min(col[u], nlist - 1)];
    }
    uint32_t kv[4];
    int c = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = b0 + u * 4 + gl < ng && col[u] < nlist;
      kv[u] = in ? key(rv[u]) : 0xFFFFFFFFu;
      c += kv[u] <= cut;
    }
    int ic = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(ic, o, kWave);
      if (lane >= o) ic += y;
    }
    const int tot = __builtin_amdgcn_readlane(ic, kWave - 1);
    if (total + tot <= kGrpSelCap) {
      int at = total + ic - c;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (kv[u] <= cut) sel[at++] = ((uint64_t)kv[u] << 32) | (uint32_t)col[u];
    }
    total += tot;
  }
  if (total <= kGrpSelCap) {
    wave_sort_sel(sel, total);
  } else {
    wave_lds_sync();   // the group list is no longer read
    // streaming form (no resident keys), so the rare fallback does not set
    // the kernel's register budget
    wave_smallest<16, 0>([&](int i) { return __float_as_uint(row[i]); },
                         [&](uint32_t v) { return key(__uint_as_float(v)); }, nlist, P, sel);
  }
  for (int i = lane; i < nprobe; i += kWave) {
    const bool live = i < P;
    const uint64_t v = sel[min(i, P - 1)];
    lists[q * nprobe + i] = live ? (int32_t)(uint32_t)(v & 0xffffffffu) : -1;
    if (dists) dists[q * nprobe + i] = live ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_inff();
  }
}

}  // namespace

// Probe rank of the neighbours' lists (training labels of the learned
// nprobe). One wave per query: among the lists of its k neighbour ids (ids < 0
// are skipped) the one latest in probe order, i.e. with the largest key
// (squared centroid distance, list id), and its rank = the number of lists
// with a smaller key, so that the smallest nprobe probing every neighbour's
// list is rank + 1 (0 when no id is valid).
__global__ __launch_bounds__(kSelThreads) void k_probe_need(const float* __restrict__ D, int64_t nq, int nlist,
                                                            const int64_t* __restrict__ nn, int k,
                                                            const int32_t* __restrict__ id2list, int64_t n,
                                                            int32_t* __restrict__ need) {
  const int64_t q = (int64_t)blockIdx.x * (kSelThreads / kWave) + (threadIdx.x >> 6);
  if (q >= nq) return;   // whole waves
  const int lane = lane_id();
  const float* row = D + q * (int64_t)nlist;
  // the largest (distance bits, list) key among the neighbours' lists
  uint64_t worst = 0;
  bool any = false;
  for (int j = lane; j < k; j += kWave) {
    const int64_t id = nn[q * k + j];
    if (id < 0 || id >= n) continue;
    const int32_t l = id2list[id];
    const uint64_t key = ((uint64_t)__float_as_uint(fmaxf(row[l], 0.f)) << 32) | (uint32_t)l;
    worst = any && worst > key ? worst : key;
    any = true;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = __shfl_xor(worst, o, kWave);
    worst = worst > y ? worst : y;
  }
  const bool has = __ballot(any) != 0ull;
  int cnt = 0;
  for (int l = lane; l < nlist; l += kWave) {
    const uint64_t key = ((uint64_t)__float_as_uint(fmaxf(row[l], 0.f)) << 32) | (uint32_t)l;
    cnt += key < worst;
  }
  cnt = wave_sum_i(cnt);
  if (lane == 0) need[q] = has ? cnt + 1 : 0;
}

hipError_t launch_probe_need(const float* D, int64_t nq, int nlist, const int64_t* nn, int k, const int32_t* id2list,
                             int64_t n, int32_t* need, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  const int per = kSelThreads / kWave;
  hipLaunchKernelGGL(k_probe_need, dim3((unsigned)((nq + per - 1) / per)), dim3(kSelThreads), 0, st, D, nq, nlist,
                     nn, k, id2list, n, need);
  return hipGetLastError();
}

hipError_t launch_select_probe(const float* D, const float* gmin, int64_t nq, int nlist, int nprobe,
                               const int32_t* nprobe_q, int32_t* lists, float* dists,
                               hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  const int G = (nlist + 63) / 64 * 4;
  if (gmin && centroid_gmin(nq, nlist) && nprobe <= kGrpMaxP && G <= kGrpMaxG) {
    const dim3 grid((unsigned)((nq + kWSelWaves - 1) / kWSelWaves));
    if (G <= 4 * kWave)
      hipLaunchKernelGGL((k_select_probe_grp<4>), grid, dim3(kSelThreads), 0, st, D, gmin, nq, nlist, nprobe,
                         nprobe_q, lists, dists);
    else
      hipLaunchKernelGGL((k_select_probe_grp<kGrpMaxG / kWave>), grid, dim3(kSelThreads), 0, st, D, gmin, nq,
                         nlist, nprobe, nprobe_q, lists, dists);
    return hipGetLastError();
  }
  if (nprobe > kWSelMaxP && rank_select(nq, nlist)) {
    const dim3 grid((unsigned)((nlist + kRankElems - 1) / kRankElems), (unsigned)nq);
    const int kp = (nlist + kRankThreads - 1) / kRankThreads;
    if (kp <= 1)
      hipLaunchKernelGGL(k_select_probe_rank<1>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    else if (kp <= 2)
      hipLaunchKernelGGL(k_select_probe_rank<2>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    else if (kp <= 4)
      hipLaunchKernelGGL(k_select_probe_rank<4>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    else if (kp <= 8)
      hipLaunchKernelGGL(k_select_probe_rank<8>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    else if (kp <= 16)
      hipLaunchKernelGGL(k_select_probe_rank<16>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    else
      hipLaunchKernelGGL(k_select_probe_rank<32>, grid, dim3(kRankThreads), 0, st, D, nlist, nprobe, nprobe_q, lists, dists);
    return hipGetLastError();
  }
  if (nprobe > kSelCap) {
    int n2 = 1;
    while (n2 < nprobe) n2 <<= 1;
    const size_t big = (size_t)n2 * sizeof(uint64_t);
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return hipErrorInvalidValue;
    if (big + 8192 > (size_t)lim) return hipErrorInvalidConfiguration;   // 8 KiB for the static LDS
    static bool big_attr = false;
    if (!big_attr) {
      (void)hipFuncSetAttribute((const void*)k_select_probe_large,
                                hipFuncAttributeMaxDynamicSharedMemorySize, lim - 8192);
      big_attr = true;
    }
    hipLaunchKernelGGL(k_select_probe_large, dim3((unsigned)nq), dim3(kSelLargeThreads), big, st, D, nlist,
                       nprobe, nprobe_q, lists, dists);
    return hipGetLastError();
  }
  if (nprobe <= kWSelMaxP) {
    hipLaunchKernelGGL(k_select_probe_wave, dim3((unsigned)((nq + kWSelWaves - 1) / kWSelWaves)),
                       dim3(kSelThreads), 0, st, D, nq, nlist, nprobe, nprobe_q, lists, dists);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_select_probe, dim3((unsigned)nq), dim3(kSelThreads), 0, st, D, nlist,
                     nprobe, nprobe_q, lists, dists);
  return hipGetLastError();
}

}  // namespace rbq
