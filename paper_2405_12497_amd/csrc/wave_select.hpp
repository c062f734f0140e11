// Wave-level selection and sorting: one wave owns one query and a region of
// LDS, so none of these routines uses a block barrier. A wave's LDS operations
// complete in issue order; wave_lds_sync only keeps the compiler from moving
// LDS accesses across it.
#pragma once
#include "rbq_internal.hpp"

namespace rbq {

// Marks a loaded value as used at this point, unconditionally. A value that
// is only consumed under a branch lets the compiler move its load into that
// branch, where the load waits for every earlier one before it issues; a use
// placed after a batch of loads keeps them issued together.
template <typename T>
__device__ __forceinline__ void keep_loaded(const T& x) {
  asm volatile("" ::"v"(x));
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of N * 64 values held as v[r] at element r * 64 + lane,
// ascending: strides below 64 exchange across lanes, larger ones across registers.
template <int N, typename T>
__device__ __forceinline__ void wave_bitonic(T (&v)[N]) {
  const int lane = lane_id();
#pragma unroll
  for (int size = 2; size <= N * kWave; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= kWave) {
        const int rs = stride / kWave;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          if ((r & rs) == 0) {
            const bool up = (((r * kWave) & size) == 0);
            const T x = v[r], y = v[r + rs];
            if ((x > y) == up) {
              v[r] = y;
              v[r + rs] = x;
            }
          }
        }
      } else {
        const bool lower = (lane & stride) == 0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const bool up = (((r * kWave + lane) & size) == 0);
          const T y = __shfl_xor(v[r], stride, kWave);
          const bool take_min = (lower == up);
          v[r] = take_min ? (v[r] < y ? v[r] : y) : (v[r] < y ? y : v[r]);
        }
      }
    }
  }
}

// The same network over n (power of two) values in the wave's LDS region.
__device__ inline void wave_bitonic_lds_u64(uint64_t* a, int n) {
  const int lane = lane_id();
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < n / 2; i += kWave) {
        const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = a[lo], y = a[hi];
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      wave_lds_sync();
    }
  }
}

// Sorts sel[0..total) (total <= kWSelCap) ascending, in registers up to 256
// values and in LDS above.
constexpr int kWSelCap = 1024;

__device__ inline void wave_sort_sel(uint64_t* sel, int total) {
  const int lane = lane_id();
  auto in_regs = [&](auto n_tag) {
    constexpr int N = decltype(n_tag)::value;
    uint64_t v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int e = r * kWave + lane;
      v[r] = e < total ? sel[e] : ~0ull;
    }
    wave_bitonic<N>(v);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int e = r * kWave + lane;
      if (e < total) sel[e] = v[r];
    }
  };
  wave_lds_sync();
  if (total <= 64) {
    in_regs(IntC<1>{});
  } else if (total <= 128) {
    in_regs(IntC<2>{});
  } else if (total <= 256) {
    in_regs(IntC<4>{});
  } else {
    int n2 = 512;
    while (n2 < total) n2 <<= 1;
    for (int e = total + lane; e < n2; e += kWave) sel[e] = ~0ull;
    wave_lds_sync();
    wave_bitonic_lds_u64(sel, n2);
  }
  wave_lds_sync();
}

// The P smallest of the n values (key(i) << 32 | i), 1 <= P <= n, left in
// sel[0..P) in ascending order (ties between equal keys by index). key(i) is
// called for 0 <= i < n only and must return less than 0xFFFFFFFF. sel holds
// kWSelCap values; P must not exceed 256.
//
// A sorted sample of 256 keys gives a cut expected to keep about 1.5 P + 48
// values; the values at or below it are compacted into sel (ballot prefix) and
// sorted. A cut that keeps fewer than P or more than kWSelCap values is moved
// along the sample (4x further or closer) and tried again; each failed cut
// narrows the key range [lo, hi] that a final exact bisection searches, after
// which the ties at the P-th key are taken in index order.
//
// Rows of at most 64 R values take a faster path first: each lane loads all
// of its values at once (R loads in flight), and the cut is the P-th smallest
// of the 64 lane minima when P <= 64, else of 256 group minima (lane l, group
// r: the minimum of its values in batches j = r mod 4). The P smallest minima
// are P distinct values at or below the cut, so the cut always keeps at least
// P values; only more than kWSelCap sends the row to the exact path.
//
// load(i) returns the raw 32-bit word of value i and xf(raw) its key, so the
// loads of a batch stay independent of the key arithmetic.
template <int B, int R, class Load, class Xf>
__device__ void wave_smallest(Load load, Xf xf, int n, int P, uint64_t* sel) {
  const int lane = lane_id();
  auto key = [&](int i) { return xf(load(i)); };
  // fb(c0, kv): batch by batch, kv[j] = key of value c0 + j * 64 + lane
  // (0xFFFFFFFF past n). Full batches load without bounds tests (so all B
  // loads of a lane are in flight together); only a ragged last batch is
  // checked.
  auto stream = [&](auto&& fb) {
    int c0 = 0;
    for (; c0 + B * kWave <= n; c0 += B * kWave) {
      uint32_t kv[B];
#pragma unroll
      for (int j = 0; j < B; ++j) kv[j] = key(c0 + j * kWave + lane);
      fb(c0, kv);
    }
    if (c0 < n) {   // clamped loads (all in flight together), then the keys
      uint32_t kv[B];
#pragma unroll
      for (int j = 0; j < B; ++j) kv[j] = load(min(c0 + j * kWave + lane, n - 1));
#pragma unroll
      for (int j = 0; j < B; ++j) kv[j] = c0 + j * kWave + lane < n ? xf(kv[j]) : 0xFFFFFFFFu;
      fb(c0, kv);
    }
  };
  uint32_t lo = 0, hi = 0xFFFFFFFEu;
  int total = 0;   // wave-uniform count of values <= cut
  // each lane counts its kept values of a batch, one wave scan of the counts
  // places them, and each lane writes its own (order within sel is
  // immaterial: the sort orders by (key, index))
  auto compact = [&](uint32_t cut) {
    total = 0;
    stream([&](int c0, const uint32_t (&kv)[B]) {
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < B; ++j) cnt += kv[j] <= cut;
      int incl = cnt;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
      }
      const int tot = __builtin_amdgcn_readlane(incl, kWave - 1);
      if (total + tot <= kWSelCap) {
        int at = total + incl - cnt;
#pragma unroll
        for (int j = 0; j < B; ++j)
          if (kv[j] <= cut) sel[at++] = ((uint64_t)kv[j] << 32) | (uint32_t)(c0 + j * kWave + lane);
      }
      total += tot;
    });
    if (total < P) lo = max(lo, cut + 1);
    else if (total > kWSelCap) hi = min(hi, cut);
    return total >= P && total <= kWSelCap;
  };
  bool ok = false;
  if (R > 0 && n <= R * kWave) {
    constexpr int RR = R > 0 ? R : 1;
    // every lane issues all RR loads at once (indices past n read value n - 1):
    // loads under per-batch branches would each wait at the branch's join
    uint32_t kr[RR];
#pragma unroll
    for (int j = 0; j < RR; ++j) kr[j] = load(min(j * kWave + lane, n - 1));
#pragma unroll
    for (int j = 0; j < RR; ++j) keep_loaded(kr[j]);
#pragma unroll
    for (int j = 0; j < RR; ++j) kr[j] = (j * kWave + lane < n) ? xf(kr[j]) : 0xFFFFFFFFu;
    uint32_t cut = 0xFFFFFFFEu;
    if (n > 256 && P <= kWave) {
      // the P-th smallest of the 64 lane minima (every lane holds values)
      uint32_t lm[1] = {kr[0]};
#pragma unroll
      for (int j = 1; j < RR; ++j) lm[0] = min(lm[0], kr[j]);
      wave_bitonic<1>(lm);
      cut = (uint32_t)__builtin_amdgcn_readlane((int)lm[0], P - 1);
    } else if (n > 256) {
      uint32_t gm[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll
      for (int j = 0; j < RR; ++j) gm[j & 3] = min(gm[j & 3], kr[j]);
      wave_bitonic<4>(gm);
      const int sidx = P - 1;
      uint32_t pick = gm[0];
#pragma unroll
      for (int r = 1; r < 4; ++r) pick = (sidx / kWave == r) ? gm[r] : pick;
      cut = (uint32_t)__builtin_amdgcn_readlane((int)pick, sidx % kWave);
    }
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < RR; ++j) cnt += kr[j] <= cut;
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    total = __builtin_amdgcn_readlane(incl, kWave - 1);
    if (total <= kWSelCap) {
      int at = incl - cnt;
#pragma unroll
      for (int j = 0; j < RR; ++j)
        if (kr[j] <= cut) sel[at++] = ((uint64_t)kr[j] << 32) | (uint32_t)(j * kWave + lane);
    }
    if (total < P) lo = max(lo, cut + 1);
    else if (total > kWSelCap) hi = min(hi, cut);
    ok = total >= P && total <= kWSelCap;
  } else if (n > 256) {
    const int stride = n / 256;
    uint32_t sm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) sm[r] = key((r * kWave + lane) * stride);   // < 256 stride <= n
    wave_bitonic<4>(sm);
    int sidx = min(255, (int)((1.5f * P + 32.f) * 256.f / (float)n) + 1);
    for (int attempt = 0; attempt < 3 && !ok; ++attempt) {
      uint32_t pick = sm[0];
#pragma unroll
      for (int r = 1; r < 4; ++r) pick = (sidx / kWave == r) ? sm[r] : pick;
      const uint32_t cut = (uint32_t)__builtin_amdgcn_readlane((int)pick, sidx % kWave);
      ok = compact(cut);
      if (ok) break;
      const int next = total < P ? min(255, 4 * sidx + 8) : sidx / 4;
      if (next == sidx) break;
      sidx = next;
    }
  } else {
    ok = compact(0xFFFFFFFEu);
  }
  if (!ok) {
    // exact: T = the smallest key with at least P values <= T (in [lo, hi])
    auto count_le = [&](uint32_t t) {
      int c = 0;
      stream([&](int, const uint32_t (&kv)[B]) {
#pragma unroll
        for (int j = 0; j < B; ++j) c += (kv[j] <= t);
      });
      return wave_sum_i(c);
    };
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (count_le(mid) >= P) hi = mid; else lo = mid + 1;
    }
    const uint32_t T = lo;
    int nless = 0;
    stream([&](int, const uint32_t (&kv)[B]) {
#pragma unroll
      for (int j = 0; j < B; ++j) nless += (kv[j] < T);
    });
    nless = wave_sum_i(nless);
    const int need = P - nless;   // ties at T, lowest indices first
    int at_less = 0, tie_run = 0;
    stream([&](int c0, const uint32_t (&kv)[B]) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const uint32_t k = kv[j];
        const uint32_t i = (uint32_t)(c0 + j * kWave + lane);
        const uint64_t ml = __ballot(k < T), mt = __ballot(k == T);
        if (k < T) sel[at_less + __popcll(ml & lanemask_lt())] = ((uint64_t)k << 32) | i;
        const int rank = tie_run + __popcll(mt & lanemask_lt());
        if (k == T && rank < need) sel[nless + rank] = ((uint64_t)k << 32) | i;
        at_less += __popcll(ml);
        tie_run += __popcll(mt);
      }
    });
    total = P;
  }
  wave_sort_sel(sel, total);
}

// Bitonic sort of n (power of two) 64-bit keys in LDS, ascending, by the
// whole block (every thread calls it).
__device__ inline void bitonic_sort_u64(uint64_t* a, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t x = a[lo], y = a[hi];
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace rbq
