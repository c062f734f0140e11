// Batched scan: the integer <x_b, q_u> of Sec. 3.3.2 for all (query, code)
// pairs of one IVF list at once, as an int8 matrix product on the MFMA units:
//   IP[pairs x codes] = Qu[pairs x D] (values 0..15) * Xb[D x codes] (0/1).
// The paper evaluates the same batched contraction with 4-bit look-up tables
// in SIMD registers; on CDNA4 the contraction maps onto v_mfma_i32_16x16x64_i8.
//
// Grouping. The (query, list) pairs of the main phase are bucketed by list.
// A work unit is (list, chunk of the list's codes, group of 16 pairs): the 16
// quantised queries are staged in LDS once and every 64-code block of the
// chunk is multiplied against them; each wave owns 16 codes of the block,
// expands their bits to bytes in registers and issues one MFMA per 64
// dimensions. Candidates (lb <= tau) are compacted per pair in code order, so
// the segments are identical to those of the popcount scan.
#include "rbq_internal.hpp"
#include "rbq_runtime.hpp"
#include "scan_code.hpp"

namespace rbq {
namespace {

constexpr int kThreads = 256;
typedef int i32x4 __attribute__((ext_vector_type(4)));

struct RowInfo {
  PairRec rec;
  float tau;
  int32_t valid;      // 1 when this row's chunk belongs to the scanned phase
  int64_t seg_base;   // first segment slot of (pair, chunk)
  int64_t count_slot; // seg_count index of (pair, chunk)
};

// 4 bits -> 4 bytes of 0/1: the nibble's bits land on bits 0, 8, 16, 24.
__device__ __forceinline__ int nib_to_bytes(uint32_t nib) { return (int)((nib * 0x00204081u) & 0x01010101u); }

// One (list, chunk, 16-row group) unit. rows[]/A must be in LDS already.
// Writes candidates of valid rows into their segments and their counts.
template <bool DEBUG>
__device__ void mfma_unit(const SearchDev& s, int64_t start, int64_t end, const RowInfo* rows,
                          const int8_t* A, uint16_t (*masks)[4], int32_t* rowcnt, float hwk,
                          int32_t* dbg_ip, int32_t* dbg_pc, float* dbg_est, float* dbg_dist,
                          float* dbg_lb, int64_t dbg_base) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  const int dp = s.dp, W = s.W;
  for (int64_t blk = start; blk < end; blk += 64) {
    const bool pvalid = blk + wave * 16 + col < end;
    // lanes past the end read the block's first code (in bounds) and are masked
    const int64_t p = pvalid ? blk + wave * 16 + col : blk;
    const uint32_t keep = pvalid ? 0xFFFFu : 0u;
    i32x4 acc = {0, 0, 0, 0};
    int pcp = 0;
    for (int t = 0; t < W; ++t) {
      const uint32_t bits = (uint32_t)(s.codes[code_word_index(p, t, W)] >> (16 * grp)) & keep;
      pcp += __popc(bits);
      i32x4 b;
      b[0] = nib_to_bytes(bits & 15u);
      b[1] = nib_to_bytes((bits >> 4) & 15u);
      b[2] = nib_to_bytes((bits >> 8) & 15u);
      b[3] = nib_to_bytes((bits >> 12) & 15u);
      // A fragment: row `col`, dimensions 64 t + 16 grp .. +15
      const i32x4 a = *reinterpret_cast<const i32x4*>(A + (size_t)col * dp + t * 64 + grp * 16);
      acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc, 0, 0, 0);
    }
    // popcount of the code: the four lane groups hold its four 16-bit slices
    int pc = pcp + __shfl_xor(pcp, 16, kWave);
    pc += __shfl_xor(pc, 32, kWave);
    const float2 sf = s.sfac[p];
    // acc[i] + qoff * pc = IP of row 4 grp + i with code `col` (the int8 operand
    // holds q_u - qoff, so that B_q = 8 values fit)
    bool pass[4];
    float lbv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * grp + i;
      const RowInfo& ri = rows[row];
      const PairRec& r = ri.rec;
      float dist, lbe;
      const int ipv = acc[i] + s.qoff * pc;
      estimate(r, pair_terms(r, hwk), sf, ipv, pc, dist, lbe);
      const bool live = pvalid && ri.valid;
      const float lb = live ? lbe : __builtin_inff();
      if (DEBUG && row == 0 && live) {
        const int64_t o = p - dbg_base;
        dbg_ip[o] = ipv;
        dbg_pc[o] = pc;
        dbg_est[o] = estimate_est(r, s.fac[p].y, ipv, pc);
        dbg_dist[o] = dist;
        dbg_lb[o] = lb;
      }
      pass[i] = live && lb <= ri.tau;
      lbv[i] = lb;
    }
    if (DEBUG) continue;
    // per-row 16-bit masks of this wave's codes
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t m = __ballot(pass[i]);
      if (lane < 4) masks[4 * lane + i][wave] = (uint16_t)((m >> (16 * lane)) & 0xFFFFu);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!pass[i]) continue;
      const int row = 4 * grp + i;
      uint64_t m64 = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) m64 |= (uint64_t)masks[row][w] << (16 * w);
      const int bit = wave * 16 + col;
      const int before = __popcll(m64 & ((1ull << bit) - 1ull));
      Cand cd;
      cd.pos = (int32_t)p;
      cd.lb = lbv[i];
      s.seg[rows[row].seg_base + rowcnt[row] + before] = cd;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      const int row = threadIdx.x;
      uint64_t m64 = 0;
      for (int w = 0; w < 4; ++w) m64 |= (uint64_t)masks[row][w] << (16 * w);
      rowcnt[row] += __popcll(m64);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int64_t ub64(const int64_t* a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- grouping
// First main-phase chunk of pair g (chunks before it were scanned by phase 0).
__device__ __forceinline__ int first_main_chunk(const SearchDev& s, int64_t q, int r) {
  const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
  return max(0, s.q_p0[q] - choff[r]);
}

__device__ __forceinline__ int pair_chunks(const SearchDev& s, int64_t q, int r) {
  const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
  return choff[r + 1] - choff[r];
}

__global__ void k_group_count(SearchDev s) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= s.nq * s.nprobe) return;
  const int64_t q = g / s.nprobe;
  const int r = (int)(g - q * s.nprobe);
  const PairRec rec = s.pairs[g];
  if (rec.list < 0) return;
  if (first_main_chunk(s, q, r) >= pair_chunks(s, q, r)) return;
  atomicAdd(&s.mf_cnt[rec.list], 1);
}

// Single block: exclusive scans of pair counts and unit counts over lists;
// resets the fill cursors and the work counter.
__global__ __launch_bounds__(1024) void k_group_offsets(SearchDev s) {
  __shared__ int64_t bufp[1024], bufu[1024];
  __shared__ int64_t carry[2];
  if (threadIdx.x == 0) {
    carry[0] = carry[1] = 0;
    s.counters[2] = 0;
  }
  __syncthreads();
  for (int base = 0; base < s.nlist; base += 1024) {
    const int k = base + threadIdx.x;
    int64_t vp = 0, vu = 0;
    if (k < s.nlist) {
      const int c = s.mf_cnt[k];
      const int n = s.list_off[k + 1] - s.list_off[k];
      vp = c;
      vu = c > 0 ? (int64_t)((n + s.chunk - 1) / s.chunk) * ((c + 15) / 16) : 0;
      s.mf_fill[k] = 0;
    }
    bufp[threadIdx.x] = vp;
    bufu[threadIdx.x] = vu;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t tp = threadIdx.x >= (unsigned)o ? bufp[threadIdx.x - o] : 0;
      const int64_t tu = threadIdx.x >= (unsigned)o ? bufu[threadIdx.x - o] : 0;
      __syncthreads();
      bufp[threadIdx.x] += tp;
      bufu[threadIdx.x] += tu;
      __syncthreads();
    }
    if (k < s.nlist) {
      s.mf_pair_off[k] = carry[0] + bufp[threadIdx.x] - vp;
      s.mf_unit_off[k] = carry[1] + bufu[threadIdx.x] - vu;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carry[0] += bufp[1023];
      carry[1] += bufu[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s.mf_pair_off[s.nlist] = carry[0];
    s.mf_unit_off[s.nlist] = carry[1];
  }
}

__global__ void k_group_scatter(SearchDev s) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= s.nq * s.nprobe) return;
  const int64_t q = g / s.nprobe;
  const int r = (int)(g - q * s.nprobe);
  const PairRec rec = s.pairs[g];
  if (rec.list < 0) return;
  if (first_main_chunk(s, q, r) >= pair_chunks(s, q, r)) return;
  const int at = atomicAdd(&s.mf_fill[rec.list], 1);
  s.mf_pairs[s.mf_pair_off[rec.list] + at] = (int32_t)g;
}

// ---------------------------------------------------------------- persistent MFMA scan
__global__ __launch_bounds__(kThreads) void k_scan_mfma(SearchDev s) {
  extern __shared__ __attribute__((aligned(16))) int8_t A[];   // 16 x dp
  __shared__ RowInfo rows[16];
  __shared__ uint16_t masks[16][4];
  __shared__ int32_t rowcnt[16];
  __shared__ int64_t sh_u;
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t total = uniform_i64(s.mf_unit_off[s.nlist]);
  for (;;) {
    if (threadIdx.x == 0) sh_u = (int64_t)atomicAdd(&s.counters[2], 1ull);
    __syncthreads();
    const int64_t u = uniform_i64(sh_u);
    __syncthreads();
    if (u >= total) break;
    const int list = uniform_i32((int)(ub64(s.mf_unit_off, s.nlist + 1, u) - 1));
    const int64_t local = uniform_i64(u - s.mf_unit_off[list]);
    const int cnt = uniform_i32((int)(s.mf_pair_off[list + 1] - s.mf_pair_off[list]));
    const int ngroups = (cnt + 15) / 16;
    const int c = (int)(local / ngroups);
    const int gi = (int)(local - (int64_t)c * ngroups);
    const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
    const int64_t start = lbeg + (int64_t)c * s.chunk;
    const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
    if (threadIdx.x < 16) {
      const int i = threadIdx.x;
      RowInfo ri;
      ri.valid = 0;
      ri.tau = -__builtin_inff();
      ri.seg_base = 0;
      ri.count_slot = -1;
      ri.rec.k1 = ri.rec.k2 = ri.rec.k0 = ri.rec.b = 0.f;
      if (16 * gi + i < cnt) {
        const int64_t g = s.mf_pairs[s.mf_pair_off[list] + 16 * gi + i];
        const int64_t q = g / s.nprobe;
        const int r = (int)(g - q * s.nprobe);
        ri.rec = s.pairs[g];
        if (c >= first_main_chunk(s, q, r)) {
          ri.valid = 1;
          ri.tau = s.tau[q];
          const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
          const int32_t* codeoff = s.pair_codeoff + q * (s.nprobe + 1);
          ri.seg_base = s.off_seg[q] + codeoff[r] + (int64_t)c * s.chunk;
          ri.count_slot = s.off_ch[q] + choff[r] + c;
        }
      }
      rows[i] = ri;
      rowcnt[i] = 0;
    }
    // stage the 16 quantised queries (zero rows for missing pairs)
    for (int idx = threadIdx.x * 16; idx < 16 * s.dp; idx += kThreads * 16) {
      const int i = idx / s.dp, d = idx - i * s.dp;
      i32x4 v = {0, 0, 0, 0};
      if (16 * gi + i < cnt) {
        const int64_t g = s.mf_pairs[s.mf_pair_off[list] + 16 * gi + i];
        v = *reinterpret_cast<const i32x4*>(s.qu8 + g * s.dp + d);
      }
      *reinterpret_cast<i32x4*>(A + idx) = v;
    }
    __syncthreads();
    mfma_unit<false>(s, start, end, rows, A, masks, rowcnt, hwk, nullptr, nullptr, nullptr,
                     nullptr, nullptr, 0);
    if (threadIdx.x < 16 && rows[threadIdx.x].valid) s.seg_count[rows[threadIdx.x].count_slot] = rowcnt[threadIdx.x];
    __syncthreads();
  }
}

// Debug: one caller-given quantised query (row 0) against a whole list.
__global__ __launch_bounds__(kThreads) void k_debug_mfma(SearchDev s, const PairRec* recp,
                                                         const int8_t* qu8, int32_t list, int32_t* ip,
                                                         int32_t* pc, float* est, float* dist,
                                                         float* lb) {
  extern __shared__ __attribute__((aligned(16))) int8_t A[];
  __shared__ RowInfo rows[16];
  __shared__ uint16_t masks[16][4];
  __shared__ int32_t rowcnt[16];
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  if (threadIdx.x < 16) {
    RowInfo ri;
    ri.valid = threadIdx.x == 0;
    ri.tau = __builtin_inff();
    ri.seg_base = 0;
    ri.count_slot = -1;
    ri.rec = *recp;
    rows[threadIdx.x] = ri;
    rowcnt[threadIdx.x] = 0;
  }
  for (int idx = threadIdx.x; idx < 16 * s.dp; idx += kThreads) A[idx] = idx < s.dp ? qu8[idx] : (int8_t)0;
  __syncthreads();
  const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
  const int64_t start = lbeg + (int64_t)blockIdx.x * s.chunk;
  const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
  if (start >= end) return;
  mfma_unit<true>(s, start, end, rows, A, masks, rowcnt, hwk, ip, pc, est, dist, lb, lbeg);
}

// Clears the per-list pair counters (a kernel rather than a memset, so that
// the sequence can be captured in a graph).
__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

bool mfma_available() { return true; }

int scan_mfma_blocks_per_cu(int dp) {
  static int nb = 0, for_dp = -1;
  if (for_dp != dp) {
    int v = 0;
    (void)hipFuncSetAttribute((const void*)k_scan_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)k_scan_mfma, kThreads, (size_t)16 * dp) !=
            hipSuccess ||
        v < 1)
      v = 1;
    nb = v;
    for_dp = dp;
  }
  return nb;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_u32(void* p, int64_t nwords, hipStream_t st) {
  if (nwords <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, st, (uint32_t*)p, nwords);
  return hipGetLastError();
}

hipError_t launch_scan_mfma(const SearchDev& s, int phase, int grid, hipStream_t st) {
  (void)phase;
  const int64_t np = s.nq * s.nprobe;
  const unsigned g1 = (unsigned)((np + 255) / 256);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((s.nlist + 255) / 256)), dim3(256), 0, st,
                     (uint32_t*)s.mf_cnt, (int64_t)s.nlist);
  hipLaunchKernelGGL(k_group_count, dim3(g1), dim3(256), 0, st, s);
  hipLaunchKernelGGL(k_group_offsets, dim3(1), dim3(1024), 0, st, s);
  hipLaunchKernelGGL(k_group_scatter, dim3(g1), dim3(256), 0, st, s);
  const size_t shm = (size_t)16 * s.dp;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_scan_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    (void)hipFuncSetAttribute((const void*)k_debug_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL(k_scan_mfma, dim3(grid), dim3(kThreads), shm, st, s);
  return hipGetLastError();
}

hipError_t launch_debug_mfma(const SearchDev& s, const PairRec* rec, const int8_t* qu8,
                             int32_t list, int nchunks, int32_t* ip, int32_t* pc, float* est,
                             float* dist, float* lb, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  const size_t shm = (size_t)16 * s.dp;
  (void)hipFuncSetAttribute((const void*)k_debug_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  hipLaunchKernelGGL(k_debug_mfma, dim3(nchunks), dim3(kThreads), shm, st, s, rec, qu8, list, ip,
                     pc, est, dist, lb);
  return hipGetLastError();
}

}  // namespace rbq
