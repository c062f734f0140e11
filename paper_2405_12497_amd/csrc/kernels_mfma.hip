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
#include <type_traits>

#include "rbq_internal.hpp"
#include "rbq_runtime.hpp"
#include "scan_code.hpp"

namespace rbq {
namespace {

constexpr int kThreads = 256;
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Ordered "less or equal" of __builtin_amdgcn_fcmpf (the compare's lane mask
// directly; false where either operand is NaN).
constexpr int kCmpOLE = 5;

struct RowInfo {
  PairRec rec;
  PairTerms t;        // the pair's estimator constants (pair_terms / pair_terms_ip)
  float tau;
  int32_t valid;      // 1 when this row's chunk belongs to the scanned phase
  int64_t seg_base;   // first segment slot of (pair, chunk)
  int64_t count_slot; // seg_count index of (pair, chunk)
};

// 4 bits -> 4 bytes of 0/1: the nibble's bits land on bits 0, 8, 16, 24.
__device__ __forceinline__ int nib_to_bytes(uint32_t nib) { return (int)((nib * 0x00204081u) & 0x01010101u); }
__device__ __forceinline__ uint32_t nib_to_bytes_u(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }

// Masked expansion of the wave-unit int8 scan (B_q <= 4). Each block of 128
// dimensions takes two K-steps; lane group g reads the 32 code bits w of
// dimensions 32 g .. 32 g + 31 of the block (half g & 1 of code word
// 2 j + (g >> 1)). w & (0x01010101 << m) and (w >> 4) & (0x01010101 << m),
// m = 0..3, are the B dwords of the two K-steps: byte b of dword m holds bit
// 8 b + m (resp. 8 b + 4 + m) of w times 2^m, one AND per dword. The query
// side carries the matching dimension times 2^(3 - m) (at most 15 * 8 = 120),
// so every product is 8 q_u x_b and the accumulator holds 8 <x_b, q_u>
// exactly. scaled_cols returns, for rows r0..r3 of four bytes, the dwords
// whose byte b is byte m of r_b, shifted left by 3 - m (bytewise exact:
// bytes <= 15).
__device__ __forceinline__ i32x4 scaled_cols(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3) {
  const uint32_t lo01 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);   // r0.0 r1.0 r0.1 r1.1
  const uint32_t hi01 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);   // r0.2 r1.2 r0.3 r1.3
  const uint32_t lo23 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
  i32x4 v;
  v[0] = (int)(__builtin_amdgcn_perm(lo23, lo01, 0x05040100u) << 3);
  v[1] = (int)(__builtin_amdgcn_perm(lo23, lo01, 0x07060302u) << 2);
  v[2] = (int)(__builtin_amdgcn_perm(hi23, hi01, 0x05040100u) << 1);
  v[3] = (int)__builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
  return v;
}

// Masked expansion of the wave-unit FP8 x FP4 scan (B_q <= 4). The B dwords
// of a 128-dimension block are w & 0x11111111, w & 0x22222222,
// w & 0x44444444 and (w >> 1) & 0x44444444: nibble n of dword m holds bit
// 4 n + m of the lane group's 32 code bits as E2M1 0.5, 1, 2 or 2 (so B
// nibble e = 8 m + n, which is k = 32 g + e, carries dimension
// 32 g + 4 n + m of the block). The FP8 query side carries, for that k, the
// dimension times 2, 1, 1/2 or 1/2: every product is q_u x_b and the FP32
// sum is <x_b, q_u> exactly.
// fp8_scaled: four bytes q (0..15) -> E4M3 codes of 2 q (cls 0), q (1) or
// q / 2 (2), exact: a byte lookup for q < 8 and code = offset + q above.
__device__ __forceinline__ uint32_t fp8_scaled(uint32_t q, int cls) {
  const uint32_t t0 = cls == 0 ? 0x4C484000u : cls == 1 ? 0x44403800u : 0x3C383000u;
  const uint32_t t1 = cls == 0 ? 0x56545250u : cls == 1 ? 0x4E4C4A48u : 0x46444240u;
  const uint32_t off = cls == 0 ? 0x50505050u : cls == 1 ? 0x48484848u : 0x40404040u;
  const uint32_t lo = __builtin_amdgcn_perm(t1, t0, q & 0x07070707u);
  const uint32_t mask = ((q & 0x08080808u) >> 3) * 0xFFu;
  return ((q + off) & mask) | (lo & ~mask);
}
// Columns r0 = 2 o, r1 = 2 o + 1 of eight dwords d (row n = dword n): the
// bytes of column r0 for n = 0..3, 4..7, then those of column r1.
__device__ __forceinline__ void cols2(const i32x4& x0, const i32x4& x1, int o, uint32_t out[4]) {
  const uint32_t sel = o == 0 ? 0x05010400u : 0x07030602u;
  const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)x0[1], (uint32_t)x0[0], sel);
  const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)x0[3], (uint32_t)x0[2], sel);
  const uint32_t p45 = __builtin_amdgcn_perm((uint32_t)x1[1], (uint32_t)x1[0], sel);
  const uint32_t p67 = __builtin_amdgcn_perm((uint32_t)x1[3], (uint32_t)x1[2], sel);
  out[0] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
  out[1] = __builtin_amdgcn_perm(p67, p45, 0x05040100u);
  out[2] = __builtin_amdgcn_perm(p23, p01, 0x07060302u);
  out[3] = __builtin_amdgcn_perm(p67, p45, 0x07060302u);
}

// FP8 (E4M3, OCP: bias 7) encodings of the integers 0..15, all exact: the
// query operand of the FP8 x FP4 contraction (B_q <= 4).
__constant__ uint8_t kFp8Int[16] = {0x00, 0x38, 0x40, 0x44, 0x48, 0x4A, 0x4C, 0x4E,
                                    0x50, 0x51, 0x52, 0x53, 0x54, 0x55, 0x56, 0x57};

// 8 code bits -> 8 FP4 (E2M1) values 0 or 1.0 (0b0010) in one dword. The
// nibbles come out in the order of dimensions 0, 4, 1, 5, 2, 6, 3, 7 of the
// byte.
__device__ __forceinline__ int bits_to_fp4x8(uint32_t x) {
  const uint32_t lo = (uint32_t)nib_to_bytes_u(x & 15u), hi = (uint32_t)nib_to_bytes_u((x >> 4) & 15u);
  return (int)((lo | (hi << 4)) << 1);
}

// Operand layouts of v_mfma_scale_f32_16x16x128_f8f6f4 (FP8 A, FP4 B), as
// measured on gfx950: lane group g of the B operand holds the 32 values
// k = 32 g .. 32 g + 31 (nibble e is k = 32 g + e), while lane group g of the
// A operand holds k = 16 g .. 16 g + 15 in bytes 0..15 and k = 64 + 16 g ..
// 64 + 16 g + 15 in bytes 16..31. The B side carries the code bits of
// dimensions 128 t + 32 g .. +31 in the nibble order of bits_to_fp4x8, so the
// query byte at A position x (0..127 within a 128-dimension block) must be the
// dimension that B's k(x) holds: k(x) = 16 (x / 32) + x % 32 for x % 32 < 16,
// else 64 + 16 (x / 32) + x % 32 - 16. A group of 8 consecutive positions
// maps to the 8 dimensions starting at k(x) rounded down to 8, in the nibble order.
// Wait states between the last scaled FP8 x FP4 MFMA of a code block and the
// first read of its result. The compiler's own distance for this mixed-format
// instruction (about 12) returned wrong sums on gfx950 once nothing else sat
// between the product and the read. The accumulator passes through the wait
// (in the accumulation registers the product wrote), so the product comes
// before it and every read of the result after it.
__device__ __forceinline__ void f4_result_wait(f32x4& acc) {
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(acc));
}

__device__ __forceinline__ int f4_src_dim(int d) {
  const int x = d & 127, g = x >> 5, e = x & 31;
  return (d & ~127) + (e < 16 ? 16 * g + e : 64 + 16 * g + (e - 16));
}

// One (list, chunk, RG x 16-row group) unit. rows[], rg_live[] and A must be
// in LDS already. Each wave takes 16 codes of every 64-code block, expands
// their bits once per code word and multiplies them against the RG row groups
// (one MFMA each; row groups without a live row are skipped), then writes the
// candidates of valid rows into their segments and their counts.
// F4: the query rows in LDS are FP8 codes placed by f4_src_dim and in the
// nibble order of bits_to_fp4x8, each row padded to a multiple of 128
// dimensions, and every v_mfma_scale_f32_16x16x128_f8f6f4 takes 128 dimensions
// (two code words) of 16 codes against 16 query rows; FP32 accumulation of
// integer products below 16 over at most 4096 dimensions is exact, so the
// inner products are those of the int8 contraction bit for bit.
template <bool DEBUG, bool F4, int WS, int RG>
__device__ void mfma_unit(const SearchDev& s, int64_t start, int64_t end, const RowInfo* rows,
                          const int32_t* rg_live, const int8_t* A, uint16_t (*masks)[4], int32_t* rowcnt,
                          int32_t* dbg_ip, int32_t* dbg_pc, float* dbg_est, float* dbg_dist,
                          float* dbg_lb, int64_t dbg_base) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  const int dp = s.dp, W = s.W;
  const int dpa = F4 ? (dp + 127) / 128 * 128 : dp;
  bool hl[RG];
#pragma unroll
  for (int h = 0; h < RG; ++h) hl[h] = uniform_i32(rg_live[h]) != 0;
  for (int64_t blk = start; blk < end; blk += 64) {
    const bool pvalid = blk + wave * 16 + col < end;
    // lanes past the end read the block's first code (in bounds) and are masked
    const int64_t p = pvalid ? blk + wave * 16 + col : blk;
    const uint32_t keep = pvalid ? 0xFFFFu : 0u;
    i32x4 acc[RG];
#pragma unroll
    for (int h = 0; h < RG; ++h) acc[h] = i32x4{0, 0, 0, 0};
    int pcp = 0;
    if constexpr (F4) {
      // lane group grp: dimensions 128 t2 + 32 grp .. +31, half (grp & 1) of
      // word 2 t2 + (grp >> 1); every word read is issued before the first product
      const uint32_t keep32 = pvalid ? 0xFFFFFFFFu : 0u;
      const uint32_t* c32 = reinterpret_cast<const uint32_t*>(s.codes);
      f32x4 accf[RG];
#pragma unroll
      for (int h = 0; h < RG; ++h) accf[h] = f32x4{0.f, 0.f, 0.f, 0.f};
      auto step = [&](uint32_t bits, int t2) {
        pcp += __popc(bits);
        i32x8 b = {bits_to_fp4x8(bits & 0xFFu), bits_to_fp4x8((bits >> 8) & 0xFFu),
                   bits_to_fp4x8((bits >> 16) & 0xFFu), bits_to_fp4x8(bits >> 24), 0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < RG; ++h) {
          if (!hl[h]) continue;
          const i32x8 a = *reinterpret_cast<const i32x8*>(A + (size_t)(16 * h + col) * dpa + t2 * 128 + grp * 32);
          // formats: A FP8 E4M3 (0), B FP4 E2M1 (4); E8M0 scales 127 = 2^0
          accf[h] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, accf[h], 0, 4, 0, 127, 0, 127);
        }
      };
      auto load = [&](int t2) -> uint32_t {
        const int w = 2 * t2 + (grp >> 1);
        const uint32_t v = c32[2 * code_word_index(p, min(w, W - 1), W) + (grp & 1)];
        return w < W ? v & keep32 : 0u;
      };
      if constexpr (WS > 0) {
        constexpr int T2 = (WS + 1) / 2;
        uint32_t bw[T2];
#pragma unroll
        for (int t2 = 0; t2 < T2; ++t2) bw[t2] = load(t2);
#pragma unroll
        for (int t2 = 0; t2 < T2; ++t2) step(bw[t2], t2);
      } else {
        const int T2 = (W + 1) / 2;
        for (int t0 = 0; t0 < T2; t0 += 4) {
          uint32_t bw[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) bw[j] = load(min(t0 + j, T2 - 1));
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (t0 + j < T2) step(bw[j], t0 + j);
        }
      }
#pragma unroll
      for (int h = 0; h < RG; ++h) {
        f4_result_wait(accf[h]);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[h][i] = (int)accf[h][i];
      }
    } else {
      // the lane's 16-bit slice (dimensions 64 t + 16 grp .. +15) of each code
      // word; every word read is issued before the first product
      const uint16_t* c16 = reinterpret_cast<const uint16_t*>(s.codes);
      auto step = [&](uint32_t bits, int t) {
        bits &= keep;
        pcp += __popc(bits);
        i32x4 b;
        b[0] = nib_to_bytes(bits & 15u);
        b[1] = nib_to_bytes((bits >> 4) & 15u);
        b[2] = nib_to_bytes((bits >> 8) & 15u);
        b[3] = nib_to_bytes((bits >> 12) & 15u);
#pragma unroll
        for (int h = 0; h < RG; ++h) {
          if (!hl[h]) continue;
          // A fragment: row 16 h + col, dimensions 64 t + 16 grp .. +15
          const i32x4 a = *reinterpret_cast<const i32x4*>(A + (size_t)(16 * h + col) * dp + t * 64 + grp * 16);
          acc[h] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[h], 0, 0, 0);
        }
      };
      if constexpr (WS > 0) {
        uint32_t bw[WS];
#pragma unroll
        for (int t = 0; t < WS; ++t) bw[t] = c16[4 * code_word_index(p, t, WS) + grp];
#pragma unroll
        for (int t = 0; t < WS; ++t) step(bw[t], t);
      } else {
        for (int t0 = 0; t0 < W; t0 += 4) {
          uint32_t bw[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) bw[j] = c16[4 * code_word_index(p, min(t0 + j, W - 1), W) + grp];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (t0 + j < W) step(bw[j], t0 + j);
        }
      }
    }
    // popcount of the code: the four lane groups hold its four 16-bit slices
    int pc = pcp + __shfl_xor(pcp, 16, kWave);
    pc += __shfl_xor(pc, 32, kWave);
    const float2 sf = s.sfac[p];
    const float ct = s.metric != 0 ? -s.fip[p] : code_term_l2(sf);
    // acc[h][i] + qoff * pc = IP of row 16 h + 4 grp + i with code `col` (the
    // int8 operand holds q_u - qoff, so that B_q = 8 values fit)
    bool pass[RG][4];
    float lbv[RG][4];
#pragma unroll
    for (int h = 0; h < RG; ++h) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pass[h][i] = false;
        lbv[h][i] = __builtin_inff();
        if (!hl[h]) continue;
        const int row = 16 * h + 4 * grp + i;
        const RowInfo& ri = rows[row];
        float d0, l0;
        const int ipv = acc[h][i] + s.qoff * pc;
        est_dl(ri.t, sf, ct, est_y(ri.t, ipv, pc), d0, l0);
        const bool live = pvalid && ri.valid;
        const float lb = live ? l0 + ri.t.pt : __builtin_inff();
        if (DEBUG && row == 0 && live) {
          const int64_t o = p - dbg_base;
          dbg_ip[o] = ipv;
          dbg_pc[o] = pc;
          dbg_est[o] = estimate_est(ri.rec, s.fac[p].y, ipv, pc);
          dbg_dist[o] = d0 + ri.t.pt;
          dbg_lb[o] = lb;
        }
        pass[h][i] = live && l0 <= ri.tau - ri.t.pt;   // the bound test without the pair term
        lbv[h][i] = lb;
      }
    }
    if (DEBUG) continue;
    // per-row 16-bit masks of this wave's codes
#pragma unroll
    for (int h = 0; h < RG; ++h) {
      if (!hl[h]) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint64_t m = __ballot(pass[h][i]);
        if (lane < 4) masks[16 * h + 4 * lane + i][wave] = (uint16_t)((m >> (16 * lane)) & 0xFFFFu);
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < RG; ++h) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (!pass[h][i]) continue;
        const int row = 16 * h + 4 * grp + i;
        uint64_t m64 = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) m64 |= (uint64_t)masks[row][w] << (16 * w);
        const int bit = wave * 16 + col;
        const int before = __popcll(m64 & ((1ull << bit) - 1ull));
        Cand cd;
        cd.pos = (int32_t)p;
        cd.lb = lbv[h][i];
        s.seg[rows[row].seg_base + rowcnt[row] + before] = cd;
      }
    }
    __syncthreads();
    if (threadIdx.x < 16 * RG && rg_live[threadIdx.x >> 4]) {
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
  if (threadIdx.x < kScanSlices) s.counters[kScanSliceCtr + kScanSliceStride * threadIdx.x] = 0;
  __syncthreads();
  for (int base = 0; base < s.nlist; base += 1024) {
    const int k = base + threadIdx.x;
    int64_t vp = 0, vu = 0;
    if (k < s.nlist) {
      const int c = s.mf_cnt[k];
      const int n = s.list_off[k + 1] - s.list_off[k];
      vp = c;
      const int rows = 16 * s.mf_rg;
      vu = c > 0 ? (int64_t)((n + s.chunk - 1) / s.chunk) * ((c + rows - 1) / rows) : 0;
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
// FP8 row of the F4 path from 8 int8 query values (0..15) at a time: byte m
// of each group of 8 holds dimension pi(m) of the group, pi = 0, 4, 1, 5, 2, 6, 3, 7.
__device__ __forceinline__ uint64_t fp8_group(uint64_t v) {
  uint64_t out = 0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int src = (m & 1) ? 4 + (m >> 1) : (m >> 1);
    out |= (uint64_t)kFp8Int[(v >> (8 * src)) & 15u] << (8 * m);
  }
  return out;
}

template <bool F4, int WS, int RG>
__global__ __launch_bounds__(kThreads) void k_scan_mfma(SearchDev s) {
  constexpr int R = 16 * RG;
  extern __shared__ __attribute__((aligned(16))) int8_t A[];   // R x dpa
  __shared__ RowInfo rows[R];
  __shared__ uint16_t masks[R][4];
  __shared__ int32_t rowcnt[R];
  __shared__ int32_t rg_live[RG];
  __shared__ int64_t sh_u;
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t total = uniform_i64(s.mf_unit_off[s.nlist]);
  const int dpa = F4 ? (s.dp + 127) / 128 * 128 : s.dp;
  for (;;) {
    if (threadIdx.x == 0) {
      sh_u = (int64_t)atomicAdd(&s.counters[2], 1ull);
#pragma unroll
      for (int h = 0; h < RG; ++h) rg_live[h] = 0;
    }
    __syncthreads();
    const int64_t u = uniform_i64(sh_u);
    __syncthreads();
    if (u >= total) break;
    const int list = uniform_i32((int)(ub64(s.mf_unit_off, s.nlist + 1, u) - 1));
    const int64_t local = uniform_i64(u - s.mf_unit_off[list]);
    const int cnt = uniform_i32((int)(s.mf_pair_off[list + 1] - s.mf_pair_off[list]));
    const int ngroups = (cnt + R - 1) / R;
    const int c = (int)(local / ngroups);
    const int gi = (int)(local - (int64_t)c * ngroups);
    const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
    const int64_t start = lbeg + (int64_t)c * s.chunk;
    const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
    if (threadIdx.x < R) {
      const int i = threadIdx.x;
      RowInfo ri;
      ri.valid = 0;
      ri.tau = -__builtin_inff();
      ri.seg_base = 0;
      ri.count_slot = -1;
      ri.rec.k1 = ri.rec.k2 = ri.rec.k0 = ri.rec.b = 0.f;
      ri.t.a1 = ri.t.a2 = ri.t.a0 = ri.t.pt = ri.t.coefh = 0.f;
      if (R * gi + i < cnt) {
        const int64_t g = s.mf_pairs[s.mf_pair_off[list] + R * gi + i];
        const int64_t q = g / s.nprobe;
        const int r = (int)(g - q * s.nprobe);
        ri.rec = s.pairs[g];
        ri.t = s.metric != 0 ? pair_terms_ip(ri.rec, hwk, s.pair_pt[g]) : pair_terms(ri.rec, hwk);
        if (c >= first_main_chunk(s, q, r)) {
          ri.valid = 1;
          ri.tau = s.tau[q];
          const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
          const int32_t* codeoff = s.pair_codeoff + q * (s.nprobe + 1);
          ri.seg_base = s.off_seg[q] + codeoff[r] + (int64_t)c * s.chunk;
          ri.count_slot = s.off_ch[q] + choff[r] + c;
          rg_live[i >> 4] = 1;
        }
      }
      rows[i] = ri;
      rowcnt[i] = 0;
    }
    // stage the R quantised queries (zero rows for missing pairs)
    if constexpr (F4) {   // FP8, rows padded to a multiple of 128 dimensions
      for (int idx = threadIdx.x * 8; idx < R * dpa; idx += kThreads * 8) {
        const int i = idx / dpa, d = idx - i * dpa;
        uint64_t v = 0;
        const int src = f4_src_dim(d);
        if (R * gi + i < cnt && src < s.dp) {
          const int64_t g = s.mf_pairs[s.mf_pair_off[list] + R * gi + i];
          v = fp8_group(*reinterpret_cast<const uint64_t*>(s.qu8 + g * s.dp + src));
        }
        *reinterpret_cast<uint64_t*>(A + idx) = v;
      }
    } else {
      for (int idx = threadIdx.x * 16; idx < R * s.dp; idx += kThreads * 16) {
        const int i = idx / s.dp, d = idx - i * s.dp;
        i32x4 v = {0, 0, 0, 0};
        if (R * gi + i < cnt) {
          const int64_t g = s.mf_pairs[s.mf_pair_off[list] + R * gi + i];
          v = *reinterpret_cast<const i32x4*>(s.qu8 + g * s.dp + d);
        }
        *reinterpret_cast<i32x4*>(A + idx) = v;
      }
    }
    __syncthreads();
    mfma_unit<false, F4, WS, RG>(s, start, end, rows, rg_live, A, masks, rowcnt, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, 0);
    if (threadIdx.x < R && rows[threadIdx.x].valid) s.seg_count[rows[threadIdx.x].count_slot] = rowcnt[threadIdx.x];
    __syncthreads();
  }
}

// Debug: one caller-given quantised query (row 0) against a whole list, with
// the kernel instantiation the search uses for this code width.
template <bool F4, int WS, int RG>
__global__ __launch_bounds__(kThreads) void k_debug_mfma(SearchDev s, const PairRec* recp,
                                                         const int8_t* qu8, int32_t list, int32_t* ip,
                                                         int32_t* pc, float* est, float* dist,
                                                         float* lb) {
  constexpr int R = 16 * RG;
  extern __shared__ __attribute__((aligned(16))) int8_t A[];
  __shared__ RowInfo rows[R];
  __shared__ uint16_t masks[R][4];
  __shared__ int32_t rowcnt[R];
  __shared__ int32_t rg_live[RG];
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int dpa = F4 ? (s.dp + 127) / 128 * 128 : s.dp;
  if (threadIdx.x < R) {
    RowInfo ri;
    ri.valid = threadIdx.x == 0;
    ri.tau = __builtin_inff();
    ri.seg_base = 0;
    ri.count_slot = -1;
    ri.rec = *recp;
    ri.t = s.metric != 0 ? pair_terms_ip(ri.rec, hwk, s.pair_pt[0]) : pair_terms(ri.rec, hwk);
    rows[threadIdx.x] = ri;
    rowcnt[threadIdx.x] = 0;
  }
  if (threadIdx.x < RG) rg_live[threadIdx.x] = threadIdx.x == 0;
  if constexpr (F4) {
    for (int idx = threadIdx.x * 8; idx < R * dpa; idx += kThreads * 8)
      *reinterpret_cast<uint64_t*>(A + idx) =
          idx < dpa && f4_src_dim(idx) < s.dp ? fp8_group(*reinterpret_cast<const uint64_t*>(qu8 + f4_src_dim(idx))) : 0ull;
  } else {
    for (int idx = threadIdx.x; idx < R * s.dp; idx += kThreads) A[idx] = idx < s.dp ? qu8[idx] : (int8_t)0;
  }
  __syncthreads();
  const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
  const int64_t start = lbeg + (int64_t)blockIdx.x * s.chunk;
  const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
  if (start >= end) return;
  mfma_unit<true, F4, WS, RG>(s, start, end, rows, rg_live, A, masks, rowcnt, ip, pc, est, dist, lb, lbeg);
}

// ---------------------------------------------------------------- wave-unit MFMA scan
// The same work units (list, chunk, group of R = 16 RG pairs), each taken by a
// single wave: the wave keeps its R query rows' MFMA fragments in registers
// for the whole unit (no LDS traffic per code block), counts each row's
// candidates in registers and places them with ballots alone, so no unit
// needs a block barrier. Only the rows' estimator constants sit in LDS, in the
// wave's own slice. Widths up to 16 words (the fragments of 16 RG rows must
// fit in registers); wider codes use the block kernel above.

// The list holding unit u: the largest l < n with off[l] <= u, by a 64-way
// search (three rounds of loads for 16,384 lists).
__device__ __forceinline__ int wave_find_list(const int64_t* __restrict__ off, int n, int64_t u) {
  int lo = 0, hi = n;   // off[lo] <= u, and the list is in [lo, hi)
  const int lane = lane_id();
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int idx = lo + lane * step;
    const bool ok = idx < hi && off[min(idx, n - 1)] <= u;
    const uint64_t m = __ballot(ok);
    const int j = 63 - __clzll((long long)m);   // lane 0 always holds (off[lo] <= u)
    lo = uniform_i32(lo + j * step);
    hi = min(hi, lo + step);
  }
  return lo;
}

// One unit on one wave. rows: the wave's R row records (LDS); g: lane i < R
// holds its row's pair id (-1: none), whose quantised query is row g of `qbase`
// (dp bytes per row). Counts and candidates as mfma_unit.
template <bool DEBUG, bool F4, int WS, int RG>
__device__ void mfma_wave_unit(const SearchDev& s, int64_t start, int64_t end, const RowInfo* rows, int g,
                               const int8_t* __restrict__ qbase, int32_t* dbg_ip, int32_t* dbg_pc,
                               float* dbg_est, float* dbg_dist, float* dbg_lb, int64_t dbg_base) {
  static_assert(WS >= 1 && WS <= 16, "fragments held in registers");
  const int lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  const int dp = s.dp, W = s.W;
  constexpr int T2 = (WS + 1) / 2;
  constexpr int NA = F4 ? T2 : 2 * T2;   // MFMA steps per code (int8: two per 128 dimensions)
  // query fragments of rows 16 h + col: int8 dims 64 t + 16 grp .. +15, or
  // FP8 positions 128 t2 + 32 grp .. +31 (dimensions by f4_src_dim)
  typedef typename std::conditional<F4, i32x8, i32x4>::type AFrag;
  AFrag a[RG][NA];
#pragma unroll
  for (int h = 0; h < RG; ++h) {
    const int gh = __shfl(g, 16 * h + col, kWave);
    const int8_t* qr = qbase + (int64_t)max(gh, 0) * dp;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      if constexpr (F4) {
        // masked FP4 expansion: lane group grp = 2 h2 + o holds, in bytes
        // 8 b + n (b = 0..3), dimension 128 t + 64 (b >> 1) + 32 h2 + 4 n +
        // 2 o + (b & 1) (column 2 o + (b & 1) of a 32-dimension window), times
        // 2 (o = 0, b even), 1 (o = 0, b odd) or 1/2 (o = 1); zero past the row
        const int h2 = grp >> 1, o = grp & 1;
        const int w0 = 128 * t + 32 * h2, w1 = w0 + 64;
        i32x4 x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0}, y0 = {0, 0, 0, 0}, y1 = {0, 0, 0, 0};
        if (gh >= 0 && w0 < dp) {
          x0 = *reinterpret_cast<const i32x4*>(qr + w0);
          x1 = *reinterpret_cast<const i32x4*>(qr + w0 + 16);
        }
        if (gh >= 0 && w1 < dp) {
          y0 = *reinterpret_cast<const i32x4*>(qr + w1);
          y1 = *reinterpret_cast<const i32x4*>(qr + w1 + 16);
        }
        uint32_t cx[4], cy[4];
        cols2(x0, x1, o, cx);
        cols2(y0, y1, o, cy);
        const int c0 = o == 0 ? 0 : 2, c1 = o == 0 ? 1 : 2;   // scale class of columns 2 o and 2 o + 1
        i32x8 v;
        v[0] = (int)fp8_scaled(cx[0], c0);
        v[1] = (int)fp8_scaled(cx[1], c0);
        v[2] = (int)fp8_scaled(cx[2], c1);
        v[3] = (int)fp8_scaled(cx[3], c1);
        v[4] = (int)fp8_scaled(cy[0], c0);
        v[5] = (int)fp8_scaled(cy[1], c0);
        v[6] = (int)fp8_scaled(cy[2], c1);
        v[7] = (int)fp8_scaled(cy[3], c1);
        a[h][t] = v;
      } else if (t % 2 == 0) {
        // int8: K-steps t and t + 1 of the masked expansion, dimensions
        // 64 t + 32 grp .. +31 (zero past the row)
        const int d0 = 64 * t + 32 * grp;
        i32x4 l0 = {0, 0, 0, 0}, l1 = {0, 0, 0, 0};
        if (gh >= 0 && d0 < dp) {
          l0 = *reinterpret_cast<const i32x4*>(qr + d0);
          l1 = *reinterpret_cast<const i32x4*>(qr + d0 + 16);
        }
        a[h][t] = scaled_cols((uint32_t)l0[0], (uint32_t)l0[2], (uint32_t)l1[0], (uint32_t)l1[2]);
        a[h][t + 1] = scaled_cols((uint32_t)l0[1], (uint32_t)l0[3], (uint32_t)l1[1], (uint32_t)l1[3]);
      }
    }
  }
  bool hl[RG];   // row group with a live row (wave-uniform)
#pragma unroll
  for (int h = 0; h < RG; ++h) {
    const bool mine = lane < 16 && rows[16 * h + lane].valid;
    hl[h] = __ballot(mine) != 0ull;
  }
  int cnt[RG][4];
#pragma unroll
  for (int h = 0; h < RG; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) cnt[h][i] = 0;
  // Code words of 16 codes, the next block's in flight while this one
  // computes, addressed from the unit's first 64-code row with 32-bit offsets:
  // unit position x (the start at o0) has word w at ((x >> 6) W + w) 64 + (x & 63).
  const int n = (int)(end - start);
  const int o0 = (int)(start & 63);
  const int64_t row0 = start >> 6;
  constexpr int NB = T2;   // registers of code bits per block
  // wave-uniform bases (the unit's first code row, its first factors) and
  // per-lane 32-bit byte offsets, so the loads take the scalar-base form
  const char* cbase = reinterpret_cast<const char*>(s.codes) + (size_t)row0 * WS * 512;
  const char* sbase = reinterpret_cast<const char*>(s.sfac + start);
  const char* fbase = s.metric != 0 ? reinterpret_cast<const char*>(s.fip + start) : nullptr;
  // this lane's half (grp & 1) of word 2 t + (grp >> 1)
  const uint32_t lane_b = 4u * (128u * (uint32_t)(grp >> 1) + (uint32_t)(grp & 1));
  // the block at unit offset rel: this lane's code (clamped into the unit; the
  // columns past its end are never used), its bits and its scan factors (and
  // inner-product term)
  auto load_block = [&](int rel, uint32_t* bw, float2& sf, float& fi) {
    const uint32_t r = (uint32_t)min(rel + col, n - 1);
    const uint32_t x = (uint32_t)o0 + r;
    // word 0 of position x (the wave-unit kernels have W == WS), in bytes
    const uint32_t wb = 8u * ((x >> 6) * (uint32_t)WS * 64u + (x & 63u));
    // 32 bits of dimensions 128 t + 32 grp .. +31: half grp & 1 of word
    // 2 t + (grp >> 1) (for an odd width, zero past the code's last word)
#pragma unroll
    for (int t = 0; t < T2; ++t) {
      if (WS % 2 == 0 || t + 1 < T2) {
        bw[t] = *reinterpret_cast<const uint32_t*>(cbase + (wb + lane_b + 1024u * (uint32_t)t));
      } else {
        const uint32_t v =
            *reinterpret_cast<const uint32_t*>(cbase + (wb + 512u * (uint32_t)(WS - 1) + 4u * (uint32_t)(grp & 1)));
        bw[t] = grp < 2 ? v : 0u;
      }
    }
    sf = *reinterpret_cast<const float2*>(sbase + 8u * r);
    fi = fbase != nullptr ? *reinterpret_cast<const float*>(fbase + 4u * r) : 0.f;
  };
  if constexpr (RG == 1) {
    if (!hl[0]) return;   // no live row in the unit
  }
  // this lane's rows' estimator constants in registers: y = a1 acc + a2 pc +
  // a0 (the int8 accumulator is 8 <x_b, q_u>, so its a1 is divided by 8,
  // exactly), coefh, and the threshold tau - pt of the bound test (-inf for
  // rows outside the scanned phase, so the loop reads it without a branch);
  // their validity for the parity export
  bool rval[RG][4];
  float ra1[RG][4], ra2[RG][4], ra0[RG][4], rch[RG][4], rtp[RG][4];
#pragma unroll
  for (int h = 0; h < RG; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const RowInfo& ri = rows[16 * h + 4 * grp + i];
      rval[h][i] = ri.valid != 0;
      ra1[h][i] = F4 ? ri.t.a1 : ri.t.a1 * 0.125f;
      ra2[h][i] = ri.t.a2;
      ra0[h][i] = ri.t.a0;
      rch[h][i] = ri.t.coefh;
      rtp[h][i] = ri.valid != 0 ? ri.tau - ri.t.pt : -__builtin_inff();
    }
  // one block of 16 codes at unit offset rb, from its loaded bits and factors
  auto block = [&](int rb, const uint32_t* bw, float2 sf, float fi) {
    // a lane past the end computes on the last code of the unit: its column's
    // results (and that code's popcount) are never used
    const bool pvalid = rb + col < n;
    const int64_t p = start + (pvalid ? rb + col : rb);
    i32x4 acc[RG];
    int pcp = 0;
    if constexpr (F4) {
      f32x4 accf[RG];
#pragma unroll
      for (int h = 0; h < RG; ++h) accf[h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < T2; ++t) {
        const uint32_t bits = bw[t];
        pcp += __popc(bits);
        const i32x8 b = {(int)(bits & 0x11111111u), (int)(bits & 0x22222222u), (int)(bits & 0x44444444u),
                         (int)((bits >> 1) & 0x44444444u), 0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < RG; ++h)
          if (RG == 1 || hl[h])
            accf[h] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[h][t], b, accf[h], 0, 4, 0, 127, 0, 127);
      }
#pragma unroll
      for (int h = 0; h < RG; ++h) {
        f4_result_wait(accf[h]);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[h][i] = (int)accf[h][i];
      }
    } else {
#pragma unroll
      for (int h = 0; h < RG; ++h) acc[h] = i32x4{0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < T2; ++j) {
        const uint32_t w = bw[j], w4 = w >> 4;
        pcp += __popc(w);
        const i32x4 b0 = {(int)(w & 0x01010101u), (int)(w & 0x02020202u), (int)(w & 0x04040404u),
                          (int)(w & 0x08080808u)};
        const i32x4 b1 = {(int)(w4 & 0x01010101u), (int)(w4 & 0x02020202u), (int)(w4 & 0x04040404u),
                          (int)(w4 & 0x08080808u)};
#pragma unroll
        for (int h = 0; h < RG; ++h)
          if (RG == 1 || hl[h]) {
            acc[h] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[h][2 * j], b0, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[h][2 * j + 1], b1, acc[h], 0, 0, 0);
          }
      }
    }
    int pc = pcp + __shfl_xor(pcp, 16, kWave);
    pc += __shfl_xor(pc, 32, kWave);
    const float pcf = (float)pc;
    const uint64_t pvmask = __builtin_amdgcn_ballot_w64(pvalid);
    // lanes past the end hold the last code's factors; their rows do not pass
    const float ct = s.metric != 0 ? -fi : code_term_l2(sf);
#pragma unroll
    for (int h = 0; h < RG; ++h) {
      if (RG > 1 && !hl[h]) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * h + 4 * grp + i;
        // the same y, d0 and l0 as est_y / est_dl on the integer inner product
        const float y = fmaf(ra1[h][i], (float)acc[h][i], fmaf(ra2[h][i], pcf, ra0[h][i]));
        const float d0 = fmaf(sf.x, y, ct);
        const float l0 = fmaf(rch[h][i], sf.y, d0);
        if constexpr (DEBUG) {
          if (row == 0 && pvalid && rval[h][i]) {
            const RowInfo& ri = rows[row];
            const int ipv = F4 ? acc[h][i] : acc[h][i] >> 3;   // B_q <= 4 here: q_u - qoff = q_u
            const int64_t o = p - dbg_base;
            dbg_ip[o] = ipv;
            dbg_pc[o] = pc;
            dbg_est[o] = estimate_est(ri.rec, s.fac[p].y, ipv, pc);
            dbg_dist[o] = d0 + ri.t.pt;
            dbg_lb[o] = l0 + ri.t.pt;
          }
        } else {
          // this row group's 16 codes: bits 16 grp .. +15 of the ballot (most
          // blocks have no candidate at all)
          const uint64_t m = __builtin_amdgcn_fcmpf(l0, rtp[h][i], kCmpOLE) & pvmask;
          if (m != 0ull) {
            const uint32_t mine = (uint32_t)(m >> (16 * grp)) & 0xFFFFu;
            if ((mine >> col) & 1u) {
              const RowInfo& ri = rows[row];
              Cand cd;
              cd.pos = (int32_t)p;
              cd.lb = l0 + ri.t.pt;
              s.seg[ri.seg_base + cnt[h][i] + __popc(mine & ((1u << col) - 1u))] = cd;
            }
            cnt[h][i] += __popc(mine);
          }
        }
      }
    }
  };
  // three register sets in turn: the next two blocks' loads are in flight
  // while this one computes (blocks past the end reload the last code)
  uint32_t bA[NB], bB[NB], bC[NB];
  float2 sA, sB, sC;
  float fA, fB, fC;
  load_block(0, bA, sA, fA);
  load_block(min(16, n - 1), bB, sB, fB);
  for (int rb = 0; rb < n; rb += 48) {
    load_block(min(rb + 32, n - 1), bC, sC, fC);
    block(rb, bA, sA, fA);
    if (rb + 16 >= n) break;
    load_block(min(rb + 48, n - 1), bA, sA, fA);
    block(rb + 16, bB, sB, fB);
    if (rb + 32 >= n) break;
    load_block(min(rb + 64, n - 1), bB, sB, fB);
    block(rb + 32, bC, sC, fC);
  }
  if constexpr (!DEBUG) {
    if (col == 0) {
#pragma unroll
      for (int h = 0; h < RG; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const RowInfo& ri = rows[16 * h + 4 * grp + i];
          if (ri.valid) s.seg_count[ri.count_slot] = cnt[h][i];
        }
    }
  }
}

template <bool F4, int WS, int RG>
__global__ __launch_bounds__(kThreads) void k_scan_mfma_w(SearchDev s) {
  constexpr int R = 16 * RG;
  __shared__ RowInfo rows_all[kThreads / kWave][R];
  const int lane = lane_id();
  RowInfo* rows = rows_all[threadIdx.x / kWave];
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  const int64_t total = uniform_i64(s.mf_unit_off[s.nlist]);
  // The units (ordered by list, then chunk, then row group) are cut into
  // kScanSlices contiguous slices; a block starts on the slice of its XCD
  // (workgroups go to the XCDs in turn), so the row groups of one code chunk
  // run on one XCD and share its L2, then moves on to the other slices.
  const int x0 = (int)(blockIdx.x % kScanSlices);
  for (int j = 0; j < kScanSlices; ++j) {
    const int x = (x0 + j) % kScanSlices;
    const int64_t hi = total * (x + 1) / kScanSlices;
    const int64_t lo = total * x / kScanSlices;
    unsigned long long* ctr = s.counters + kScanSliceCtr + kScanSliceStride * x;
    for (;;) {
      unsigned long long cl = 0;
      if (lane == 0) cl = atomicAdd(ctr, 1ull);
      const int64_t u = lo + uniform_i64((int64_t)cl);   // lane 0's claim (every lane is active)
      if (u >= hi) break;
      const int list = wave_find_list(s.mf_unit_off, s.nlist, u);
      const int64_t local = uniform_i64(u - s.mf_unit_off[list]);
      const int cnt = uniform_i32((int)(s.mf_pair_off[list + 1] - s.mf_pair_off[list]));
      const int ngroups = (cnt + R - 1) / R;
      const int c = (int)(local / ngroups);
      const int gi = (int)(local - (int64_t)c * ngroups);
      const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
      const int64_t start = lbeg + (int64_t)c * s.chunk;
      const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
      int g = -1;
      if (lane < R) {
        RowInfo ri;
        ri.valid = 0;
        ri.tau = -__builtin_inff();
        ri.seg_base = 0;
        ri.count_slot = -1;
        ri.rec.k1 = ri.rec.k2 = ri.rec.k0 = ri.rec.b = 0.f;
        ri.t.a1 = ri.t.a2 = ri.t.a0 = ri.t.pt = ri.t.coefh = 0.f;
        if (R * gi + lane < cnt) {
          g = s.mf_pairs[s.mf_pair_off[list] + R * gi + lane];
          const int64_t q = g / s.nprobe;
          const int r = (int)(g - q * s.nprobe);
          ri.rec = s.pairs[g];
          ri.t = s.metric != 0 ? pair_terms_ip(ri.rec, hwk, s.pair_pt[g]) : pair_terms(ri.rec, hwk);
          if (c >= first_main_chunk(s, q, r)) {
            ri.valid = 1;
            ri.tau = s.tau[q];
            const int32_t* choff = s.pair_choff + q * (s.nprobe + 1);
            const int32_t* codeoff = s.pair_codeoff + q * (s.nprobe + 1);
            ri.seg_base = s.off_seg[q] + codeoff[r] + (int64_t)c * s.chunk;
            ri.count_slot = s.off_ch[q] + choff[r] + c;
          }
        }
        rows[lane] = ri;
      }
      mfma_wave_unit<false, F4, WS, RG>(s, start, end, rows, g, s.qu8, nullptr, nullptr, nullptr, nullptr, nullptr,
                                        0);
    }
  }
}

// Debug: one caller-given quantised query (row 0) against a whole list, one
// wave per chunk, through the wave-unit code the search runs.
template <bool F4, int WS, int RG>
__global__ __launch_bounds__(kWave) void k_debug_mfma_w(SearchDev s, const PairRec* recp, const int8_t* qu8,
                                                        int32_t list, int32_t* ip, int32_t* pc, float* est,
                                                        float* dist, float* lb) {
  constexpr int R = 16 * RG;
  __shared__ RowInfo rows[R];
  const int lane = lane_id();
  const float hwk = s.eps0 / sqrtf((float)(s.dp - 1));
  if (lane < R) {
    RowInfo ri;
    ri.valid = lane == 0;
    ri.tau = __builtin_inff();
    ri.seg_base = 0;
    ri.count_slot = -1;
    ri.rec = *recp;
    ri.t = s.metric != 0 ? pair_terms_ip(ri.rec, hwk, s.pair_pt[0]) : pair_terms(ri.rec, hwk);
    rows[lane] = ri;
  }
  const int64_t lbeg = uniform_i64(s.list_off[list]), lend = uniform_i64(s.list_off[list + 1]);
  const int64_t start = lbeg + (int64_t)blockIdx.x * s.chunk;
  const int64_t end = lend < start + s.chunk ? lend : start + s.chunk;
  if (start >= end) return;
  mfma_wave_unit<true, F4, WS, RG>(s, start, end, rows, lane == 0 ? 0 : -1, qu8, ip, pc, est, dist, lb, lbeg);
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

// Kernels per (code width, row groups): W words of 64 bits, compile-time for
// the common widths (every word read is then issued before the first
// product) and a runtime width otherwise; RG groups of 16 query rows per unit.
template <bool F4, bool DBG>
const void* kernel_for(int W, int rg) {
#define RBQ_MF(WS_, RG_) (DBG ? (const void*)k_debug_mfma<F4, WS_, RG_> : (const void*)k_scan_mfma<F4, WS_, RG_>)
  if (rg == 4) {
    switch (W) {
      case 12: return RBQ_MF(12, 4);
      default: return RBQ_MF(0, 4);
    }
  }
  if (rg == 2) {
    switch (W) {
      case 12: return RBQ_MF(12, 2);
      case 15: return RBQ_MF(15, 2);
      case 16: return RBQ_MF(16, 2);
      default: return RBQ_MF(0, 2);
    }
  }
  switch (W) {
    case 1: return RBQ_MF(1, 1);
    case 2: return RBQ_MF(2, 1);
    case 3: return RBQ_MF(3, 1);
    case 4: return RBQ_MF(4, 1);
    case 8: return RBQ_MF(8, 1);
    case 12: return RBQ_MF(12, 1);
    case 15: return RBQ_MF(15, 1);
    case 16: return RBQ_MF(16, 1);
    default: return RBQ_MF(0, 1);
  }
#undef RBQ_MF
}

// Wave-unit kernels: the query fragments of 16 RG rows in registers, for the
// exact compile-time widths (RG = 2 up to 12 words).
template <bool F4, bool DBG>
const void* wave_kernel_for(int W, int rg) {
#define RBQ_MW(WS_, RG_) (DBG ? (const void*)k_debug_mfma_w<F4, WS_, RG_> : (const void*)k_scan_mfma_w<F4, WS_, RG_>)
  if (rg == 1) {
    switch (W) {
      case 1: return RBQ_MW(1, 1);
      case 2: return RBQ_MW(2, 1);
      case 3: return RBQ_MW(3, 1);
      case 4: return RBQ_MW(4, 1);
      case 8: return RBQ_MW(8, 1);
      case 12: return RBQ_MW(12, 1);
      case 15: return RBQ_MW(15, 1);
      case 16: return RBQ_MW(16, 1);
      default: return nullptr;
    }
  }
  if (rg == 2) {
    switch (W) {
      case 2: return RBQ_MW(2, 2);
      case 4: return RBQ_MW(4, 2);
      case 12: return RBQ_MW(12, 2);
      default: return nullptr;
    }
  }
  return nullptr;
#undef RBQ_MW
}

// The batched scan kernel for (W, rg): the wave-unit form where it exists
// (for the int8 contraction only when B_q <= 4, `narrow`: its masked expansion
// needs query values below 16), else the block form. *wave tells which.
const void* pick_kernel(bool f4, bool dbg, int W, int rg, bool narrow, bool* wave) {
  const void* f = f4 ? (dbg ? wave_kernel_for<true, true>(W, rg) : wave_kernel_for<true, false>(W, rg))
                : !narrow ? nullptr
                          : (dbg ? wave_kernel_for<false, true>(W, rg) : wave_kernel_for<false, false>(W, rg));
  *wave = f != nullptr;
  if (f) return f;
  if (f4) return dbg ? kernel_for<true, true>(W, rg) : kernel_for<true, false>(W, rg);
  return dbg ? kernel_for<false, true>(W, rg) : kernel_for<false, false>(W, rg);
}

int row_bytes(bool f4, int dp) { return f4 ? (dp + 127) / 128 * 128 : dp; }

// LDS for the query tile: at most what a block may hold beyond the kernel's
// static arrays (8 KiB reserved for them).
size_t lds_budget() {
  static size_t lim = 0;
  if (!lim) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 16384)
      lim = (size_t)v - 8192;
    else
      lim = 56 * 1024;
  }
  return lim;
}

void allow_lds(const void* f, size_t bytes) {
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

bool mfma_available() { return true; }

int mfma_row_groups(int dp, bool f4, int want) {
  const size_t rb = (size_t)row_bytes(f4, dp);
  // default one group: with more, every wave re-reads RG query tiles from LDS
  // per 64 codes, and LDS bandwidth, not the MFMA rate, sets the pace
  int rg = want == 1 || want == 2 || want == 4 ? want : 1;
  while (rg > 1 && (size_t)16 * rg * rb > lds_budget()) rg >>= 1;
  return rg;
}

int scan_mfma_blocks_per_cu(int dp, bool f4, int rg, bool narrow) {
  bool wave = false;
  const void* f = pick_kernel(f4, false, dp / 64, rg, narrow, &wave);
  const size_t bytes = wave ? 0 : (size_t)16 * rg * row_bytes(f4, dp);
  if (!wave) allow_lds(f, bytes);
  int v = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, f, kThreads, bytes) != hipSuccess || v < 1) v = 1;
  return v;
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

hipError_t launch_group_mfma(const SearchDev& s, hipStream_t st) {
  const int64_t np = s.nq * s.nprobe;
  const unsigned g1 = (unsigned)((np + 255) / 256);
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((s.nlist + 255) / 256)), dim3(256), 0, st,
                     (uint32_t*)s.mf_cnt, (int64_t)s.nlist);
  hipLaunchKernelGGL(k_group_count, dim3(g1), dim3(256), 0, st, s);
  hipLaunchKernelGGL(k_group_offsets, dim3(1), dim3(1024), 0, st, s);
  hipLaunchKernelGGL(k_group_scatter, dim3(g1), dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_scan_mfma(const SearchDev& s, int phase, int grid, hipStream_t st) {
  (void)phase;
  const bool f4 = s.mfma_f4 != 0;
  bool wave = false;
  const void* f = pick_kernel(f4, false, s.W, s.mf_rg, s.npl == 4, &wave);
  const size_t bytes = wave ? 0 : (size_t)16 * s.mf_rg * row_bytes(f4, s.dp);
  if (!wave) allow_lds(f, bytes);
  void* args[] = {(void*)&s};
  return hipLaunchKernel(f, dim3(grid), dim3(kThreads), args, bytes, st);
}

hipError_t launch_debug_mfma(const SearchDev& s, const PairRec* rec, const int8_t* qu8,
                             int32_t list, int nchunks, int32_t* ip, int32_t* pc, float* est,
                             float* dist, float* lb, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  const bool f4 = s.mfma_f4 != 0;
  bool wave = false;
  const void* f = pick_kernel(f4, true, s.W, s.mf_rg, s.npl == 4, &wave);
  const size_t bytes = wave ? 0 : (size_t)16 * s.mf_rg * row_bytes(f4, s.dp);
  if (!wave) allow_lds(f, bytes);
  void* args[] = {(void*)&s, (void*)&rec, (void*)&qu8, (void*)&list, (void*)&ip, (void*)&pc,
                  (void*)&est, (void*)&dist, (void*)&lb};
  return hipLaunchKernel(f, dim3(nchunks), dim3(wave ? kWave : kThreads), args, bytes, st);
}

}  // namespace rbq
