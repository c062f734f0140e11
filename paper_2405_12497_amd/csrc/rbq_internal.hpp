// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace rbq {

constexpr int kWave = 64;          // CDNA wavefront
// Work counters of the wave-unit MFMA scan: one per slice of its units (one
// slice per XCD), 128 bytes apart, after the 8 general counters.
constexpr int kScanSlices = 8;
constexpr int kScanSliceCtr = 16;
constexpr int kScanSliceStride = 16;
constexpr size_t kCounterBytes = 8 * (kScanSliceCtr + kScanSliceStride * kScanSlices);
constexpr int kMaxK = 256;         // largest k returned by a search
constexpr int kMaxNprobe = 16384;   // the selection of more than 2048 lists sorts them in LDS
constexpr int kMaxNlist = 24576;    // probe selection keeps a query's centroid distances in LDS
constexpr int kMaxCodeBits = 4096;
constexpr int kDefaultChunk = 1024;  // codes per scan work unit
constexpr int kMaxP0 = 2048;       // bootstrap codes per query: boot - 1 + chunk <= kMaxP0
constexpr int kOffQ = 1024;       // queries per block of the query-offset scan
constexpr int kBootCodes = 512;    // bootstrap target: at least this many codes (and k)
constexpr int64_t kSegBudget = 8ll << 30;   // bytes of candidate segments per (sub-)batch

// Bootstrap target for a search with k results and `chunk` codes per unit
// (chunk <= kMaxP0 + 1 - k): a query's bootstrap covers whole chunks until it
// holds >= boot codes, i.e. at most boot - 1 + chunk <= kMaxP0 codes.
inline int boot_codes(int k, int chunk) {
  const int cap = kMaxP0 + 1 - chunk;
  return k > (kBootCodes < cap ? kBootCodes : cap) ? k : (kBootCodes < cap ? kBootCodes : cap);
}

// Per (query, probed list) constants of the quantised query (Sec. 3.3.1-3.3.2).
// <x_bar, q_bar> = k1 * <x_b, q_u> + k2 * popcount(x_b) + k0
struct PairRec {
  float k1, k2, k0;
  float b;        // ||q_r - c||
  float vl;       // v_l
  float delta;    // Delta
  int32_t sq;     // sum of q_u
  int32_t list;   // list id (-1: unused slot)
};

// Rerank candidate written by the scan: position in list order + lower bound.
struct Cand {
  int32_t pos;
  float lb;
};

// Bootstrap entry: estimated distance + list-order position. Entry i of a
// query's bootstrap buffer is its code i, so its segment slot is i.
struct EstEnt {
  float dist;
  int32_t pos;   // list-order position of the code (its slot is the entry's index)
};

struct SeedEnt {
  float dist;
  int32_t id;   // original id (< 2^31), -1 for none
};

// One work unit of a scan phase: at most `chunk` consecutive codes of one
// probed (query, list) pair, with every offset the scan needs precomputed.
struct __attribute__((aligned(16))) UnitDesc {
  int64_t start;       // first code position (list order)
  int64_t g;           // pair index q * nprobe + rank
  int64_t seg;         // candidate-segment slot of the first code
  int64_t qcode;       // the first code's index in the query's probed-code space
  int64_t p0slot;      // bootstrap-buffer slot of the first code
  int64_t count_slot;  // seg_count entry of the unit
  int32_t len;         // codes
  int32_t q;           // query
  int64_t pad;
};

// ------------------------------------------------------------------ device helpers
#if defined(__HIPCC__)

// Wave-wide reductions for full waves (all 64 lanes active). Within each row
// of 16 lanes: DPP quad swaps (xor 1, xor 2), half-row mirror, row mirror —
// plain VALU ops, every lane ends with its row's result; the four row results
// are combined through readlane, so the result is uniform and bit-identical
// in every lane.
template <int kCtrl>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}
template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(dpp_i32<kCtrl>(__float_as_int(v)));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16

template <typename T, typename Op>
__device__ __forceinline__ T row_reduce(T v, Op op) {
  if constexpr (sizeof(T) == 4 && !__is_same(T, int)) {
    v = op(v, dpp_f32<kDppXor1>(v));
    v = op(v, dpp_f32<kDppXor2>(v));
    v = op(v, dpp_f32<kDppHalfMirror>(v));
    v = op(v, dpp_f32<kDppMirror>(v));
  } else {
    v = op(v, dpp_i32<kDppXor1>(v));
    v = op(v, dpp_i32<kDppXor2>(v));
    v = op(v, dpp_i32<kDppHalfMirror>(v));
    v = op(v, dpp_i32<kDppMirror>(v));
  }
  return v;
}
__device__ __forceinline__ float readlane_f32(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ float wave_sum(float v) {
  auto add = [](float a, float b) { return a + b; };
  v = row_reduce(v, add);
  return (readlane_f32(v, 0) + readlane_f32(v, 16)) + (readlane_f32(v, 32) + readlane_f32(v, 48));
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
  auto add = [](int a, int b) { return a + b; };
  v = row_reduce(v, add);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
__device__ __forceinline__ float wave_min(float v) {
  auto mn = [](float a, float b) { return fminf(a, b); };
  v = row_reduce(v, mn);
  return fminf(fminf(readlane_f32(v, 0), readlane_f32(v, 16)), fminf(readlane_f32(v, 32), readlane_f32(v, 48)));
}
__device__ __forceinline__ float wave_max(float v) {
  auto mx = [](float a, float b) { return fmaxf(a, b); };
  v = row_reduce(v, mx);
  return fmaxf(fmaxf(readlane_f32(v, 0), readlane_f32(v, 16)), fmaxf(readlane_f32(v, 32), readlane_f32(v, 48)));
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Value of the first active lane, as a wave-uniform (scalar) value. Every loop
// bound or exit test that encloses cross-lane operations or barriers goes
// through these, so the compiler emits uniform control flow for it (a loop whose
// exit it believes divergent may be split per lane, which strands lanes that
// wait on a cross-lane read).
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float uniform_f32(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Compile-time integer carried as a type, for dispatching a runtime count to
// one of a few unrolled template instances.
template <int N>
struct IntC {
  static constexpr int value = N;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// SplitMix64 output for state x (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The uniforms u_i and u_{i+64} (i % 128 < 64) of a (query, list) pair, in
// [0, 1) with 24 bits: both come from one SplitMix64 output z of draw
// j = (i / 128) * 64 + i % 64, u_i from bits 40..63 and u_{i+64} from bits
// 16..39 (the final xor with z >> 31 reaches bit 32 downwards only).
__device__ __forceinline__ void rounding_u2(uint64_t seed, uint64_t qid, uint32_t list, uint32_t i, float& u0,
                                           float& u1) {
  const uint32_t j = ((i >> 7) << 6) | (i & 63u);
  const uint64_t z = splitmix64(seed ^ ((qid << 40) + ((uint64_t)list << 12) + (uint64_t)j));
  // 24-bit fields from the two 32-bit halves (exact in FP32)
  const uint32_t hi = (uint32_t)(z >> 32), lo = (uint32_t)z;
  u0 = (float)(hi >> 8) * (1.0f / 16777216.0f);
  u1 = (float)(__builtin_amdgcn_alignbit(hi, lo, 16) & 0xFFFFFFu) * (1.0f / 16777216.0f);
}

// Workgroups go to the XCDs in turn (workgroup b to XCD b % 8): this block
// order gives each XCD a contiguous run of the nb blocks (the remainder past
// a multiple of 8 keeps its place), so work on neighbouring items shares one
// L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = nb / kScanSlices;
  if (b >= per * kScanSlices) return b;
  return (b % kScanSlices) * per + b / kScanSlices;
}

// Interleaved code layout: for position p (list order), 64-bit word w lives at
// codes[((p >> 6) * W + w) * 64 + (p & 63)], so word w of 64 consecutive codes
// is one contiguous 512-byte row.
__device__ __forceinline__ size_t code_word_index(int64_t p, int w, int W) {
  return ((size_t)(p >> 6) * W + w) * 64 + (size_t)(p & 63);
}

#endif  // __HIPCC__

// ------------------------------------------------------------------ launchers
// (defined in the .hip files; all take a hipStream_t and return hipError_t of the launch)

// Y[M x N] = (A[M x K] - C[sel[m]]) * B[K x N]   (A row stride lda; B row stride ldb)
// sel == nullptr: no subtraction. FP32 FMA tiles.
hipError_t launch_gemm_f32(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                           const float* B, int64_t ldb, float* Y, int64_t ldy, int64_t M, int N,
                           int K, hipStream_t st);
// Same product with split-BF16 MFMA: Bhi/Blo are [K x N] BF16 (stored as uint16).
hipError_t launch_gemm_bf16x3(const float* A, int64_t lda, const float* sub, const int32_t* sel,
                              const uint16_t* Bhi, const uint16_t* Blo, float* Y, int64_t ldy,
                              int64_t M, int N, int K, hipStream_t st);
// D[b][k] = ||q_b||^2 + cn[k] - 2 <q_b, c_k>, clamped at 0 (Ct is [K x nlist],
// D is [nq x nlist]). When
// centroid_gmin(nq, nlist) holds and gmin is not null, gmin receives the
// minimum of each 16-list group of a row ([nq x ceil(nlist / 64) * 4]; group g
// holds lists 64 (g / 4) + 4 (g % 4) + 16 j + e, j, e < 4).
bool gemm_f32_wide_tile(int64_t M, int N);
inline bool centroid_gmin(int64_t nq, int nlist) { return gemm_f32_wide_tile(nq, nlist); }
// Chi, Clo (optional): the centroids as BF16 hi/lo planes [nlist][dim]; given,
// batches of more than 8 queries take split-BF16 products (hi*hi + hi*lo +
// lo*hi) on the BF16 matrix cores, always with 128-wide tiles (gmin written
// when given).
hipError_t launch_centroid_dist(const float* Q, int64_t nq, int dim, const float* Ct,
                                const float* cn, int nlist, float* D, float* gmin, hipStream_t st,
                                const uint16_t* Chi = nullptr, const uint16_t* Clo = nullptr);
// The FP32 query rotation qrot = Q * P (P is [dim x dp]) and launch_centroid_dist's
// outputs, in one launch when the distances use 128-wide tiles.
hipError_t launch_rotate_centroid(const float* Q, int64_t nq, int dim, const float* P, int dp, float* qrot,
                                  const float* Ct, const float* cn, int nlist, float* D, float* gmin,
                                  hipStream_t st);
// FP64 product of rows with P: Y[M x N] = X[M x K] * P[K x N] (stored as FP32).
hipError_t launch_rotate_f64(const float* X, int64_t M, int K, const double* P, int N, float* Y,
                             hipStream_t st);

// dst[p] = src[ids[p]] (rows of D floats): raw vectors in list order.
hipError_t launch_gather_raw(const float* src, const int64_t* ids, int64_t n, int D, float* dst, hipStream_t st);
hipError_t launch_encode(const float* Y, int64_t m, int W, const float* raw, const float* cent,
                         const int32_t* list_of, int dim, int64_t pos0, uint64_t* codes,
                         float2* fac, hipStream_t st);
hipError_t launch_scan_factors(const float2* fac, int64_t n, float2* sfac, hipStream_t st);

// The nprobe (or nprobe_q[b], at most nprobe) smallest entries of each row of
// D, ties to the lower list id; gmin (optional, read when centroid_gmin holds)
// as written by launch_centroid_dist lets small selections read only the
// groups that can hold them.
hipError_t launch_select_probe(const float* D, const float* gmin, int64_t nq, int nlist, int nprobe,
                               const int32_t* nprobe_q, int32_t* lists, float* dists,
                               hipStream_t st);

// Per query: 1 + the probe rank of the latest-probed list among the lists of
// its k neighbour ids nn[nq x k] (ids < 0 skipped; 0 if none), ranks by (D, list id).
hipError_t launch_probe_need(const float* D, int64_t nq, int nlist, const int64_t* nn, int k, const int32_t* id2list,
                             int64_t n, int32_t* need, hipStream_t st);

struct SearchDev {
  // index
  const uint64_t* codes;
  const float2* fac;        // {||o_r - c||, <o_bar,o>}
  const float2* sfac;       // scan factors {a / <o_bar,o>, a sqrt(1 - <o_bar,o>^2) / <o_bar,o>}
  const float* raw;         // list order
  const int64_t* ids;       // list order -> original id
  const int32_t* list_off;  // nlist + 1
  const float* cent;        // nlist x dim
  const float* crot;        // nlist x Dp (P^T c_k)
  const float* cnorm;       // nlist: ||c_k||^2
  int dim, dp, W, nlist;
  int qmax;                 // 2^B_q - 1: largest quantised query value (Sec. 3.3.1)
  int npl;                  // bit planes stored per pair: 4 (B_q <= 4) or 8
  int qoff;                 // int8 copy of q_u holds q_u - qoff (128 for B_q = 8, else 0)
  int metric;               // 0: squared L2; 1: inner product (cosine runs as IP on unit vectors)
  int mfma_f4;              // batched scan on FP8 x FP4 scaled MFMA instead of int8
  int boot_planes_only;     // 1: bit planes only for the pairs phase 0 scans (the rest go to the MFMA scan)
  int mf_rg;                // batched scan: groups of 16 query rows per work unit (1, 2 or 4)
  const float* fip;         // inner product: per code <o_r - c, c>
  float* pair_pt;           // inner product: per pair M_q - <q_r, c>
  float* q_m;               // inner product: per query M_q = ||q_r|| max ||o_r|| (1 + 1e-5)
  double rd, ird;            // sqrt(dp), 1 / sqrt(dp)
  float eps0;
  uint64_t seed;
  // batch
  const float* q;           // nq x dim
  const float* qrot;        // nq x Dp
  int64_t nq;
  int64_t qid_base;
  int nprobe;               // row stride of per-pair arrays
  int k;
  int chunk;                // codes per work unit
  int boot;                 // bootstrap target: phase 0 covers >= boot codes (boot >= k)
  const int32_t* probe;     // nq x nprobe
  const int32_t* nprobe_q;  // nq or null
  const int32_t* q_order;   // nq or null: the rerank's query order (largest nprobe first)
  // per pair
  PairRec* pairs;           // nq x nprobe
  uint64_t* planes;         // nq x nprobe x npl x W
  int8_t* qu8;              // nq x nprobe x Dp (MFMA path) or null
  int32_t* pair_choff;      // nq x (nprobe+1) local chunk prefix
  int32_t* pair_codeoff;    // nq x (nprobe+1) local code prefix
  // per query
  int32_t* q_nch;           // chunks
  int32_t* q_p0;            // bootstrap chunks
  int32_t* q_n0;            // bootstrap codes
  int64_t* q_ncode;         // probed codes
  int64_t* off_ch;          // nq+1 exclusive prefix of q_nch
  int64_t* off_p0;          // nq+1 prefix of q_p0
  int64_t* off_p1;          // nq+1 prefix of q_nch - q_p0
  int64_t* off_seg;         // nq+1 prefix of q_ncode
  int64_t* off_n0;          // nq+1 prefix of q_n0
  int64_t* blk_sums;        // 5 per block of kOffQ queries (query-offset scan)
  int32_t* chunk_qcode;     // per chunk (query order): first query-code index of the chunk
  unsigned long long* counters;  // work counters: [2] MFMA scan
  unsigned long long* prof_acc;  // profiling: codes of scan phase 0 / 1 (null when off)
  UnitDesc* units0;         // bootstrap work units
  UnitDesc* units1;         // main-phase work units
  // buffers
  Cand* seg;                // segment slots
  int32_t* seg_count;       // per chunk
  EstEnt* p0buf;
  float* tau;               // nq
  SeedEnt* seedk;           // nq x k
  int32_t* q_boot;          // nq: exact distances of the bootstrap rerank
  int32_t* q_rerank;        // nq: exact distances of the final rerank
  int32_t* q_cand;          // nq
  // MFMA grouping of main-phase pairs by list
  int32_t* mf_cnt;          // nlist: pairs per list
  int32_t* mf_fill;         // nlist: scatter cursors
  int64_t* mf_pair_off;     // nlist + 1
  int64_t* mf_unit_off;     // nlist + 1: (chunk, 16-pair group) units per list
  int32_t* mf_pairs;        // pair ids bucketed by list
  // outputs
  int64_t* out_ids;
  float* out_d;
  // parity export (scan phase 2): per code of the list at positions >= dbg_base
  int64_t dbg_base;
  int32_t *dbg_ip, *dbg_pc;
  float *dbg_est, *dbg_dist, *dbg_lb;
};

// Work planning: per-query chunk and code prefixes, bootstrap extent, and the
// query offsets (prefix sums over queries).
hipError_t launch_plan(const SearchDev& s, hipStream_t st);
// Per-pair quantisation (S3); with units = true also the scan's unit
// descriptors, which need launch_plan's results.
hipError_t launch_prep(const SearchDev& s, bool units, hipStream_t st);
int scan_popcnt_blocks_per_cu(int W, int npl);
// Row groups of the batched scan for code length dp: `want` (1, 2 or 4; other
// values mean 1), lowered until the query tile fits a block's LDS.
int mfma_row_groups(int dp, bool f4, int want);
int scan_mfma_blocks_per_cu(int dp, bool f4, int rg, bool narrow);
// phase 0: bootstrap units, 1: main units with the bound filter, 2: parity
// export of the main-phase table (s.dbg_*).
hipError_t launch_scan_popcnt(const SearchDev& s, int phase, int grid, hipStream_t st);
// The main-phase pairs grouped by list (mf_cnt, mf_pair_off, mf_unit_off,
// mf_pairs), which launch_scan_mfma's units read; independent of tau.
hipError_t launch_group_mfma(const SearchDev& s, hipStream_t st);
hipError_t launch_scan_mfma(const SearchDev& s, int phase, int grid, hipStream_t st);
hipError_t launch_tau(const SearchDev& s, hipStream_t st);
hipError_t launch_finalize(const SearchDev& s, hipStream_t st);
// Query order for the rerank: queries by descending per-query nprobe (64
// bins; order within a bin unspecified), so the longest reranks start first.
// hist: 128 int32 of scratch; order: nq int32.
hipError_t launch_query_order(const int32_t* nprobe_q, int64_t nq, int nprobe, int32_t* hist, int32_t* order,
                              hipStream_t st);

// debug: list scan with a given quantised query
hipError_t launch_debug_pack(const uint8_t* qu, int dp, int W, int npl, int qoff, float b, float vl, float delta,
                             float pt, PairRec* rec, uint64_t* planes, int8_t* qu8, float* pair_pt, int32_t list,
                             hipStream_t st);
// k-means building blocks (kernels_index.hip): max |x| as float bits
// (atomicMax into *out, which the caller zeroes), per-row argmin over a
// distance matrix (ties to the lower list), fixed-point member sums
// (sums[l][d] += round(x * scale), cnt[l] += 1), and the centroid update
// (non-empty lists: sum / (scale cnt); writes cent, its transpose and norms).
hipError_t launch_absmax(const float* x, int64_t n, uint32_t* out, hipStream_t st);
hipError_t launch_row_argmin(const float* D, int64_t rows, int nlist, int32_t* lab, hipStream_t st);
hipError_t launch_fixed_sums(const float* x, const int32_t* lab, int64_t rows, int dim, double scale,
                             unsigned long long* sums, unsigned int* cnt, hipStream_t st);
hipError_t launch_update_centroids(const unsigned long long* sums, const unsigned int* cnt, int nlist, int dim,
                                   double inv_scale, float* cent, float* centT, float* cnorm, hipStream_t st);
// Inner-product support (kernels_index.hip): per code fip[p] = <o_r - c, c>
// and the largest squared norm (float bits, atomicMax into *r2max, zeroed by
// the caller) of raw vectors in list order; rows normalised to unit length in
// place (zero rows stay zero); per query q_m[i] = ||q_i|| sqrt(r2max) (1 + 1e-5).
hipError_t launch_ip_terms(const float* raw, const float* cent, const int32_t* list_of, int64_t n, int dim,
                           float* fip, uint32_t* r2max, hipStream_t st);
hipError_t launch_normalize_rows(const float* x, int64_t n, int dim, float* y, hipStream_t st);
hipError_t launch_query_m(const float* q, int64_t nq, int dim, float rmax, float* q_m, hipStream_t st);
// x[i] ^= v for n bytes (the int8 copy of q_u back to 0 .. 2^B_q - 1)
hipError_t launch_xor_u8(uint8_t* x, int64_t n, uint8_t v, hipStream_t st);
hipError_t launch_debug_mfma(const SearchDev& s, const PairRec* rec, const int8_t* qu8,
                             int32_t list, int nchunks, int32_t* ip, int32_t* pc, float* est,
                             float* dist, float* lb, hipStream_t st);
hipError_t launch_debug_scan(const SearchDev& s, const PairRec* rec, const uint64_t* planes,
                             const int8_t* qu8, int32_t list, int kernel, int32_t* ip,
                             int32_t* pc, float* est, float* dist, float* lb, hipStream_t st);

}  // namespace rbq
