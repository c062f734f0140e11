// Host-side index object and workspace (runtime.cpp, mlp_runtime.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rabitq.h"
#include "rbq_internal.hpp"

namespace rbq {

// Bytes of the device array that rbq_search_noalloc carves its workspace from.
constexpr size_t kNoAllocScratchBytes = 128ull << 20;

// Device buffer that grows on demand and is freed with its owner. While an
// Arena is active on the calling thread, ensure() carves from it instead of
// allocating (and such buffers are never freed: the arena owns the memory).
struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes);
  void release();
};

// A DBuf for temporaries of one call: released when it goes out of scope,
// on every return path (hipFree waits for the device work that uses it).
struct TmpBuf : DBuf {
  TmpBuf() = default;
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  ~TmpBuf() { release(); }
};

// Bumped whenever any DBuf is (re)allocated or released: a captured graph
// holds device addresses and is replayed only while this is unchanged.
uint64_t buffer_generation();
// Rerank waves per query for a batch of nq queries with k results (1 for
// large batches), and the rerank with W waves per query (W > 1 needs part,
// nq * W * k keys, and pst, nq * W * 2 counters).
int finalize_split(int64_t nq, int k);
// Waves sharing a query's bootstrap rerank (at least 32 of its min(256, 4k)
// codes each), and that rerank with W waves (W > 1 needs tpart, nq *
// min(256, 4k) keys).
int tau_split(int fin_w, int k);
hipError_t launch_tau_split(const SearchDev& s, int W, uint64_t* tpart, hipStream_t st);
// Rerank waves for a requested count (0: finalize_split's choice), clamped to
// 1 .. min(64, kFinMergeCap / k).
constexpr int kFinMergeCap = 4096;   // keys of a query's split-rerank merge (W k)
constexpr int kFinSplitMaxWaves = 64;   // most rerank waves per query
inline int fin_waves(int requested, int64_t nq, int k) {
  if (requested <= 0) return finalize_split(nq, k);
  const int cap = std::max(1, std::min(64, kFinMergeCap / std::max(k, 1)));
  return std::min(requested, cap);
}
hipError_t launch_finalize_split(const SearchDev& s, int W, uint64_t* part, int32_t* pst, hipStream_t st);
// Bytes of candidate segments a (sub-)batch may use (see rbq_debug_seg_budget).
int64_t seg_budget();
void g_seg_budget_set(int64_t b);

// Per batch-size bucket choices of the autotuner: batches of at most max_nq
// queries use this chunk length (codes per work unit), scan kernel and rerank
// waves per query (0: chosen from the batch size).
struct TuneEntry {
  int64_t max_nq = INT64_MAX;
  int chunk = kDefaultChunk;
  int kernel = RBQ_SCAN_POPCNT;
  int fin_w = 0;
  int mf_rg = 0;    // batched scan: 16-row query groups per work unit (0: one)
  float ms = 0.f;   // measured time of the trial batch
};

// One captured search (graph replay of rbq_search with use_graph = 1).
struct GraphEntry {
  int64_t nqb = 0;        // rows (rounded batch size)
  int k = 0, nprobe = 0, kernel = 0, chunk = 0, mf_rg = 0;
  bool learned = false, per_query = false;
  int64_t qid_base = 0;
  int fin_w = 1;          // rerank waves per query
  uint64_t gen = 0;       // buffer_generation() at capture
  uint64_t last_use = 0;
  hipGraphExec_t exec = nullptr;
};

hipError_t dmalloc(void** p, size_t bytes);
rbq_status set_error(rbq_status st, const char* msg);

// Caller-provided device memory that DBuf::ensure carves from on this thread.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};
// rbq_search_noalloc's body: the search of rbq_search (device queries and
// outputs, one batch, no stats, no graph, no profiling) with every workspace
// buffer carved from [base, base + cap); fails with RBQ_EINVAL naming the
// bytes it would need when they exceed cap.
rbq_status search_in_arena(rbq_index* idx, const float* queries, int64_t nq, const rbq_search_opts* opts,
                           int64_t* out_ids, float* out_dists, void* base, size_t cap, hipStream_t st);
bool is_device_ptr(const void* p);
uint64_t host_splitmix64(uint64_t x);

struct Workspace {
  DBuf qrot, cd, cgmin, probe, probe_d, pairs, planes, qu8, pair_choff, pair_codeoff;
  DBuf q_nch, q_p0, q_n0, q_ncode, offs, counters, seg, seg_count, p0buf, tau, seedk;
  DBuf q_order, order_hist;   // rerank query order (per-query nprobe)
  DBuf lstats;                // learned nprobe: statistics of each query's 8 nearest lists
  DBuf chunk_qcode;   // chunk (query order) -> first query-code index
  DBuf q_boot, q_rerank, q_cand, nprobe_q, q_fb, feats, tmp;
  DBuf pair_pt, q_m, qn;    // inner-product metrics: pair constants, M_q, normalised queries (cosine)
  DBuf mf_cnt, mf_fill, mf_pair_off, mf_unit_off, mf_pairs, units0, units1;
  DBuf fin_part, fin_pst;   // split rerank of small batches: partial top-k lists, statistics
  DBuf tau_part;            // split bootstrap rerank: exact keys, min(256, 4k) per query
};

struct ProfState {
  bool on = false;
  int level = 0;   // RBQ_PROFILE_STAGES or RBQ_PROFILE_SCAN while on
  int64_t searches = 0;
  // per search: 7 events delimiting front, prep, scan0, tau, scan1, finalize
  // (null where the level records none)
  std::vector<hipEvent_t> events;
  DBuf acc;    // int64 [2]: codes of scan0, scan1
  void clear();
};

struct MlpState {
  bool has_model = false;
  float threshold = 0.9f;
  std::vector<float> host_w;   // FP32 weights, rbq_nprobe_model_set order
  DBuf w32, wbf, wfrag, grad, m, v, act;   // wfrag: BF16 weights in MFMA fragment order
};

// MFMA scan availability (kernels_mfma.hip).
bool mfma_available();
// Zero-fill by a kernel (no memset node when a caller captures the stream).
hipError_t launch_zero_u32(void* p, int64_t nwords, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_pairs_to_scal(const SearchDev& s, float* scal, hipStream_t st);

}  // namespace rbq

struct rbq_index {
  rbq_params prm{};
  int dim = 0, dp = 0, W = 0, nlist = 0;
  int64_t n = 0;
  bool built = false;
  int64_t device_bytes = 0;
  std::mutex mu;
  hipEvent_t done_event = nullptr;

  // host copies
  std::vector<double> h_P;          // dp x dp
  std::vector<float> h_cent;        // nlist x dim
  std::vector<int64_t> h_list_off;  // nlist + 1
  std::vector<int64_t> h_ids;       // position -> original id
  std::vector<int64_t> sizes_desc, codes_prefix;

  // device index
  rbq::DBuf d_codes, d_fac, d_raw, d_ids, d_list_off, d_cent, d_centT, d_cnorm, d_crot;
  rbq::DBuf d_sfac;   // scan factors per code (see estimate), derived from d_fac
  rbq::DBuf d_P32, d_Phi, d_Plo;
  // BF16X3 indexes: the centroids as BF16 hi/lo planes [nlist][dim] for the
  // split-BF16 centroid distances (null otherwise)
  rbq::DBuf d_chi, d_clo;
  const uint16_t* cent_hi() const { return (const uint16_t*)d_chi.p; }
  const uint16_t* cent_lo() const { return (const uint16_t*)d_clo.p; }
  rbq::DBuf d_id2list;   // id -> list (built on first use by rbq_nprobe_labels)
  // inner-product metrics: per code <o_r - c, c>, the centroid norms the probe
  // GEMM uses (all max ||c||^2, so its ||q||^2 + . - 2 <q, c> ranks by <q, c>),
  // and max ||o_r||
  rbq::DBuf d_fip, d_cnorm_probe;
  float rmax = 0.f;
  const float* probe_cnorm() const { return (const float*)(prm.metric != RBQ_METRIC_L2 ? d_cnorm_probe.p : d_cnorm.p); }

  rbq::Workspace ws;
  rbq::MlpState mlp;
  rbq::ProfState prof;

  // autotuned choices per batch-size bucket (empty: defaults)
  std::vector<rbq::TuneEntry> tune;
  rbq::TuneEntry tuned_for(int64_t nq) const;

  ~rbq_index();
  std::vector<rbq::DBuf*> all_buffers();
  int64_t max_codes(int nprobe) const;
  int64_t max_chunks(int nprobe, int chunk) const;
  // captured searches (LRU, at most kMaxGraphs) and their staging buffers
  std::vector<rbq::GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t graph_rows_hint = 0;   // rows the graph-mode workspace is sized for
  int64_t graph_mem_cap = 0;     // bytes of candidate segments graph mode may reserve
  int64_t graph_captures = 0;
  hipStream_t cap_stream = nullptr;
  rbq::DBuf g_q, g_ids, g_d, g_npq;
  rbq::DBuf h_stage_q, h_stage_npq, h_stage_ids, h_stage_d;   // device copies of host search arguments
  void graphs_clear();
};

namespace rbq {
rbq_status learned_nprobe(rbq_index* idx, const float* queries, int64_t nq, int nprobe_max, int stride,
                          int64_t qid_base, hipStream_t st, const int32_t** out);
// Reserves the MLP activation buffers for `rows` queries.
rbq_status mlp_reserve(rbq_index* idx, int64_t rows);
rbq_status rotate_rows(rbq_index* idx, const float* X, int64_t lda, const float* sub,
                       const int32_t* sel, int64_t M, float* Y, hipStream_t st);
// seg_exact: leave the candidate segments to the caller (sized after the plan
// from the exact code counts) instead of the worst case nq * max_codes(nprobe).
rbq_status ensure_workspace(rbq_index* idx, int64_t nq, int nprobe, int k, int chunk, bool mfma,
                            int fin_w = 1, bool seg_exact = false);
SearchDev make_dev(rbq_index* idx, const float* queries, int64_t nq, int nprobe, int k, int chunk,
                   const int32_t* nprobe_q, int64_t qid_base, bool mfma, int64_t* out_ids,
                   float* out_d);
rbq_status scan_factors(rbq_index* idx, hipStream_t st);
// Inner-product metrics: per code <o_r - c, c> and max ||o_r|| from the raw
// vectors in list order (list_of: device, list of each position).
rbq_status ip_factors(rbq_index* idx, const int32_t* list_of, hipStream_t st);
// The queries a search works on: normalised into the workspace for the cosine
// metric, and M_q computed for the inner-product metrics (workspace sized).
rbq_status prepare_queries(rbq_index* idx, const float* queries, int64_t nq, hipStream_t st, const float** out);
rbq_status front(rbq_index* idx, const float* queries, int64_t nq, int nprobe,
                 const int32_t* nprobe_q, hipStream_t st);
// One search on `st`. `learned`: per-query nprobe from the model (the caller
// checked that one is set). Reports the per-query nprobe array in effect
// (NULL: all use the fixed value) and the probe stride.
rbq_status search_locked(rbq_index* idx, const float* queries, int64_t nq, rbq_search_opts o, int64_t* out_ids,
                         float* out_dists, rbq_search_stats* stats, hipStream_t st, const TuneEntry* force);
// seg_cap > 0: size the candidate segments from the plan's exact code counts
// (one stream synchronisation) and search only the first *done queries whose
// segments fit in seg_cap bytes (at least one); seg_cap = 0: all nq queries
// with worst-case segments.
rbq_status run_search(rbq_index* idx, const float* queries, int64_t nq, const rbq_search_opts& opts,
                      int scan_kernel, int chunk, int mf_rg, bool learned, int64_t* out_ids, float* out_d,
                      hipStream_t st, const int32_t** used_npq, int* used_stride, int64_t seg_cap = 0,
                      int64_t* done = nullptr);
}  // namespace rbq
