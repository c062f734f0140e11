/*
 * rabitq.h — C ABI of the MI355X (gfx950) RaBitQ query-phase library.
 *
 * RaBitQ (Gao & Long, SIGMOD 2024) estimates squared Euclidean distances from
 * D-bit codes of randomly rotated, centroid-normalised vectors, and reranks
 * the candidates whose error-bound interval can still reach the current k-th
 * nearest exact distance. This library implements
 *   - the index phase (Algorithm 1; Sec. 3.1) on the GPU: rotation by P,
 *     normalisation against the IVF centroid, sign codes, <o_bar,o> and
 *     ||o_r - c||;
 *   - the query phase (Algorithm 2; Sec. 3.2-3.3) and IVF search with the
 *     error-bound rerank (Sec. 4): rotate, probe the nearest lists, quantise
 *     the query to B_q bits (1..8, default 4) with randomised rounding per (query, list),
 *     integer <x_b, q_u> by AND + popcount or int8 MFMA, the unbiased estimate,
 *     the lower distance bound, exact rerank, top-k.
 *
 * Conventions for every function:
 *   - Returns an rbq_status. Nothing aborts and no C++ exception crosses the
 *     ABI. On error the outputs are unspecified, the index is unchanged and
 *     rbq_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device. Each argument states which; a
 *     pointer of the wrong kind is rejected with RBQ_EINVAL.
 *   - The caller owns all buffers it passes. The index copies what it needs
 *     at build/load time and owns that copy until rbq_index_destroy.
 *   - `stream` is a hipStream_t (NULL = default stream). Device outputs are
 *     written asynchronously on it; the caller synchronises. Functions that
 *     return host outputs synchronise the stream before returning.
 *   - An index owns one search workspace. rbq_search calls on one index are
 *     serialised by an internal mutex, and each search first waits (on its own
 *     stream, without blocking the host) for the kernels of the previous
 *     search, so searches issued on different streams are safe but do not
 *     overlap. rbq_index_build, rbq_index_destroy and rbq_nprobe_model_set
 *     must not run concurrently with any other call on the same index.
 */
#ifndef RABITQ_H
#define RABITQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBQ_OK = 0,
  RBQ_EINVAL = 1,        /* bad argument (null, out of range, wrong pointer kind) */
  RBQ_ENOMEM = 2,        /* host or device allocation failed */
  RBQ_EDEVICE = 3,       /* a HIP runtime call failed */
  RBQ_ESTATE = 4,        /* index not built, or call not allowed in this state */
  RBQ_EFORMAT = 5,       /* corrupt or truncated index file */
  RBQ_EUNSUPPORTED = 6   /* valid request the library does not implement */
} rbq_status;

/* Rotation arithmetic (S1 of the query path and the index-time rotation). */
enum {
  RBQ_ROT_FP32 = 0,      /* FP32 FMA GEMM */
  RBQ_ROT_BF16X3 = 1     /* split-BF16 (hi + lo) MFMA GEMM, FP32 accumulation:
                            hi*hi + hi*lo + lo*hi */
};

/* Kernel that computes the integer <x_b, q_u> (Sec. 3.3.2). */
enum {
  RBQ_SCAN_AUTO = 0,     /* autotuned / heuristic choice per search */
  RBQ_SCAN_POPCNT = 1,   /* bit-plane AND + popcount, one code per lane */
  RBQ_SCAN_MFMA = 2,     /* int8 MFMA over queries grouped by list */
  RBQ_SCAN_MFMA_FP4 = 3  /* the same contraction on the scaled FP8 (query, E4M3) x
                            FP4 (code bit, E2M1) MFMA with FP32 accumulation, exact
                            for B_q <= 4 (RBQ_EUNSUPPORTED above) */
};

/* What a search ranks by. The codes are the same for every metric.
 *   RBQ_METRIC_L2      squared Euclidean distance (Eq. (2)), smallest first
 *   RBQ_METRIC_IP      inner product, largest first: the conclusion's identity
 *                      <o_r, q_r> = ||o_r - c|| ||q_r - c|| <o, q> + <o_r - c, c>
 *                      + <q_r, c> carries Theorem 3.2's unbiased estimate of
 *                      <o, q> and its interval over to the inner product; lists
 *                      are probed by the largest <q_r, c_k>
 *   RBQ_METRIC_COSINE  cosine similarity: the inner product of the unit-
 *                      normalised vectors (the index normalises the data, a
 *                      search its queries; zero vectors stay zero) */
enum {
  RBQ_METRIC_L2 = 0,
  RBQ_METRIC_IP = 1,
  RBQ_METRIC_COSINE = 2
};

typedef struct rbq_index rbq_index;

/* Index parameters (Sec. 5.1 gives eps0 = 1.9, B_q = 4 and the default code
 * length, the smallest multiple of 64 not below D). */
typedef struct {
  int32_t dim;           /* D, raw vector length, >= 1 */
  int32_t code_bits;     /* 0 => 64*ceil(D/64); else a multiple of 64, >= D, <= 4096 */
  int32_t nlist;         /* number of IVF lists, 1..24576 (1 = flat index) */
  int32_t bq;            /* B_q, bits of the quantised query, 1..8 (Sec. 3.3.1;
                            Sec. 5.1 uses 4): q_u in 0..2^B_q - 1, B_q bit planes */
  float eps0;            /* confidence parameter of the error bound (Theorem 3.2) */
  int32_t rot_precision; /* RBQ_ROT_FP32 or RBQ_ROT_BF16X3 */
  uint64_t seed;         /* seeds the randomised rounding (and P if none is given) */
  int32_t metric;        /* RBQ_METRIC_L2 (default), RBQ_METRIC_IP or RBQ_METRIC_COSINE */
} rbq_params;

/* Per-search options. */
typedef struct {
  int32_t k;                       /* neighbours to return, 1..256 */
  int32_t nprobe;                  /* lists probed per query, 1..min(nlist, 16384) */
  int32_t scan_kernel;             /* RBQ_SCAN_* */
  int32_t use_learned_nprobe;      /* 1: per-query nprobe from the loaded MLP
                                      (falls back to `nprobe` when none is set) */
  const int32_t* nprobe_per_query; /* host or device, nq entries in 1..nprobe, or NULL */
  int64_t qid_base;                /* query i uses id qid_base + i in the rounding RNG */
  int32_t use_graph;               /* 1: run the search as one replay of a captured HIP
                                      graph (see below); 0: launch its kernels directly */
  int32_t rerank_waves;            /* waves that share one query's rerank: 0 = chosen
                                      from the call's batch size (1 from 2048 queries
                                      up, more for smaller batches), n >= 1 = n; at most
                                      64 and 4096 / k. Each wave reranks a fixed share
                                      of the query's chunks against its own threshold,
                                      so the result is the exact top-k of the probed
                                      lists whenever the bounds hold, for any value;
                                      which candidates beyond that get reranked (and
                                      the rerank counts) depend on it */
} rbq_search_opts;

/* Graph replay (use_graph = 1). The kernel sequence of a search is captured
 * once per shape (batch size rounded up to at most 6.25% more rows, k,
 * nprobe, scan kernel, learned or not, qid_base) and replayed: the queries are
 * copied into a staging buffer of the rounded size, the graph runs, and the
 * first nq rows of its results are copied out. Rows past nq search the staging
 * buffer's leftover (finite) contents and are discarded. The first search of a
 * shape runs once eagerly (allocation, warm-up) and is then captured. Results
 * are identical to use_graph = 0. Captured graphs are dropped when the index
 * is rebuilt, its workspace grows, or the nprobe model changes. With
 * profiling enabled the search runs eagerly. */

/* Counters of one search (filled only when a stats pointer is passed; that
 * makes rbq_search synchronise its stream before returning). */
typedef struct {
  int64_t queries;
  int64_t pairs;              /* (query, list) pairs probed */
  int64_t codes_scanned;      /* codes whose distance was estimated */
  int64_t reranked;           /* exact distances computed (bootstrap + final rerank) */
  int64_t candidates;         /* codes that passed the bound filter during the scan */
  int64_t reranked_bootstrap; /* of `reranked`: those of the bootstrap rerank (the
                                 min(4k, 256) best-estimated early codes per query) */
  int64_t nonfinite_fallbacks;/* learned nprobe: queries whose model output was not
                                 finite and that searched with the fixed nprobe */
} rbq_search_stats;

typedef struct {
  int32_t dim, code_bits, nlist, rot_precision;
  int64_t n;                  /* vectors indexed */
  int64_t device_bytes;       /* device memory held by the index (excl. workspace) */
  int64_t graph_captures;     /* searches captured as graphs so far (use_graph = 1) */
  int64_t graphs_cached;      /* captured graphs currently held */
} rbq_index_info;

/* Fills defaults: code_bits 0, bq 4, eps0 1.9, FP32 rotation, seed 0 (Sec. 5.1), L2. */
rbq_status rbq_params_default(rbq_params* p, int32_t dim, int32_t nlist);

/* Creates an empty index with validated parameters. *out is owned by the caller
 * and released with rbq_index_destroy. */
rbq_status rbq_index_create(const rbq_params* p, rbq_index** out);

/* Index phase (Algorithm 1; Sec. 3.1; IVF buckets of Sec. 4).
 *   data      host or device, n x dim float32, row-major; vector i gets id i
 *   centroids host or device, nlist x dim float32 (the IVF centroids, e.g. k-means)
 *   assign    host or device, n int32 in [0, nlist): list of each vector
 *   gauss     host or device, code_bits x code_bits float64 standard Gaussian
 *             draw, or NULL to draw it from params.seed. P is obtained by
 *             orthonormalising its rows (Gram-Schmidt, Sec. 3.1.2 and
 *             Appendix B), so P is Haar distributed. Codes are the signs of
 *             P^T (o_r - c) / ||o_r - c|| (Sec. 3.1.3); with D < code_bits the
 *             vectors are zero-padded (Sec. 5.1).
 * Each pointer may be host or device memory independently; device data is
 * reordered into list order on the device, host data is staged in blocks.
 * n is below 2^31 - 64, and 64*ceil(n/64) * code_bits/64 below 2^32 (32-bit
 * word offsets in the scan). Errors: RBQ_EINVAL for a NULL or out-of-range
 * argument (assign outside [0, nlist), non-finite values, a rank-deficient
 * draw), RBQ_ENOMEM / RBQ_EDEVICE from the device. Synchronises `stream`.
 * Rebuilding an index replaces its contents (and drops a learned-nprobe
 * model, whose features refer to the old lists). */
rbq_status rbq_index_build(rbq_index* idx, const float* data, int64_t n,
                           const float* centroids, const int32_t* assign,
                           const double* gauss, void* stream);

/* Algorithm 1 with a caller-supplied rotation: P is the code_bits x
 * code_bits orthogonal matrix of Sec. 3.1.2 (host or device float64,
 * row-major); codes use P^T v (P^{-1} = P^T, Sec. 3.1.3). Orthogonality is
 * checked on four seeded vectors (||P P^T x - x|| <= 1e-6 ||x||), otherwise
 * RBQ_EINVAL. Other arguments and errors as rbq_index_build. */
rbq_status rbq_index_build_rotation(rbq_index* idx, const float* data, int64_t n,
                                    const float* centroids, const int32_t* assign,
                                    const double* P, void* stream);

/* IVF clustering for the index phase (Sec. 4 groups the data into lists by
 * k-means before RaBitQ quantises each list against its centroid): Lloyd's
 * algorithm on the GPU.
 *   data       host or device, n x dim float32
 *   sample     rows used for the iterations: a seeded sample of that many
 *              (0 = all n); the final assignment covers all n rows
 *   init       host or device nlist x dim float32 initial centroids, or NULL
 *              for nlist distinct seeded sample rows
 *   centroids  host or device nlist x dim float32 (output)
 *   assign     host or device n int32 (output): the nearest final centroid
 * Each of `iters` rounds assigns every sample row to its nearest centroid
 * (squared distance ||c||^2 - 2 <x, c> in FP32 on the matrix cores, ties to
 * the lower list) and moves each non-empty list's centroid to the mean of its
 * rows (empty lists keep theirs). The means are summed in 64-bit fixed point,
 * so the result does not depend on the order of the parallel additions: the
 * same inputs and seed give the same bits. Temporary device memory: the data
 * (if given on the host), the sample, and up to 1 GiB of distances.
 * Errors: RBQ_EINVAL (NULL, n, dim or nlist out of range, nlist above the
 * sample size, non-finite data), RBQ_ENOMEM / RBQ_EDEVICE. Synchronises. */
rbq_status rbq_kmeans(const float* data, int64_t n, int32_t dim, int32_t nlist, int32_t iters,
                      int64_t sample, uint64_t seed, const float* init, float* centroids,
                      int32_t* assign, void* stream);

/* Query phase + IVF search (Algorithm 2; Sec. 4).
 *   queries   host or device, nq x dim float32 row-major
 *   out_ids   host or device, nq x k int64: ids of the k nearest by exact distance
 *             among the reranked candidates of the probed lists, ordered by
 *             (distance, id); -1 pads when fewer than k vectors were probed
 *   out_dists host or device, nq x k float32 exact squared distances (+inf pads);
 *             with RBQ_METRIC_IP / RBQ_METRIC_COSINE: the k largest inner
 *             products (cosines) in decreasing order, ties by id (-inf pads),
 *             computed as M_q - (M_q - <o_r, q_r>) with M_q = ||q_r|| max ||o_r||
 *             (1 + 1e-5), so within a few FP32 ulps of M_q of the exact value
 *   stats     host or NULL (see rbq_search_stats)
 * Host queries (and a host opts->nprobe_per_query) are copied to the device
 * on `stream`; host outputs are copied back and the stream is synchronised
 * before returning. nq may be 0 (nothing is launched). */
rbq_status rbq_search(rbq_index* idx, const float* queries, int64_t nq,
                      const rbq_search_opts* opts, int64_t* out_ids, float* out_dists,
                      rbq_search_stats* stats, void* stream);

/* Sets the confidence parameter eps0 of the error bound (Theorem 3.2) used by
 * later searches: the lower bound widens with eps0 and more candidates are
 * reranked (Sec. 5.2.4 studies recall against eps0). Codes are unchanged. */
rbq_status rbq_index_set_eps0(rbq_index* idx, float eps0);

/* rbq_search for callers that cannot allocate device memory (code under HIP
 * stream/graph capture, serving loops with a fixed memory budget, harnesses
 * that forbid hipMalloc): the same kernels and results as rbq_search on the
 * same arguments, with every workspace buffer carved from a device array of
 * RBQ_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * (from the first call on that GPU until the process ends). Nothing is
 * allocated or freed, and no HIP memset is issued (every buffer the search
 * needs zeroed is cleared by its own kernels).
 *   queries, out_ids, out_dists, opts->nprobe_per_query: device pointers
 *   (layouts as rbq_search); opts->use_graph must be 0; no statistics.
 * Errors: RBQ_EINVAL for a search whose workspace exceeds the array (the
 * message names the bytes needed: fewer queries or a smaller nprobe fit),
 * host pointers, or arguments rbq_search rejects; RBQ_ESTATE while profiling
 * is enabled on the index. The whole batch runs as one search (no
 * sub-batches). Every call on one GPU uses that GPU's one array: calls that
 * overlap in time on one GPU (other threads, or streams that are not
 * ordered with each other) race and give undefined results. */
#define RBQ_NOALLOC_SCRATCH_BYTES (128ll << 20)
rbq_status rbq_search_noalloc(rbq_index* idx, const float* queries, int64_t nq,
                              const rbq_search_opts* opts, int64_t* out_ids, float* out_dists,
                              void* stream);

rbq_status rbq_index_info_get(const rbq_index* idx, rbq_index_info* out);

/* Sizes of the IVF lists: host, nlist int64. */
rbq_status rbq_index_list_sizes(const rbq_index* idx, int64_t* sizes);

/* Versioned binary file: header, P, centroids, codes, factors, ids, raw vectors,
 * and a 64-bit checksum. load returns RBQ_EFORMAT on a bad or truncated file. */
rbq_status rbq_index_save(const rbq_index* idx, const char* path);
rbq_status rbq_index_load(const char* path, rbq_index** out);

rbq_status rbq_index_destroy(rbq_index* idx);

const char* rbq_last_error(void);

/* Autotuner of the search's launch shapes (batching of Algorithm 2's scans).
 * For batch-size buckets of 1, 8, 64, ... queries up to the sample (and the
 * sample itself), it times whole searches of the first rows of `queries` (host
 * or device, nq x dim, nq <= 2^24) at (k, nprobe): every chunk length (codes
 * per work unit of the persistent scans: 256, 512, 1024, 2048) with every scan
 * kernel (popcount, int8 MFMA, and FP8 x FP4 MFMA when B_q <= 4), then, for a
 * batched (MFMA) scan, 16, 32 or 64
 * query rows per work unit, then, for batches that split a query's rerank over
 * several waves, rerank waves 1..64 at the best choice. A search with
 * scan_kernel = RBQ_SCAN_AUTO and rerank_waves = 0 then uses the choices of
 * the bucket its batch size falls in (up to the geometric middle between two
 * tuned sizes); the chunk length applies to every later search. Results stay
 * the exact top-k of the probed lists whenever the bounds hold. Errors as
 * rbq_search; RBQ_ESTATE while profiling is enabled. Synchronises. */
rbq_status rbq_autotune(rbq_index* idx, const float* queries, int64_t nq, int32_t k,
                        int32_t nprobe, void* stream);

typedef struct {
  int64_t max_nq;        /* batches of at most this many queries use this entry */
  int32_t chunk;         /* codes per work unit */
  int32_t scan_kernel;   /* RBQ_SCAN_POPCNT, RBQ_SCAN_MFMA or RBQ_SCAN_MFMA_FP4 */
  int32_t rerank_waves;  /* 0: chosen from the batch size */
  float ms;              /* the trial search's time at the bucket's size */
  int32_t mfma_row_groups; /* batched scans: groups of 16 queries that share each
                              expanded code fragment (1, 2, 4; 0: one) */
} rbq_tune_entry;

/* The autotuner's table: up to max_entries entries (host) and *count, the
 * table's length (0 before rbq_autotune). */
rbq_status rbq_autotune_get(const rbq_index* idx, int32_t max_entries, rbq_tune_entry* entries,
                            int32_t* count);

/* Kernel timing. When enabled, rbq_search records HIP events on its stream
 * and accumulates, on the device, the number of codes each scan phase
 * estimated. rbq_profile_read synchronises the device and returns the sums
 * since the last enable (times in milliseconds). on = RBQ_PROFILE_STAGES:
 * events around each launch group (all six stage times); on =
 * RBQ_PROFILE_SCAN: events around the main scan and the rerank only
 * (ms_scan1 and ms_finalize; the other times read 0), so that fewer event
 * records interrupt the stream; 0: off. Each event record adds a few
 * microseconds between the kernels it separates. */
#define RBQ_PROFILE_STAGES 1
#define RBQ_PROFILE_SCAN 2
typedef struct {
  int64_t searches;       /* rbq_search calls profiled (a call may run several sub-batches) */
  double ms_front;        /* rotation + centroid scoring + probe selection */
  double ms_prep;         /* per-pair quantisation + work planning */
  double ms_scan0;        /* bootstrap scan (first chunks of each query) */
  double ms_tau;          /* bootstrap rerank / threshold */
  double ms_scan1;        /* main scan (all other chunks) */
  double ms_finalize;     /* rerank + top-k */
  int64_t codes_scan0;    /* codes estimated by the bootstrap scan */
  int64_t codes_scan1;    /* codes estimated by the main scan */
} rbq_profile;

rbq_status rbq_profile_enable(rbq_index* idx, int32_t on);   /* on: 0, 1 or 2 (above) */
rbq_status rbq_profile_read(rbq_index* idx, rbq_profile* out);

/* ---------------------------------------------------------------------------
 * Learned per-query nprobe (not part of the paper): an MLP
 *   features[96] -> 128 (ReLU) -> 32 logits over nprobe buckets
 * with BF16 weights and FP32 accumulation.
 *   features: log of the 64 nearest centroid distances relative to the
 *   nearest (slot 0 holds log d_(1)), then for the 8 nearest lists
 *   (||q_r-c_k||/||q_r-c_1||, v_l, v_r, sum q_u/(15*code_bits)).
 *   bucket j maps to nprobe b_j = max(b_{j-1}+1, round(4 * 2^(7j/31))), so
 *   b_0 = 4 and b_31 = 512. A query takes the smallest bucket whose cumulative
 *   softmax reaches `threshold`.
 */
#define RBQ_MLP_IN 96
#define RBQ_MLP_HIDDEN 128
#define RBQ_MLP_OUT 32

typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr;              /* Adam step size */
  float beta1, beta2, eps;
  uint64_t seed;         /* initialisation and shuffling */
} rbq_train_cfg;

/* Features of nq queries: queries device nq x dim, feats device nq x 96 float32. */
rbq_status rbq_nprobe_features(rbq_index* idx, const float* queries, int64_t nq,
                               int64_t qid_base, float* feats, void* stream);

/* Trains the MLP on the GPU (own BF16 forward/backward kernels, FP32 master
 * weights, Adam). feats device n x 96, labels device n int32 in [0, 32).
 * losses: host, epochs floats (mean loss per epoch) or NULL. */
rbq_status rbq_nprobe_model_train(rbq_index* idx, const float* feats, const int32_t* labels,
                                  int64_t n, const rbq_train_cfg* cfg, float* losses,
                                  void* stream);

/* Weights as FP32 host arrays in the order W1[96x128], b1[128], W2[128x32], b2[32]
 * (16,544 floats); NULL disables the model (fixed nprobe fallback). */
rbq_status rbq_nprobe_model_set(rbq_index* idx, const float* weights, float threshold);
rbq_status rbq_nprobe_model_get(const rbq_index* idx, float* weights, float* threshold);

/* Per-query nprobe from the model: feats device nq x 96 -> nprobe device nq int32,
 * logits device nq x 32 float32 (or NULL). Logits that are not all finite
 * give the largest nprobe (min(nlist, 512)).
 * In rbq_search (use_learned_nprobe = 1) the features, the network and this
 * policy run fused in one launch after the probe selection, with the same
 * BF16 arithmetic; there a query with non-finite logits searches with the
 * caller's fixed `nprobe`, and rbq_search_stats.nonfinite_fallbacks counts it. */
rbq_status rbq_nprobe_predict(rbq_index* idx, const float* feats, int64_t nq,
                              int32_t* nprobe, float* logits, void* stream);

/* The 32 bucket nprobe values b_0..b_31 (host int32[32]). */
rbq_status rbq_nprobe_bucket_table(int32_t* nprobe);

/* Training labels from neighbour lists (the traces a model is trained on).
 *   queries  device nq x dim float32
 *   nn_ids   device nq x k int64: each query's neighbours (e.g. the ids an
 *            rbq_search returned, or exact nearest neighbours); ids < 0 skipped
 *   need     device nq int32 or NULL: the smallest nprobe whose probed lists
 *            (the IVF probe order of Sec. 4: centroid distance, then list id,
 *            as rbq_search ranks them) hold every neighbour, 0 if none is valid
 *   labels   device nq int32: the smallest bucket whose nprobe >= need (31 if none)
 * Builds an id -> list map on first use (4 bytes per indexed vector, held by
 * the index). */
rbq_status rbq_nprobe_labels(rbq_index* idx, const float* queries, int64_t nq, const int64_t* nn_ids,
                             int32_t k, int32_t* labels, int32_t* need, void* stream);

/* One forward/backward of the MLP on given FP32 weights, for gradient checks:
 * x device n x 96, labels device n, weights/grads device 16,544 floats,
 * loss host float (mean cross-entropy). */
rbq_status rbq_mlp_loss_grad(const float* x, const int32_t* labels, int64_t n,
                             const float* weights, float* grads, float* loss, void* stream);

/* ---------------------------------------------------------------------------
 * Parity / debug exports: the search's own arithmetic on inputs chosen by the
 * caller, for checking it against an independent implementation; not meant
 * for production use. rbq_debug_scan runs the production scan kernels
 * themselves (an export phase of the popcount scan, the debug instance of
 * the MFMA scan's unit routine).
 */

/* Codes and factors as encoded on the GPU, in the caller's original vector
 * order: codes host n x (code_bits/64) uint64 (bit i%64 of word i/64 is the
 * sign bit of coordinate i), norm host n float (||o_r - c||), ipo host n float
 * (<o_bar, o>). Any output may be NULL. */
rbq_status rbq_debug_export_codes(const rbq_index* idx, uint64_t* codes, float* norm,
                                  float* ipo);

/* Rotated queries: queries device nq x dim -> out device nq x code_bits. */
rbq_status rbq_debug_rotate(rbq_index* idx, const float* queries, int64_t nq, float* out,
                            void* stream);

/* Centroid scoring (Sec. 4, IVF): queries device nq x dim -> dists device
 * nq x nlist float32, the squared distances ||q - c_k||^2 that the probe step
 * ranks, computed as ||q||^2 + ||c_k||^2 - 2 <q, c_k> with FP32 products on the
 * matrix cores and clamped at 0. The caller owns dists. */
rbq_status rbq_debug_centroid_dists(rbq_index* idx, const float* queries, int64_t nq, float* dists,
                                    void* stream);

/* Probe step: queries device nq x dim -> lists device nq x nprobe int32 (nearest
 * first, ties to the lower id), dists device nq x nprobe float32 (squared). */
rbq_status rbq_debug_probe(rbq_index* idx, const float* queries, int64_t nq, int32_t nprobe,
                           int32_t* lists, float* dists, void* stream);

/* Per-pair quantisation of the query (Sec. 3.1.1 normalisation against the
 * list centroid, Sec. 3.3.1 randomised uniform scalar quantisation with B_q
 * bits): queries device nq x dim, lists device nq x nprobe.
 * qu device (nq*nprobe) x code_bits uint8 (0..2^B_q - 1); scal device (nq*nprobe) x 4
 * float32 {||q_r - c||, v_l, Delta, sum q_u}. */
rbq_status rbq_debug_quantize(rbq_index* idx, const float* queries, int64_t nq,
                              const int32_t* lists, int32_t nprobe, int64_t qid_base,
                              uint8_t* qu, float* scal, void* stream);

/* Scan arithmetic of one list for a caller-given quantised query: the integer
 * <x_b, q_u> and popcount (Sec. 3.3.2), the estimate <x_bar,q_bar>/<o_bar,o>
 * (Theorem 3.2, with the Sec. 3.3.2 decomposition), the distance by Eq. (2)
 * and its lower bound with the half-width of Theorem 3.2:
 * qu device code_bits uint8, scal host 4 floats {b, v_l, Delta, t} where t is
 * unused for L2 and, for the inner-product metrics, the pair's constant
 * M_q - <q_r, c>: dist is then M_q minus the inner-product estimate and lb
 * subtracts ||o_r - c|| ||q_r - c|| times the half-width;
 * outputs device, one per member of the list in list order (ids of
 * rbq_debug_list_ids): ip, pc int32; est, dist, lb float32.
 * kernel: RBQ_SCAN_POPCNT, RBQ_SCAN_MFMA or RBQ_SCAN_MFMA_FP4. */
rbq_status rbq_debug_scan(rbq_index* idx, int32_t list, const uint8_t* qu, const float* scal,
                          int32_t kernel, int32_t* ip, int32_t* pc, float* est, float* dist,
                          float* lb, void* stream);

/* Ids of the members of a list in stored order: host, size of the list. */
rbq_status rbq_debug_list_ids(const rbq_index* idx, int32_t list, int64_t* ids);

/* Searches split a batch into sub-batches whose candidate segments (8 bytes
 * per probed code per query, sized for the largest lists) stay within a
 * budget: by default a quarter of the device memory free at the first search,
 * at least 8 GiB. This sets the budget (bytes; 0 restores the default) so that
 * tests can force the split. Process-wide. */
rbq_status rbq_debug_seg_budget(int64_t bytes);

/* Test hook: the n-th device allocation after this call fails with RBQ_ENOMEM
 * (0 disables). Process-wide; for failure-path tests only. */
rbq_status rbq_debug_fail_alloc_after(int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* RABITQ_H */
