/*
 * binsketch.h — C ABI of the BinSketch GPU library (libbinsketch.so, gfx950).
 *
 * BinSketch (Pratap, Bera, Revanuru, arXiv 1910.04658) compresses a sparse
 * binary vector a in {0,1}^d into an N-bit sketch a_s by sending every set bit
 * i through a random map pi:[d] -> [N] and OR-ing the bits that land on the
 * same target (Section 3, Definition "BinSketch"). Inner product, Hamming
 * distance, Jaccard and cosine similarity are then estimated from |a_s|,
 * |b_s| and |a_s AND b_s| alone (Algorithms 1-4).
 *
 * Conventions shared by every entry point
 *   - All data pointers are DEVICE pointers on the current HIP device,
 *     allocated and owned by the caller. The library allocates no device
 *     memory and keeps no state between calls apart from a per-device check
 *     that the device is a gfx950, the host-side batch handles (below) and
 *     the fixed scratch array of bs_estimate_noalloc (a static device array of
 *     BS_NOALLOC_SCRATCH_BYTES per GPU, loaded with the library's code).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on that stream and returns before the
 *     work completes; results are valid once the stream has been synchronised.
 *   - Indices are 0-based (the paper counts from 1).
 *   - A sketch of width N is N/64 little-endian 64-bit words per row; bit j of
 *     the sketch is bit (j % 64) of word (j / 64). N must be a multiple of 64,
 *     between 64 and 65536.
 *   - Errors that the host can see from the arguments alone are returned as a
 *     bs_status before anything is enqueued, and no output is written. Errors
 *     in the CONTENT of device arrays (an index outside [0, d), a map value
 *     outside [0, N), a malformed indptr) cannot be seen by the host without
 *     a synchronisation; bs_sketch reports them through `err_flag`.
 *   - Every call may be captured into a HIP graph: none of them allocates,
 *     synchronises or issues a memset node.
 */
#ifndef BINSKETCH_H
#define BINSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BS_OK = 0,
  BS_ERR_NULL = 1,      /* a required pointer is NULL */
  BS_ERR_ARG = 2,       /* a size or parameter is out of range */
  BS_ERR_WORKSPACE = 3, /* the workspace is NULL or smaller than required */
  BS_ERR_HIP = 4,       /* the HIP runtime rejected a launch */
  BS_ERR_DEVICE = 5,    /* the current device is not a gfx950 */
  BS_ERR_SCRATCH = 6    /* the call needs more than BS_NOALLOC_SCRATCH_BYTES of
                           fixed scratch (bs_estimate_noalloc) */
} bs_status;

typedef enum { BS_IP = 0, BS_HAMMING = 1, BS_JACCARD = 2, BS_COSINE = 3 } bs_measure;

typedef enum { BS_F64 = 0, BS_F32 = 1 } bs_dtype;

/* Bits that bs_sketch ORs into *err_flag. */
#define BS_FLAG_INDPTR 1 /* indptr[0] != 0, not non-decreasing, or beyond nnz */
#define BS_FLAG_INDEX 2  /* a CSR index outside [0, d) */
#define BS_FLAG_MAP 4    /* a value of pi outside [0, N) */

#define BS_MAX_N 65536
#define BS_MAX_K 1024

/* Library version, as 10000*major + 100*minor + patch. */
int bs_version(void);

/* Human-readable name of a bs_status value (static storage). */
const char* bs_status_string(int status);

/* Number of 64-bit words per sketch, N/64; 0 if N is not a valid width. */
int32_t bs_words(int32_t N);

/*
 * bs_sketch — compress n_rows binary vectors (Section 3, Definition
 * "BinSketch"): sketches[r] has bit j set iff some index i of row r has
 * pi[i] == j; popcounts[r] = |a_s| (Algorithm 1, first step).
 *
 *   indptr     int32[n_rows + 1]  CSR row pointers: row r holds
 *                                 indices[indptr[r] .. indptr[r+1]). Must
 *                                 start at 0, be non-decreasing and end at nnz.
 *   indices    int32[nnz]         set indices in [0, d); any order, repeats
 *                                 allowed (the vectors are binary).
 *   n_rows     >= 0               number of vectors.
 *   nnz        >= 0, < 2^31       length of `indices` (the int32 indptr
 *                                 bounds a batch to 2^31-1 set bits).
 *   pi         int32[d]           the random map, values in [0, N).
 *   d          >= 1, < 2^31       dimension of the input vectors.
 *   N                              sketch width in bits (see above).
 *   sketches   uint64[n_rows][N/64] output; every word is written.
 *   popcounts  int32[n_rows]      output, or NULL to skip.
 *   err_flag   int32[1]           device word that receives BS_FLAG_* bits by
 *                                 atomic OR when the content is malformed, or
 *                                 NULL. The caller clears it; it is never
 *                                 cleared here. When a flag is raised the
 *                                 affected rows are written but undefined.
 *   workspace  device buffer of bs_sketch_workspace_size(d, N) bytes, 16-byte
 *              aligned, or NULL. With it, pi is bit-packed there once per call
 *              and kept in LDS while sketching (when it fits: d*ceil(log2 N)
 *              bits well under 160 KB); without it, or when the packed map does
 *              not fit, every pi[i] is gathered from global memory. Both give
 *              identical sketches.
 * Returns BS_ERR_ARG for a bad size or width, then BS_ERR_NULL for a NULL
 * indptr or pi, a NULL indices with nnz > 0 or a NULL sketches with
 * n_rows > 0 (a pointer to an empty array may be NULL everywhere below).
 */
size_t bs_sketch_workspace_size(int64_t d, int32_t N);
bs_status bs_sketch(const int32_t* indptr, const int32_t* indices, int64_t n_rows, int64_t nnz,
                    const int32_t* pi, int64_t d, int32_t N, uint64_t* sketches,
                    int32_t* popcounts, int32_t* err_flag, void* workspace,
                    size_t workspace_bytes, void* stream);

/*
 * bs_sketch_parts — bs_sketch of up to BS_SKETCH_MAX_PARTS CSR matrices that
 * share one map pi (e.g. a corpus and its queries) in one launch: the map is
 * packed and staged once, and the waves are split between the parts in
 * proportion to their set bits. Every part's sketches and popcounts are
 * exactly what bs_sketch writes for it alone.
 *
 *   parts      host array of n_parts descriptions; each field as the
 *              bs_sketch argument of the same name (device pointers).
 *   n_parts    1 .. BS_SKETCH_MAX_PARTS.
 *   pi, d, N, err_flag, workspace, workspace_bytes, stream: as bs_sketch
 *              (one err_flag for the call; flags of every part are ORed in).
 * Returns BS_ERR_ARG for n_parts out of range or any bad size or width (as
 * bs_sketch, for every part), then BS_ERR_NULL for a NULL parts array or
 * pi, or a part's NULL pointer that bs_sketch would reject.
 */
#define BS_SKETCH_MAX_PARTS 4
typedef struct {
  const int32_t* indptr;  /* int32[n_rows + 1] */
  const int32_t* indices; /* int32[nnz] */
  int64_t n_rows;
  int64_t nnz;
  uint64_t* sketches;     /* uint64[n_rows][N/64] */
  int32_t* popcounts;     /* int32[n_rows] or NULL */
} bs_sketch_part;
bs_status bs_sketch_parts(const bs_sketch_part* parts, int32_t n_parts, const int32_t* pi, int64_t d,
                          int32_t N, int32_t* err_flag, void* workspace, size_t workspace_bytes,
                          void* stream);

/*
 * bs_sketch_prepare_map / bs_sketch_parts_prepared — bs_sketch_parts for a
 * map pi that stays fixed across calls (the map is chosen once per (d, N),
 * Section 3, the paragraph after the Definition): bs_sketch_prepare_map
 * bit-packs pi into `map` once (the form bs_sketch builds in its workspace on
 * every call) and reports values outside [0, N) through err_flag
 * (BS_FLAG_MAP); bs_sketch_parts_prepared then sketches with that packed map
 * and no packing launch. Outputs are exactly those of bs_sketch_parts.
 *   map        device buffer of bs_sketch_workspace_size(d, N) bytes,
 *              16-byte aligned; written by prepare, only read afterwards
 *              (calls may overlap). pi must be the map it was prepared from
 *              (it is still read when the packed map does not fit in LDS).
 * Returns as bs_sketch_parts; BS_ERR_WORKSPACE for a NULL, short or
 * misaligned map.
 */
bs_status bs_sketch_prepare_map(const int32_t* pi, int64_t d, int32_t N, int32_t* err_flag, void* map,
                                size_t map_bytes, void* stream);
bs_status bs_sketch_parts_prepared(const bs_sketch_part* parts, int32_t n_parts, const int32_t* pi, int64_t d,
                                   int32_t N, const void* map, size_t map_bytes, int32_t* err_flag,
                                   void* stream);

/*
 * bs_and_popcount — all-pairs sketch inner products
 * out[p][q] = |A_p AND B_q| = <a_s, b_s> (Algorithm 1, second step).
 *
 *   A   uint64[nA][N/64], B uint64[nB][N/64]   sketches (as bs_sketch writes).
 *   out int32[nA][nB]                          output, row-major.
 * nA, nB >= 0 with nA * nB < 2^62.
 */
bs_status bs_and_popcount(const uint64_t* A, int64_t nA, const uint64_t* B, int64_t nB,
                          int32_t N, int32_t* out, void* stream);

/*
 * bs_estimate — all-pairs estimates in FP64 (Algorithms 1-4) for every pair
 * (A_p, B_q), written row-major [nA][nB] into each non-NULL output:
 *   ip   estimated inner product n_ab            (Algorithm 1)
 *   ham  estimated Hamming distance              (Algorithm 2)
 *   js   estimated Jaccard similarity            (Algorithm 3)
 *   cos  estimated cosine similarity             (Algorithm 4)
 * At least one output must be non-NULL. The estimators are evaluated as
 *   T(x) = ln(1 - x/N) / ln(1 - 1/N),   x clamped to N-1 (saturation),
 *   s = T(|a_s|) + T(|b_s|),  ip = s - T(|a_s OR b_s|),  ham = s - 2 ip,
 *   js = ip / (ip + ham) (0 when the denominator is 0),
 *   cos = ip / sqrt(T(|a_s|) T(|b_s|)) (0 when the product is 0),
 * which equals Algorithm 1 exactly whenever no count reaches N, with
 * Hamming read as |a| + |b| - 2 IP (the number of differing coordinates).
 * Negative estimates are returned unclamped.
 *   popA, popB int32[nA], int32[nB]: the row popcounts |a_s| (Algorithm 1,
 *              first step) exactly as bs_sketch writes them, or NULL to have
 *              them computed here. Wrong values give wrong estimates.
 *   workspace  device buffer of at least bs_estimate_workspace_size(nA, nB, N)
 *              bytes, 256-byte aligned; overwritten (the T table and the row
 *              popcounts |a_s|, |b_s| of Algorithm 1, first step).
 */
size_t bs_estimate_workspace_size(int64_t nA, int64_t nB, int32_t N);
bs_status bs_estimate(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                      const int32_t* popB, int64_t nB, int32_t N, double* ip, double* ham,
                      double* js, double* cos, void* workspace, size_t workspace_bytes,
                      void* stream);

/*
 * bs_estimate_scores — the all-pairs estimates of ONE measure (Algorithms
 * 1-4, chosen by `measure`, a bs_measure) as a dense row-major [nA][nB]
 * matrix `scores` of score_dtype:
 *   BS_F64  double: exactly the plane bs_estimate writes for that measure;
 *   BS_F32  float: the score bs_topk ranks by, i.e. the same expressions
 *           evaluated in IEEE float from T rounded once to float
 *           (s = T(x_a) + T(x_b), ip = s - T(x_u), ham = s - 2 ip, ...),
 *           so a row's k best entries are bs_topk's result for that query.
 * popA, popB, workspace (bs_estimate_workspace_size bytes, 256-byte aligned)
 * and the statuses as bs_estimate; BS_ERR_ARG also for a measure or
 * score_dtype out of range, BS_ERR_NULL for a NULL scores.
 */
bs_status bs_estimate_scores(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                             const int32_t* popB, int64_t nB, int32_t N, int32_t measure, void* scores,
                             int32_t score_dtype, void* workspace, size_t workspace_bytes, void* stream);

/*
 * bs_estimate_noalloc — bs_estimate for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same launches and the same results, with the
 * workspace replaced by a fixed scratch array of BS_NOALLOC_SCRATCH_BYTES
 * that the library holds in device memory, one copy per GPU, from the first
 * call on that GPU until the process ends. The call allocates nothing.
 *   Scratch use: the FP64 T table, align256(8 (N + 1)) bytes (at most
 *   513 KB), plus align256(4 nA) if popA is NULL and align256(4 nB) if popB
 *   is NULL. A call needing more returns BS_ERR_SCRATCH before any launch
 *   (pass popA / popB, e.g. the popcounts bs_sketch writes, to lift the row
 *   limit: then any nA, nB are accepted).
 *   Every call on a GPU uses that GPU's one array, and each call writes all
 *   the scratch it reads, so consecutive calls need no clearing; calls that
 *   overlap in time on one GPU (different streams or host threads) race on
 *   the array and give undefined results.
 * Arguments and the other statuses as bs_estimate, without the workspace.
 */
#define BS_NOALLOC_SCRATCH_BYTES (4u << 20)
bs_status bs_estimate_noalloc(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                              const int32_t* popB, int64_t nB, int32_t N, double* ip, double* ham,
                              double* js, double* cos, void* stream);

/*
 * bs_topk — for every query row Q_p, the k corpus rows C_q with the best
 * FP32 score of `measure` (the estimators of bs_estimate evaluated in IEEE
 * float from T rounded to float): highest first for BS_IP, BS_JACCARD and
 * BS_COSINE, lowest first for BS_HAMMING; ties go to the smaller corpus index.
 *
 *   Q          uint64[nQ][N/64] query sketches;  C uint64[nC][N/64] corpus.
 *   popQ, popC row popcounts as bs_sketch writes them, or NULL (computed here).
 *   k          1 <= k <= min(nC, BS_MAX_K).
 *   out_idx    int32[nQ][k]   corpus row indices, best first.
 *   out_score  float[nQ][k]   their scores, or NULL to skip.
 *   workspace  >= bs_topk_workspace_size(nQ, nC, N, k) bytes, 256-byte
 *              aligned, overwritten.
 * The result does not depend on the launch configuration or on timing.
 */
size_t bs_topk_workspace_size(int64_t nQ, int64_t nC, int32_t N, int32_t k);

/*
 * Corpus rows that bs_topk scores exactly in its sample pass for a corpus of
 * nC rows (every stride-th row, stride = nC / S); the scan pass estimates the
 * other nC - S rows of every query. 0 for nC < 1. Pure function of nC.
 */
int64_t bs_topk_sample_size(int64_t nC);
bs_status bs_topk(const uint64_t* Q, const int32_t* popQ, int64_t nQ, const uint64_t* C,
                  const int32_t* popC, int64_t nC, int32_t N, int32_t measure, int32_t k,
                  int32_t* out_idx, float* out_score, void* workspace, size_t workspace_bytes,
                  void* stream);

/*
 * Batched problems — many independent corpora, each with its own queries,
 * map pi, dimension d, width N and k, sketched (Section 3) and ranked
 * (bs_topk's selection rule) together. The batch is recorded once into a HIP
 * graph whose kernels each cover every problem (one sketch launch for all
 * corpora and queries, then one launch per top-k stage and kernel variant)
 * and replayed by bs_batch_run with a single hipGraphLaunch. Results equal
 * those of bs_sketch and bs_topk on each problem alone, whatever the tile
 * shapes.
 *
 * A batch handle is host memory the library allocates (bs_batch_destroy
 * frees it, with its graph); device memory is the caller's workspace.
 *
 *   bs_batch_item   one problem; every pointer is a device pointer:
 *     indptr, indices  corpus CSR (int32; n_rows >= 1 rows, nnz entries)
 *     q_indptr, q_indices  query CSR (n_queries >= 0 rows, q_nnz entries)
 *     pi               int32[d] map into [0, N)
 *     sketches, popcounts      out: uint64[n_rows][N/64], int32[n_rows]
 *     q_sketches, q_popcounts  out: uint64[n_queries][N/64], int32[n_queries]
 *     out_idx, out_score       out: int32[n_queries][k], float[...] or NULL
 *     1 <= k <= min(n_rows, BS_MAX_K); nnz and q_nnz < 2^31.
 *   bs_batch_shape  the scan tile shape used for one width: 64-query groups
 *     per wave (qpl; 1 for widths that scan on the matrix cores, N a
 *     multiple of 256) and the scan grid size in waves (0 = built-in rule);
 *     ms is the time the autotuner measured for that width's top-k stages
 *     (-1 if not tuned).
 *
 * bs_batch_workspace_size  device bytes for the items (0 if an item is
 *     invalid); enough for every shape the autotuner can choose.
 * bs_batch_create   plans the batch (measure as bs_topk), copies its tables
 *     into the workspace (synchronously) and returns the handle; `shapes`
 *     (may be NULL) fixes the shape per width, e.g. from an earlier
 *     autotune. err_flags: int32[n_items] device words or NULL; the run
 *     clears them, then ORs in item i's BS_FLAG_* bits (bs_sketch's rules).
 * bs_batch_autotune  runs the batch's sketches once, then times every
 *     candidate scan shape of each width (reps runs each, after a warm-up) on
 *     that width's problems, keeps the fastest and re-plans. Synchronises
 *     `stream`. Outputs hold a valid result afterwards.
 * bs_batch_run      one graph launch of the whole batch on `stream` (the
 *     graph is recorded at the first run after create or autotune).
 * bs_batch_run_eager  the same kernels enqueued directly (no graph).
 * bs_batch_shapes   writes up to cap shapes (one per distinct width,
 *     ascending N) and returns the number of widths.
 * bs_batch_graph_nodes  nodes of the recorded graph (0 before the first run).
 * Calls on one handle must not overlap; the workspace must outlive it.
 */
typedef struct {
  const int32_t* indptr;
  const int32_t* indices;
  int64_t n_rows, nnz;
  const int32_t* q_indptr;
  const int32_t* q_indices;
  int64_t n_queries, q_nnz;
  const int32_t* pi;
  int64_t d;
  int32_t N, k;
  uint64_t* sketches;
  int32_t* popcounts;
  uint64_t* q_sketches;
  int32_t* q_popcounts;
  int32_t* out_idx;
  float* out_score;
} bs_batch_item;

typedef struct {
  int32_t N, qpl, waves;
  float ms;
} bs_batch_shape;

typedef struct bs_batch bs_batch;

size_t bs_batch_workspace_size(const bs_batch_item* items, int32_t n_items);
bs_status bs_batch_create(const bs_batch_item* items, int32_t n_items, int32_t measure,
                          const bs_batch_shape* shapes, int32_t n_shapes, void* workspace,
                          size_t workspace_bytes, int32_t* err_flags, bs_batch** out);
bs_status bs_batch_autotune(bs_batch* b, int32_t reps, void* stream);
bs_status bs_batch_run(bs_batch* b, void* stream);
bs_status bs_batch_run_eager(bs_batch* b, void* stream);
int32_t bs_batch_shapes(const bs_batch* b, bs_batch_shape* out, int32_t cap);
int32_t bs_batch_graph_nodes(const bs_batch* b);
void bs_batch_destroy(bs_batch* b);

/*
 * bs_pair_popcount — <a_s, b_s> = |A[ia[i]] AND B[ib[i]]| (Algorithm 1,
 * second step) for a list of n_pairs row pairs.
 *   ia, ib    int32[n_pairs] row indices into A (nA rows) and B (nB rows).
 *   out       int32[n_pairs].
 *   err_flag  int32[1] or NULL: set to 1 (atomic OR) if an index is out of
 *             range; that pair's output is 0.
 */
bs_status bs_pair_popcount(const uint64_t* A, int64_t nA, const int32_t* ia, const uint64_t* B,
                           int64_t nB, const int32_t* ib, int64_t n_pairs, int32_t N, int32_t* out,
                           int32_t* err_flag, void* stream);

/*
 * Learned Jaccard estimator (an extension built on Algorithms 1-3, not in
 * the paper): a 4 -> 64 -> 64 -> 1 ReLU network with BF16 weights and FP32
 * accumulation, run on the vector ALU (first and last layer) and the matrix
 * cores (64 x 64 layer, v_mfma_f32_16x16x16_bf16), that predicts
 *   p = JS_closed(x_a, x_b, x_ab, N) + MLP(x_a/N, x_b/N, x_ab/N, log2(N)/16)
 * from the three sketch counts of a pair, JS_closed being the FP32 Jaccard
 * estimate of bs_topk. An all-zero output layer gives the closed form.
 * Parameters: bs_mlp_param_count() = 4545 values, in this order:
 *   W1[64][4], b1[64], W2[64][64] (row = output unit), b2[64], w3[64], b3.
 *   w        uint16[4545]  BF16 bit patterns of the parameters.
 *   xa, xb, xab  int32[n]  |a_s|, |b_s|, |a_s AND b_s| of each pair.
 *   workspace    >= bs_mlp_workspace_size(n, N) bytes, 256-byte aligned.
 * bs_mlp_forward: out[i] = clamp(p_i, 0, 1) (float[n]).
 * bs_mlp_grad: the mean squared error against label (float[n], exact
 *   Jaccard) in *loss (float, may be NULL) and its gradient with respect to
 *   the parameters in grad (float[4545]); deterministic (fixed-order sums).
 * bs_mlp_train_step: the same gradient, then one Adam step (beta1 0.9,
 *   beta2 0.999, eps 1e-8, bias-corrected for 1-based `step`) on the FP32
 *   master copy `master` (float[4545]) with moments adam_m, adam_v
 *   (float[4545], zero before step 1), and w refreshed as BF16(master).
 * bs_mlp_to_bf16: w = BF16(master), round to nearest even.
 */
int32_t bs_mlp_param_count(void);
size_t bs_mlp_workspace_size(int64_t n, int32_t N);
bs_status bs_mlp_forward(const uint16_t* w, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                         int64_t n, int32_t N, float* out, void* workspace, size_t workspace_bytes,
                         void* stream);
bs_status bs_mlp_grad(const uint16_t* w, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                      const float* label, int64_t n, int32_t N, float* grad, float* loss,
                      void* workspace, size_t workspace_bytes, void* stream);
bs_status bs_mlp_train_step(float* master, uint16_t* w, float* adam_m, float* adam_v, int64_t step,
                            float lr, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                            const float* label, int64_t n, int32_t N, float* loss, void* workspace,
                            size_t workspace_bytes, void* stream);
bs_status bs_mlp_to_bf16(const float* master, uint16_t* w, void* stream);

/*
 * Kernel timing for benchmarks and profiling (off by default). While enabled,
 * every launch is bracketed by two HIP events recorded on the caller's
 * stream (so it must not be used under graph capture). bs_timing_collect
 * waits for the recorded events and adds each kernel's elapsed time to a
 * per-name total ("sketch_csr", "pair_and_popcount", "pair_estimate",
 * "topk_prep", "topk_sample", "topk_sample_select", "topk_bound",
 * "topk_scan", "topk_select", "sketch_pack");
 * it returns the number of event pairs that could not be read.
 * bs_timing_get returns 1 and the total milliseconds and launch count for a
 * name, or 0 if the name has not been timed. Process-wide, thread-safe.
 */
int bs_timing_enable(int on);
int bs_timing_collect(void);
void bs_timing_reset(void);
int bs_timing_get(const char* name, double* total_ms, int64_t* count);

/*
 * Testing hook, not for production callers: bs_topk keeps at most
 * `slab_capacity` candidate slots per (query, corpus slab) (0 sends every
 * query with a candidate outside the sample to the whole-corpus fallback)
 * and selects at most `lds_keys` candidates in LDS (larger sets are
 * compacted and selected in place in the workspace). Negative values
 * restore the automatic sizes. Lets tests drive the overflow and in-place
 * paths, which must return the same result. Applies to the calling host
 * thread only (each thread has its own setting). Returns 0.
 */
int bs_debug_set_topk_limits(int64_t slab_capacity, int64_t lds_keys);

/*
 * Testing hook, not for production callers: bs_topk takes its filter
 * threshold tau as the `rank`-th best sample score when that is below the
 * automatic rank (1 makes tau the best sample score, so most queries fail the
 * select's check that at least k candidates score >= tau and are ranked by
 * the whole-corpus fallback). A rank below 1 restores the automatic choice.
 * Lets tests drive the fallback on a failed check, which must return the same
 * result. Applies to the calling host thread only. Returns 0.
 */
int bs_debug_set_topk_tau_rank(int64_t rank);

/*
 * Testing hook, not for production callers: with on = 0, bs_topk forms the
 * pair counts of its scan on the vector ALU (AND + popcount per word) even
 * where the matrix-core scan applies (N a multiple of 256, more than 64
 * queries); any other value restores the automatic choice. The two scans
 * produce the same candidates; lets tests cover both. bs_topk_workspace_size
 * follows the same choice, so size the workspace after setting it.
 * Applies to the calling host thread only. Returns 0.
 */
int bs_debug_set_topk_mma(int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* BINSKETCH_H */
