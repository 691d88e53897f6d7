/*
 * BinSketch CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the BinSketch
 * hot path computes (Pratap, Bera, Revanuru, "Efficient Sketching Algorithm
 * for Sparse Binary Data", arXiv 1910.04658). It exists to judge the GPU
 * library. Only the tests, the package smoke check and the benchmark's CPU
 * baseline may load it; the library never calls it and shares no code with it.
 *
 * Representation (Section 1.1): a binary vector is the sorted list of its set
 * indices. Rows arrive in CSR form (indptr int32[n+1], indices int32[nnz],
 * 0-based) and are normalised to sorted sets with duplicates removed, since
 * the vectors are binary.
 *
 * What is computed, each with the passage it follows:
 *   - the sketch (Section 3, Definition "BinSketch"): a_s[j] is the OR of a[i]
 *     over all i with pi(i) = j. With a held as a set this is the set image
 *     S_a = { pi(i) : i in a }, so a_s is the indicator of S_a. The oracle
 *     builds S_a as a sorted, de-duplicated list and packs bit j into 64-bit
 *     word j/64 at bit position j%64 (least significant bit first);
 *   - |a_s| (Algorithm 1, first step) as |S_a|, and <a_s, b_s> (Algorithm 1,
 *     second step) as |S_a intersect S_b| by a sorted merge — never from the
 *     packed words, never with a popcount instruction;
 *   - exact similarities by sorted merge: IP = |a n b|, Ham = |a|+|b|-2|a n b|
 *     (the number of differing positions, Section 1.1), JS = |a n b|/|a u b|
 *     (Section 2, MinHash paragraph), Cos = IP/sqrt(|a||b|) (Section 3.4);
 *   - the estimators of Algorithms 1-4 in FP64, both literally in the
 *     printed form and in the canonical form the library must reproduce (see
 *     the notes at orc_estimate_canonical);
 *   - top-k ranking by a full sort (the ranking use of Section 4.2, with a
 *     fixed k instead of a threshold).
 *
 * Readings where the paper is silent or misprinted are stated at each
 * function.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INDEX 1 /* a CSR index outside [0, d) */
#define ORC_ERR_MAP 2   /* a map value outside [0, N) */
#define ORC_ERR_INDPTR 4
#define ORC_ERR_ARG 8

static int cmp_i32(const void* x, const void* y) {
  int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

/* Sort ascending and drop repeats; returns the new length. */
static int64_t sort_unique(int32_t* v, int64_t m) {
  if (m <= 1) return m;
  qsort(v, (size_t)m, sizeof(int32_t), cmp_i32);
  int64_t w = 1;
  for (int64_t i = 1; i < m; ++i)
    if (v[i] != v[w - 1]) v[w++] = v[i];
  return w;
}

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/*
 * Normalise rows to sorted sets (binary semantics): out_len[r] = |a_r|, and
 * out_vals (capacity nnz, laid out at the row's CSR offset) holds the sorted
 * distinct indices in its first out_len[r] slots. Errors: index outside
 * [0, d), or a malformed indptr.
 */
int orc_normalize(const int32_t* indptr, const int32_t* indices, int64_t n, int64_t d,
                  int32_t* out_vals, int32_t* out_len) {
  if (n < 0 || d < 0) return ORC_ERR_ARG;
  if (n > 0 && indptr[0] != 0) return ORC_ERR_INDPTR;
  for (int64_t r = 0; r < n; ++r)
    if (indptr[r + 1] < indptr[r]) return ORC_ERR_INDPTR;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err)
  for (int64_t r = 0; r < n; ++r) {
    int64_t b = indptr[r], e = indptr[r + 1];
    for (int64_t k = b; k < e; ++k) {
      if (indices[k] < 0 || indices[k] >= d) err |= ORC_ERR_INDEX;
      out_vals[k] = indices[k];
    }
    out_len[r] = (int32_t)sort_unique(out_vals + b, e - b);
  }
  return err;
}

/*
 * The sketch as a set image (Section 3, Definition "BinSketch"):
 * S_a = sorted distinct { pi[i] : i in row }. Same layout as orc_normalize:
 * row r's image starts at indptr[r] in out_vals, out_len[r] = |S_a| = |a_s|.
 */
int orc_sketch_sets(const int32_t* indptr, const int32_t* indices, int64_t n, int64_t d,
                    const int32_t* pi, int32_t N, int32_t* out_vals, int32_t* out_len) {
  if (n < 0 || d < 0 || N <= 0) return ORC_ERR_ARG;
  if (n > 0 && indptr[0] != 0) return ORC_ERR_INDPTR;
  for (int64_t r = 0; r < n; ++r)
    if (indptr[r + 1] < indptr[r]) return ORC_ERR_INDPTR;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err)
  for (int64_t r = 0; r < n; ++r) {
    int64_t b = indptr[r], e = indptr[r + 1], m = 0;
    for (int64_t k = b; k < e; ++k) {
      int32_t i = indices[k];
      if (i < 0 || i >= d) { err |= ORC_ERR_INDEX; continue; }
      int32_t j = pi[i];
      if (j < 0 || j >= N) { err |= ORC_ERR_MAP; continue; }
      out_vals[b + m++] = j;
    }
    out_len[r] = (int32_t)sort_unique(out_vals + b, m);
  }
  return err;
}

/*
 * Pack sets into bit vectors: bit j of row r goes to word r*(N/64) + j/64,
 * bit position j%64. Requires N % 64 == 0. Words not named by any j are 0.
 */
int orc_pack(const int32_t* set_vals, const int32_t* set_start, const int32_t* set_len,
             int64_t n, int32_t N, uint64_t* out_words) {
  if (N <= 0 || N % 64 != 0 || n < 0) return ORC_ERR_ARG;
  int64_t W = N / 64;
  memset(out_words, 0, (size_t)(n * W) * sizeof(uint64_t));
  for (int64_t r = 0; r < n; ++r) {
    const int32_t* s = set_vals + set_start[r];
    for (int32_t t = 0; t < set_len[r]; ++t) {
      int32_t j = s[t];
      out_words[r * W + j / 64] |= (uint64_t)1 << (j % 64);
    }
  }
  return ORC_OK;
}

/* |x n y| for two sorted distinct lists, by merge. */
static int64_t merge_count(const int32_t* x, int64_t nx, const int32_t* y, int64_t ny) {
  int64_t i = 0, j = 0, c = 0;
  while (i < nx && j < ny) {
    if (x[i] < y[j]) ++i;
    else if (x[i] > y[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

/*
 * All-pairs intersection sizes: out[p*nB + q] = |A_p n B_q| for sorted
 * distinct lists (rows of A at a_vals + a_start[p], length a_len[p]).
 * Used both on normalised rows (giving IP = <a,b>) and on sketch images
 * (giving <a_s, b_s>, Algorithm 1 second step).
 */
int orc_intersections(const int32_t* a_vals, const int32_t* a_start, const int32_t* a_len, int64_t nA,
                      const int32_t* b_vals, const int32_t* b_start, const int32_t* b_len, int64_t nB,
                      int32_t* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t p = 0; p < nA; ++p)
    for (int64_t q = 0; q < nB; ++q)
      out[p * nB + q] = (int32_t)merge_count(a_vals + a_start[p], a_len[p], b_vals + b_start[q], b_len[q]);
  return ORC_OK;
}

/* Exact similarities from |a|, |b|, |a n b| (definitions cited at the top).
 * Zero denominators (an empty vector) give 0 for JS and Cos. */
void orc_exact_measures(int64_t na, int64_t nb, int64_t nab, double out[4]) {
  double a = (double)na, b = (double)nb, c = (double)nab;
  out[0] = c;
  out[1] = a + b - 2.0 * c;
  out[2] = (a + b - c) == 0.0 ? 0.0 : c / (a + b - c);
  out[3] = (a * b) == 0.0 ? 0.0 : c / sqrt(a * b);
}

/*
 * Algorithms 1-4 exactly as printed, in FP64, with real-valued inputs
 * (so tests can feed the expectations of Lemma 1 and recover |a|, |b|, IP):
 *   n = 1 - 1/N
 *   n_a = ln(1 - x_a/N) / ln n, n_b likewise               (Alg. 1, step 3)
 *   n_ab = n_a + n_b - ln(n^n_a + n^n_b + x_ab/N - 1)/ln n  (Alg. 1, step 4)
 *   Ham = n_a + n_b - 2 n_ab                                 (Alg. 2, read)
 *   JS  = n_ab / (n_ab + Ham)                                (Alg. 3)
 *   Cos = n_ab / sqrt(n_a n_b)                               (Alg. 4)
 * Reading of Algorithm 2: the Hamming distance of binary vectors is
 * |a| + |b| - 2 IP (it counts the positions where exactly one is set); the
 * identity printed in Section 3.2 drops the factor 2, which would make Ham the
 * union size, Alg. 3 half the Dice coefficient, and Ham(a, a) = |a|. The
 * factor 2 keeps Section 3.3's JS = IP/(Ham + IP) equal to |a n b|/|a u b|.
 * No clamping: arguments outside the domain give NaN or infinities.
 */
void orc_estimate_literal(double xa, double xb, double xab, double N, double out[4]) {
  double n = 1.0 - 1.0 / N;
  double ln_n = log(n);
  double na = log(1.0 - xa / N) / ln_n;
  double nb = log(1.0 - xb / N) / ln_n;
  double nab = na + nb - log(pow(n, na) + pow(n, nb) + xab / N - 1.0) / ln_n;
  double ham = na + nb - 2.0 * nab;
  out[0] = nab;
  out[1] = ham;
  out[2] = nab / (nab + ham);
  out[3] = nab / sqrt(na * nb);
}

/*
 * The canonical estimator the library reproduces, FP64.
 *
 * Let T(x) = ln(1 - x/N) / ln(1 - 1/N), the set-size estimate of Algorithm 1
 * step 3. Since n^T(x) = 1 - x/N exactly, Algorithm 1 step 4 becomes
 *   n_ab = T(x_a) + T(x_b) - T(x_u),  x_u = x_a + x_b - x_ab = |a_s OR b_s|,
 * the same number in exact arithmetic (inclusion-exclusion on the sketch of
 * the union). Saturation (the paper is silent): a count equal to N makes the
 * logarithm infinite, so each of x_a, x_b, x_u is clamped to N-1 before T.
 * Negative or out-of-range estimates are returned as they are. Zero
 * denominators (an empty sketch) give 0 for JS and Cos.
 *   s   = T_a + T_b
 *   ip  = s - T_u
 *   ham = s - 2 ip
 *   js  = ip / (ip + ham)       (0 if ip + ham == 0)
 *   cos = ip / sqrt(T_a T_b)    (0 if T_a T_b == 0)
 */
static double T64(int64_t x, int64_t N) {
  if (x > N - 1) x = N - 1;
  if (x <= 0) return 0.0;
  return log(1.0 - (double)x / (double)N) / log(1.0 - 1.0 / (double)N);
}

void orc_estimate_canonical(int64_t xa, int64_t xb, int64_t xab, int64_t N, double out[4]) {
  int64_t xu = xa + xb - xab;
  double Ta = T64(xa, N), Tb = T64(xb, N), Tu = T64(xu, N);
  double s = Ta + Tb;
  double ip = s - Tu;
  double ham = s - 2.0 * ip;
  double den = ip + ham;
  double pr = Ta * Tb;
  out[0] = ip;
  out[1] = ham;
  out[2] = den == 0.0 ? 0.0 : ip / den;
  out[3] = pr == 0.0 ? 0.0 : ip / sqrt(pr);
}

/*
 * The same estimator in FP32, used only to rank (top-k): T32(x) is T(x)
 * computed in FP64 and rounded to float; every later operation is one IEEE
 * float operation in the order written at orc_estimate_canonical.
 */
static float T32(int64_t x, int64_t N) { return (float)T64(x, N); }

float orc_score_f32(int64_t xa, int64_t xb, int64_t xab, int64_t N, int measure) {
  int64_t xu = xa + xb - xab;
  float Ta = T32(xa, N), Tb = T32(xb, N), Tu = T32(xu, N);
  float s = Ta + Tb;
  float ip = s - Tu;
  float two_ip = ip + ip;
  float ham = s - two_ip;
  if (measure == 0) return ip;
  if (measure == 1) return ham;
  if (measure == 2) {
    float den = ip + ham;
    return den == 0.0f ? 0.0f : ip / den;
  }
  float pr = Ta * Tb;
  return pr == 0.0f ? 0.0f : ip / sqrtf(pr);
}

/* Dense estimates for all pairs from the three counts (FP64 canonical form).
 * out has 4 planes of nA*nB doubles: IP, Ham, JS, Cos. */
int orc_estimate_pairs(const int32_t* xa, int64_t nA, const int32_t* xb, int64_t nB,
                       const int32_t* xab, int32_t N, double* out) {
  int64_t P = nA * nB;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < nA; ++p)
    for (int64_t q = 0; q < nB; ++q) {
      double v[4];
      orc_estimate_canonical(xa[p], xb[q], xab[p * nB + q], N, v);
      for (int m = 0; m < 4; ++m) out[m * P + p * nB + q] = v[m];
    }
  return ORC_OK;
}

typedef struct { float s; int32_t i; } scored;

/* Hamming ranks ascending (a distance); the other measures descending.
 * Ties on the score are broken by the smaller corpus index. */
static int cmp_scored(const void* x, const void* y, void* ctx) {
  const scored* a = (const scored*)x;
  const scored* b = (const scored*)y;
  int ascending = *(const int*)ctx;
  if (a->s != b->s) {
    if (ascending) return a->s < b->s ? -1 : 1;
    return a->s > b->s ? -1 : 1;
  }
  return (a->i > b->i) - (a->i < b->i);
}

/*
 * Top-k of each query against a corpus by the FP32 score of `measure`
 * (0 IP, 1 Ham, 2 JS, 3 Cos), from the sketch image sets: x_ab by merge,
 * the score by orc_score_f32, then a full sort of all nC scores.
 * out_idx/out_score: [nQ][k]; k must be <= nC.
 */
int orc_topk(const int32_t* q_vals, const int32_t* q_start, const int32_t* q_len, int64_t nQ,
             const int32_t* c_vals, const int32_t* c_start, const int32_t* c_len, int64_t nC,
             int32_t N, int measure, int32_t k, int32_t* out_idx, float* out_score) {
  if (k < 0 || k > nC || measure < 0 || measure > 3) return ORC_ERR_ARG;
  int ascending = (measure == 1);
  int err = 0;
#pragma omp parallel reduction(| : err)
  {
    scored* buf = (scored*)malloc(sizeof(scored) * (size_t)(nC > 0 ? nC : 1));
    if (!buf) err |= ORC_ERR_ARG;
#pragma omp for schedule(dynamic, 1)
    for (int64_t p = 0; p < nQ; ++p) {
      if (!buf) continue;
      for (int64_t q = 0; q < nC; ++q) {
        int64_t xab = merge_count(q_vals + q_start[p], q_len[p], c_vals + c_start[q], c_len[q]);
        buf[q].s = orc_score_f32(q_len[p], c_len[q], xab, N, measure);
        buf[q].i = (int32_t)q;
      }
      qsort_r(buf, (size_t)nC, sizeof(scored), cmp_scored, &ascending);
      for (int32_t t = 0; t < k; ++t) {
        out_idx[p * k + t] = buf[t].i;
        out_score[p * k + t] = buf[t].s;
      }
    }
    free(buf);
  }
  return err;
}
