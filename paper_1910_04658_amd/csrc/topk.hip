// Query-vs-corpus top-k by estimated similarity on gfx950.
//
// For every query sketch and every corpus sketch the pair count
// x_ab = |q_s AND c_s| (Algorithm 1, second step) is formed on the matrix
// cores or the vector ALU and turned into the FP32 score of the chosen measure (Algorithms 1-4, the
// canonical form documented in binsketch.h). The k best corpus rows per query
// are returned ordered by (score, then smaller index). The paper ranks by a
// similarity threshold (Section 4.2); a fixed k is the serving form of it.
//
// Selection without a global sort, in three passes (five launches; the
// fallback runs inside the third):
//  1. sample: per query (one block), score a strided sample of S corpus rows,
//     find the kt-th best score tau among them by an LDS radix select, append
//     the sample rows scoring >= tau to the query's candidate list, and store
//     per-query constants for the filter below. kt <= k is the smallest rank
//     at which more than kt - 1 sample rows beat the true k-th best row with
//     probability below 1e-9 (a Poisson tail; kt = k when the sample is the
//     corpus), so tau is almost always <= the true k-th best score and the
//     candidates are about kt * nC / S rather than k * nC / S.
//  2. scan: every other (query, corpus row) pair. For N a multiple of 256 the
//     pair counts of a query batch against the corpus are formed on the
//     matrix cores as a product of 0/1 matrices (FP4 operands, exact FP32
//     counts); otherwise lanes hold queries (words in VGPRs) and corpus rows
//     arrive on the scalar unit. Instead of evaluating the score (an IEEE
//     division per pair) both test x_ab >= m[x_c][q], a per-query integer
//     bound that every pair scoring >= tau satisfies, and write the survivors
//     (about 1%) into the query's own slot range for that corpus slab, with
//     no global atomics.
//  3. select: per query, the sample and slab candidates are compacted (block
//     scan over slab counts), scored exactly as unique 64-bit keys (score
//     key, then inverted index), the k-th key found by radix select and the
//     k winners sorted (bitonic). Before that, tau is verified: with at least
//     k candidates scoring >= tau, the true k-th best score is >= tau, and
//     every row scoring >= tau is a candidate, so the selection is exact.
//  4. fallback: a query that fails that check, or has more survivors in one
//     slab than its slot range holds (e.g. massive exact ties), is ranked by
//     its select block over the whole corpus instead, streaming the rows
//     through an LDS buffer that is cut back to its k best whenever it fills
//     (no extra launch, no corpus-sized scratch). Results never depend on
//     which path ran.
#include <float.h>
#include <string.h>

#include <memory>
#include <type_traits>
#include <vector>

#include "bs_common.h"
#include "topk_group.h"

namespace bs {

void launch_lut(int32_t N, double* t64, float* t32, hipStream_t s);
void launch_row_popcount(const uint64_t* X, int64_t n, int32_t N, int32_t* pop, hipStream_t s);

namespace {

constexpr int kThreads = 256;
constexpr int kSampleMin = 2048;     // rows scored in the sample pass
constexpr int kSampleMax = 15360;  // keys fit 60 KB of LDS in the sample select
constexpr int kSampleBlocks = 1024;  // blocks of the sample-score grid, about
constexpr int kSelectLdsKeys = 6144; // candidate keys selected in LDS (else in a global buffer)
constexpr int kMaxSlabs = 2048;      // slot slabs per query at most (the select reads every count at once)
constexpr int kScanWaves = 16384;    // waves of the scan grid, about
constexpr int kRowWaves = 4096;      // waves of the row-lane scan (small batches)
constexpr int kRowsMaxQ = 64;        // largest batch of the row-lane scan
constexpr int kSplitWaves = 4;       // waves sharing one 64-query group in the word-split scan
constexpr int kSplitGridWaves = 32768; // waves of the word-split scan grid, about
constexpr int kSplitRows = 16;       // rows per partial-count exchange of the word-split scan
constexpr int kFbRowsPerThread = 2; // corpus rows per thread per step of the whole-corpus fallback
constexpr int kMmaRows = 64;         // corpus rows per wave tile of the matrix-core scan
// waves of the matrix-core scan grid, about: two rounds of the 3,072 that
// are resident at once (3 blocks of 4 waves on each of 256 CUs), so each wave
// runs several tiles and its set-up and final drain are amortised
constexpr int kMmaWaves = 6144;
constexpr int kXcds = 8;              // accelerator complex dies, one L2 each
constexpr int kMmaQCap = 512;         // survivor queue entries per wave of the matrix-core scan
constexpr int kMmaSlabRowBits = 26;   // a matrix-core scan slab holds at most 2^26 rows (offsets fit 26 bits)
constexpr int kMmaHoldChunks = 2;     // the matrix-core scan holds a group's query words in registers up to this many chunks

__host__ __device__ constexpr int64_t round_up64(int64_t x) { return (x + 63) / 64 * 64; }

struct QConst {  // per-query constants written by the sample pass
  float tau;     // (a lower bound on) the kt-th best sample score
  float Tq;      // T(|q_s|)
  float A, B, C; // filter bound: T(x_u) <= fma(sqrtTc, B, fma(s, A, C))
  int32_t xq;    // |q_s|
  uint32_t tau_key;  // tau as a selection key
  int32_t pad1;
};

struct Plan {
  int64_t S, stride;
  int64_t kt;  // rank of tau in the sample
  int64_t qpl, ngrp, nqb4, n_slabs, slab, scap, kmax;  // scan geometry
  int64_t s_rblocks, s_nqb, s_qb;                     // sample-score grid
  bool rows;                                          // row-lane scan (small batches)
  bool split;                                         // word-split scan (wide sketches)
  bool mma;                                           // matrix-core scan (replaces the two above)
  bool sel_lut;                                       // select keeps T in LDS
  int64_t lds_keys;                                   // select: candidate keys held in LDS
  size_t off_t32, off_popq, off_popc, off_qc, off_cnts, off_cands, off_scnt, off_qovf,
      off_mtab, off_skeys, total;
};

// Sample size: 2,048 rows, growing as nC/256 up to 15,360 for large corpora
// (the candidate count per query is about kt * nC / S), at most nC.
int64_t sample_rows(int64_t nC) {
  int64_t S = nC / 256;
  S = S < kSampleMin ? kSampleMin : (S > kSampleMax ? kSampleMax : S);
  return nC < S ? nC : S;
}

Plan make_plan(int64_t nQ, int64_t nC, int32_t N, int32_t k, const TopkTune& tune) {
  Plan p;
  p.S = sample_rows(nC);
  p.stride = p.S > 0 ? nC / p.S : 1;
  // tau's rank kt in the sample: the number of sample rows better than the
  // true k-th best row is about Poisson(lambda), lambda = (k - 1) S / nC, and
  // kt is the smallest rank with P(X >= kt) < 1e-9 (at most k; k when the
  // sample is the whole corpus or lambda is too large to evaluate)
  p.kt = k;
  if (p.S < nC) {
    const double lam = (double)(k - 1) * (double)p.S / (double)nC;
    double pmf = exp(-lam), cdf = pmf;
    int64_t r = 1;
    if (pmf > 0.0)
      while (r < k && 1.0 - cdf >= 1e-9) {
        pmf *= lam / (double)r;
        cdf += pmf;
        ++r;
      }
    else
      r = k;
    p.kt = r;
  }
  // scan geometry: waves of QPL x 64 queries, four per block, ~16k waves
  const int W32 = N / 32;
  const bool pow2 = (W32 & (W32 - 1)) == 0;
  p.qpl = (pow2 && W32 <= 8) ? 4 : ((pow2 && (W32 == 16 || W32 == 32)) ? 2 : 1);
  if (tune.qpl == 1 || (tune.qpl == 2 && pow2 && W32 <= 32) || (tune.qpl == 4 && pow2 && W32 <= 16))
    p.qpl = tune.qpl;
  const int64_t nqb = (nQ + 63) / 64;
  p.ngrp = (nqb + p.qpl - 1) / p.qpl;
  p.nqb4 = (p.ngrp + 3) / 4;
  // A batch of at most 64 queries leaves most lanes of a query-lane wave
  // idle and streams the corpus through the scalar unit: it is scanned with
  // corpus rows on the lanes instead, each wave over a run of 64-row tiles.
  const bool rows_ok = nQ <= kRowsMaxQ && pow2 && W32 <= 128;
  p.rows = rows_ok && tune.rows != 0;
  // Sketches of 256 or 512 words do not fit one lane's registers: four waves
  // share a 64-query group, each holding a quarter of the words.
  p.split = !p.rows && pow2 && (W32 == 256 || W32 == 512);
  // Widths of whole 256-bit chunks scan on the matrix cores (the word-split
  // sample pass is kept for the wide ones).
  p.mma = !p.rows && tune.mma != 0 && N % 256 == 0;
  if (p.rows || p.split || p.mma) p.qpl = 1;
  if (p.mma) {
    p.ngrp = nqb;
    p.nqb4 = (nqb + 3) / 4;  // a block: four 64-query groups x one slab
    // one round of resident waves for rows of one 256-bit chunk, whose tiles
    // are short enough that a second round's ramp costs more than the balance
    // it buys; two rounds otherwise
    const int64_t waves = tune.waves > 0 ? tune.waves : (W32 <= 8 ? kMmaWaves / 2 : kMmaWaves);
    const int64_t per = 4 * (p.nqb4 > 0 ? p.nqb4 : 1);  // waves per slab (a batch may hold no queries)
    int64_t n_slabs = (waves + per - 1) / per;
    if (n_slabs > kMaxSlabs) n_slabs = kMaxSlabs;
    if (n_slabs < 1) n_slabs = 1;
    const int64_t tiles = (nC + kMmaRows - 1) / kMmaRows;
    // survivor entries keep a row as its offset in the slab, in 26 bits
    const int64_t tiles_max = ((int64_t)1 << kMmaSlabRowBits) / kMmaRows;
    if ((tiles + n_slabs - 1) / n_slabs > tiles_max) n_slabs = (tiles + tiles_max - 1) / tiles_max;
    p.slab = (tiles + n_slabs - 1) / n_slabs * kMmaRows;  // whole wave tiles
  } else if (p.split) {
    p.ngrp = nqb;
    p.nqb4 = nqb;  // one block per (row slab, query group)
    const int64_t waves = tune.waves > 0 ? tune.waves : kSplitGridWaves;
    int64_t rslabs = p.ngrp > 0 ? (waves + kSplitWaves * p.ngrp - 1) / (kSplitWaves * p.ngrp) : 1;
    if (rslabs > kMaxSlabs / kSplitWaves) rslabs = kMaxSlabs / kSplitWaves;
    if (rslabs > nC) rslabs = nC;
    if (rslabs < 1) rslabs = 1;
    p.slab = (nC + rslabs - 1) / rslabs;
  } else if (p.rows) {
    const int64_t waves = tune.waves > 0 ? tune.waves : kRowWaves;
    const int64_t tiles = (nC + kWave - 1) / kWave;
    int64_t tpw = (tiles + waves - 1) / waves;
    const int64_t tpw_min = (tiles + kMaxSlabs - 1) / kMaxSlabs;
    if (tpw < tpw_min) tpw = tpw_min;
    p.slab = tpw * kWave;
  } else {
    const int64_t waves = tune.waves > 0 ? tune.waves : kScanWaves;
    int64_t n_slabs = p.ngrp > 0 ? (waves + p.ngrp - 1) / p.ngrp : 1;
    if (n_slabs > kMaxSlabs) n_slabs = kMaxSlabs;
    if (n_slabs > nC) n_slabs = nC;
    if (n_slabs < 1) n_slabs = 1;
    p.slab = (nC + n_slabs - 1) / n_slabs;
  }
  p.n_slabs = (nC + p.slab - 1) / p.slab;
  // candidate slots per (query, slab): the expected count e = rows * k / S
  // (the threshold is the k-th best of S sampled rows) plus six standard
  // deviations and a margin for ties at the threshold, so that overflow into
  // the fallback path is rare
  // (a slot slab of the word-split scan is one wave's quarter of a row slab)
  const bool wsplit = p.split && !p.mma;
  const int64_t slot_rows = wsplit ? (p.slab + kSplitWaves - 1) / kSplitWaves : p.slab;
  if (wsplit) p.n_slabs *= kSplitWaves;
  const double e = p.S > 0 ? (double)slot_rows * (double)p.kt / (double)p.S : 0.0;
  int64_t scap = (int64_t)ceil(2.0 * e + 6.0 * sqrt(e)) + 8;
  p.scap = scap < slot_rows ? scap : slot_rows;
  if (p.S >= nC) {  // the sample covers the corpus: no scan, no slabs
    p.n_slabs = 0;
    p.scap = 0;
  }
  p.kmax = p.S + p.n_slabs * p.scap;
  // sample-score grid: 256-row blocks (64 for the word-split pass) x query
  // blocks, ~2k blocks in all
  p.s_rblocks = p.split ? (p.S + kWave - 1) / kWave : (p.S + kThreads - 1) / kThreads;
  p.s_nqb = (kSampleBlocks + p.s_rblocks - 1) / p.s_rblocks;
  if (p.s_nqb > nQ) p.s_nqb = nQ;
  if (p.s_nqb < 1) p.s_nqb = 1;
  p.s_qb = (nQ + p.s_nqb - 1) / p.s_nqb;
  if (p.s_qb < 1) p.s_qb = 1;
  p.s_nqb = (nQ + p.s_qb - 1) / p.s_qb;
  if (p.mma) {  // matrix-core sample pass: blocks of 64 sampled rows x 64 queries
    p.s_rblocks = (p.S + kWave - 1) / kWave;
    p.s_qb = kWave;
    p.s_nqb = (nQ + kWave - 1) / kWave;
    if (p.s_nqb < 1) p.s_nqb = 1;
  }
  // LDS of the select kernel: room for 2.25x the expected candidate count
  // (kt * nC / S) plus 512, and T when the kernel scores raw survivors, all
  // within 60 KB. The count is not Poisson: queries whose scores tie heavily
  // at tau have many more candidates (in a 1,000 x 100,000 batch the largest
  // is 2.1x the mean), and a query that does not fit selects in place in its
  // candidate region, several times slower; the kernel's time is its slowest
  // block's
  {
    const double expect = p.S > 0 ? (double)p.kt * (double)nC / (double)p.S : 0.0;
    int64_t lk = ((int64_t)(2.25 * expect) + 512 + 255) / 256 * 256;
    p.lds_keys = lk < 1024 ? 1024 : (lk > kSelectLdsKeys ? kSelectLdsKeys : lk);
    int64_t kpad = 1;
    while (kpad < k) kpad <<= 1;
    const int64_t lut_bytes = round_up64(N + 1) * 4;
    p.sel_lut = !p.rows && N <= 2048 && (61440 - kpad * 8 - lut_bytes) / 8 >= 1024;  // (larger T costs occupancy)
    const int64_t cap = (61440 - kpad * 8 - (p.sel_lut ? lut_bytes : 0)) / 8;
    if (p.lds_keys > cap) p.lds_keys = cap;
  }
  const size_t nQs = (size_t)nQ;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  p.off_t32 = take((size_t)(N + 1) * 4);
  p.off_popq = take(nQs * 4);
  p.off_popc = take((size_t)nC * 4);
  p.off_qc = take(nQs * sizeof(QConst));
  p.off_cnts = take(nQs * 4);
  p.off_cands = take(nQs * (size_t)p.kmax * 8);  // per query: S sample slots, then n_slabs x scap
  p.off_scnt = take(nQs * (size_t)p.n_slabs * 4);
  p.off_qovf = take(nQs * 4);

  p.off_mtab = take((size_t)(N + 2) * (size_t)((nQ + 63) / 64 * 64) * 2);  // rows 0..N, then N + 1: all 65535
  p.off_skeys = take(nQs * (size_t)p.S * 4);
  p.total = o;
  return p;
}

// Larger key = better rank. Hamming ranks ascending, so its key is inverted.
template <int M>
__device__ __forceinline__ uint32_t score_key(float s) {
  const uint32_t k = float_key(s);
  return M == BS_HAMMING ? ~k : k;
}

template <int M>
__device__ __forceinline__ float key_score(uint32_t k) {
  return key_float(M == BS_HAMMING ? ~k : k);
}

// A survivor of a query-lane scan: row index, x_ab and (for N < 65536, where
// both counts fit 16 bits) the row's weight x_c, so that the select scores it
// without gathering x_c again.
__device__ __forceinline__ uint64_t raw_entry(uint32_t xab, int32_t xc, int64_t row, int32_t N) {
  const uint64_t hi = N < 65536 ? (((uint64_t)(uint32_t)xc << 16) | xab) : (uint64_t)xab;
  return (hi << 32) | (uint32_t)row;
}

// Inclusive scan over the 64 lanes of a wave (every lane active) by DPP row
// shifts within each 16-lane row, then row broadcasts across rows: six VALU
// steps with no LDS round trip (a lane with no source adds 0).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return v;
}

// Largest / smallest / total of v over a wave (every lane active), in every
// lane: the same DPP steps as the scan (a lane with no source takes the
// operation's identity), then lane 63's value. Reducing within the wave first
// keeps same-address LDS atomics, which serialize, to one per wave.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#define BS_DPP_MAX(ctrl, rows) \
  { const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rows, 0xF, false); v = o > v ? o : v; }
  BS_DPP_MAX(0x111, 0xF) BS_DPP_MAX(0x112, 0xF) BS_DPP_MAX(0x114, 0xF) BS_DPP_MAX(0x118, 0xF)
  BS_DPP_MAX(0x142, 0xA) BS_DPP_MAX(0x143, 0xC)
#undef BS_DPP_MAX
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) { return ~wave_max_u32(~v); }
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), kWave - 1);
}

// Appends to a block-shared list: each lane with `take` gets a distinct slot
// from *count, with one LDS atomic per wave (a ballot and a prefix count
// number the wave's lanes). Call with the wave's lanes active from lane 0 up
// (every lane that takes part has all lower lanes active).
__device__ __forceinline__ uint32_t wave_append(bool take, uint32_t* count) {
  const uint64_t m = __ballot(take);
  const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  uint32_t base = 0;
  if (m && threadIdx.x % kWave == 0) base = atomicAdd(count, (uint32_t)__popcll(m));
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)base) + before;
}

// Block-wide (256 threads) inclusive scan over thread order.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  v = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[wid] = v;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wid; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

// Largest v over the block (block-wide call).
__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, uint32_t* wsum) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  if (threadIdx.x % kWave == 0) wsum[threadIdx.x / kWave] = v;
  __syncthreads();
  uint32_t m = 0;
  for (int w = 0; w < kThreads / kWave; ++w) m = wsum[w] > m ? wsum[w] : m;
  __syncthreads();
  return m;
}

// Block-wide copy of n >= 1 32-bit words from global memory to LDS by
// direct-to-LDS loads: no registers, and one wait at the end, so the copy
// shares its round trip with the loads issued before it (the caller's barrier
// publishes the words). Lanes past n re-read word n - 1 into the padding:
// dst has room for n rounded up to 64 words.
// With wait = false the copy is left in flight (a later copy's wait, or the
// caller's, completes it).
__device__ __forceinline__ void copy_words_to_lds(uint32_t* dst, const uint32_t* src, int64_t n, bool wait = true) {
  const int lane = threadIdx.x % kWave;
  for (int64_t j = threadIdx.x / kWave; j * kWave < n; j += kThreads / kWave) {
    const int64_t i = j * kWave + lane;
    __builtin_amdgcn_global_load_lds(src + (i < n ? i : n - 1), dst + j * kWave, 4, 0, 0);
  }
  if (wait) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

struct KeyIdentity {
  template <typename K>
  __device__ K operator()(K key) const { return key; }
};

// MSB-first radix select of the k largest of n keys (1 <= k <= n), in
// digits of up to 8 bits from bit hb - 1 down to bit min_bit; every key has
// the bits pmask0 (those at and above hb) equal to prefix0. The keys are
// taken through xf (an order-preserving map; the result is in its terms). On return the k
// largest are exactly the keys with (key & *pmask_out) >= prefix (the return
// value) when min_bit is 0: either every digit was resolved (prefix is then
// the k-th largest key itself) or, with `early`, the bin holding the k-th
// key held exactly the keys still needed. Digits below min_bit are not
// resolved: the result is then the lower edge of the bin holding the k-th
// key, a lower bound on it. `keys` may be in LDS or global memory; `hist`
// holds 2 x 256 counters used in turn (the wave that scans one clears the
// other), so a pass costs two block barriers. With `unique` (no two keys
// equal), once the bin holding the k-th key has at most 2 KB of keys they
// are gathered into `hist` and the one with exactly need - 1 larger keys
// among them is the k-th key: one gather and one count instead of the
// remaining passes (prefix is then that key and *pmask_out all ones).
// Block-wide call.
template <typename K, typename Xf = KeyIdentity>
__device__ K radix_select_kth(const K* keys, int64_t n, int64_t k, uint32_t* hist, K* bcast_prefix,
                              int64_t* bcast_need, K* pmask_out, bool early, int hb, K prefix0, K pmask0,
                              int min_bit, Xf xf = Xf(), bool unique = false) {
  constexpr uint32_t kFinish = 2 * kThreads * 4 / sizeof(K);  // keys that fit hist
  __shared__ int done;
  __shared__ uint32_t bin_count, fin_n;
  const int t = threadIdx.x;
  K prefix = prefix0, pmask = pmask0;
  int64_t need = k;
  hist[t] = 0;
  hist[kThreads + t] = 0;
  if (t == 0) done = 0;
  __syncthreads();
  int buf = 0;
  while (hb > min_bit) {
    const int lo = hb - 8 > min_bit ? hb - 8 : min_bit;
    const uint32_t dmask = (1u << (hb - lo)) - 1u;
    uint32_t* h = hist + buf * kThreads;
    for (int64_t i = t; i < n; i += kThreads) {
      const K key = xf(keys[i]);
      if ((key & pmask) == prefix) atomicAdd(&h[(uint32_t)(key >> lo) & dmask], 1u);
    }
    __syncthreads();
    if (t < kWave) {  // one wave scans the 256 bins from the top, four per lane
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = h[255 - 4 * t - j];
        sum += c[j];
      }
      const uint32_t incl = wave_incl_scan(sum);
      uint32_t e = incl - sum;  // keys in the bins above this lane's
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if ((int64_t)e < need && (int64_t)(e + c[j]) >= need) {
          *bcast_prefix = prefix | ((K)(uint32_t)(255 - 4 * t - j) << lo);
          *bcast_need = need - (int64_t)e;
          bin_count = c[j];
          if (early && (int64_t)(e + c[j]) == need) done = 1;
        }
        e += c[j];
        hist[(buf ^ 1) * kThreads + 4 * t + j] = 0;
      }
    }
    __syncthreads();
    prefix = *bcast_prefix;
    need = *bcast_need;
    pmask |= (K)dmask << lo;
    if (done) break;  // block-uniform; set only before the barrier above
    if (unique && lo > min_bit && bin_count <= kFinish && bin_count <= kThreads) {  // block-uniform
      K* list = reinterpret_cast<K*>(hist);  // both count buffers are done with
      if (t == 0) fin_n = 0;
      __syncthreads();
      for (int64_t i = t; i < n; i += kThreads) {
        const K key = xf(keys[i]);
        const bool in = (key & pmask) == prefix;
        const uint32_t slot = wave_append(in, &fin_n);
        if (in) list[slot] = key;
      }
      __syncthreads();
      const uint32_t m = fin_n;  // == bin_count
      if ((uint32_t)t < m) {
        const K kt = list[t];
        uint32_t r = 0;
        for (uint32_t j = 0; j < m; ++j) r += list[j] > kt ? 1u : 0u;
        if ((int64_t)r == need - 1) *bcast_prefix = kt;
      }
      __syncthreads();
      prefix = *bcast_prefix;
      pmask = ~(K)0;
      break;
    }
    hb = lo;
    buf ^= 1;
  }
  if (pmask_out) *pmask_out = pmask;
  return prefix;
}

// Smallest and largest of n keys (block-wide call; the keys widened to 64
// bits). The radix selects start at the highest digit where they differ.
template <typename K>
__device__ void block_key_range(const K* keys, int64_t n, uint64_t* lo_out, uint64_t* hi_out) {
  __shared__ uint64_t wmin[kThreads / kWave], wmax[kThreads / kWave];
  uint64_t lo = ~(uint64_t)0, hi = 0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const uint64_t key = keys[i];
    lo = key < lo ? key : lo;
    hi = key > hi ? key : hi;
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  if (threadIdx.x % kWave == 0) {
    wmin[threadIdx.x / kWave] = lo;
    wmax[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  lo = wmin[0];
  hi = wmax[0];
#pragma unroll
  for (int w = 1; w < kThreads / kWave; ++w) {
    lo = wmin[w] < lo ? wmin[w] : lo;
    hi = wmax[w] > hi ? wmax[w] : hi;
  }
  *lo_out = lo;
  *hi_out = hi;
}


struct TopkArgs {
  const uint64_t* __restrict__ Q;  // [nQ][W64]
  const uint64_t* __restrict__ C;  // [nC][W64]
  const float* __restrict__ t32;   // T(0..N)
  const int32_t* __restrict__ popQ;
  const int32_t* __restrict__ popC;
  QConst* __restrict__ qc;
  float* __restrict__ t32w;        // null, or: the sample pass builds T itself and stores it here (= t32)
  int32_t* __restrict__ cnts;      // [nQ] sample candidates per query
  uint64_t* __restrict__ cands;    // [nQ][kmax]: S sample candidates (keys), then scap planes of n_slabs
                                   // scan candidates (slot c of slab s at S + c*n_slabs + s; keys from
                                   // the row-lane scan, raw (x_c, x_ab, row) entries from the query-lane
                                   // scans); compacted into keys by the select
  int32_t* __restrict__ scnt;      // [nQ][n_slabs] scan candidates per slab
  int32_t* __restrict__ qovf;      // [nQ] 1 when a slab's slots overflowed
  uint16_t* __restrict__ mtab;     // [N+2][nQp] pair-count thresholds (row N+1: 65535)
  uint32_t* __restrict__ skeys;    // [nQ][S] sample keys
  int32_t* __restrict__ out_idx;   // [nQ][k]
  float* __restrict__ out_score;   // [nQ][k] or null
  int64_t nQ, nQp, nC, S, stride, n_slabs, slab, nqb4, scap, kmax, lds_keys;
  int64_t s_rblocks, s_nqb, s_qb;  // sample-score grid: row blocks x query blocks of s_qb queries
  int32_t N, W32, k, kpad;
  int32_t kt;                      // rank of tau in the sample (<= k)
  int32_t qpl, rows, split;        // scan variant: queries per lane, row-lane scan, word-split scan
  int32_t mma;                     // matrix-core scan (split then only selects the sample kernel)
  int32_t sel_lut;                 // the select keeps T in LDS
  int32_t sel_per;                 // slabs per thread in the select (4, or 8 past 1024 slabs)
};

// Member-wise copy through the constant address space, so that the fields of
// a per-corpus argument block read by a grouped kernel land in scalar
// registers (the hot loops take their row pointers from them).
__device__ __forceinline__ TopkArgs load_args(const TopkArgs* p) {
  const cptr<TopkArgs> c = as_const(p);
  TopkArgs a;
  a.Q = c->Q;
  a.C = c->C;
  a.t32 = c->t32;
  a.popQ = c->popQ;
  a.popC = c->popC;
  a.qc = c->qc;
  a.t32w = c->t32w;
  a.cnts = c->cnts;
  a.cands = c->cands;
  a.scnt = c->scnt;
  a.qovf = c->qovf;
  a.mtab = c->mtab;
  a.skeys = c->skeys;
  a.out_idx = c->out_idx;
  a.out_score = c->out_score;
  a.nQ = c->nQ;
  a.nQp = c->nQp;
  a.nC = c->nC;
  a.S = c->S;
  a.stride = c->stride;
  a.n_slabs = c->n_slabs;
  a.slab = c->slab;
  a.nqb4 = c->nqb4;
  a.scap = c->scap;
  a.kmax = c->kmax;
  a.lds_keys = c->lds_keys;
  a.s_rblocks = c->s_rblocks;
  a.s_nqb = c->s_nqb;
  a.s_qb = c->s_qb;
  a.N = c->N;
  a.W32 = c->W32;
  a.k = c->k;
  a.kpad = c->kpad;
  a.kt = c->kt;
  a.qpl = c->qpl;
  a.rows = c->rows;
  a.split = c->split;
  a.mma = c->mma;
  a.sel_lut = c->sel_lut;
  a.sel_per = c->sel_per;
  return a;
}

// x_ab of one query (words in LDS) against one corpus row (global).
__device__ __forceinline__ int32_t and_popcount_row(const uint64_t* qw, const uint64_t* __restrict__ crow,
                                                    int W64) {
  uint32_t acc = 0;
  int w = 0;
  for (; w + 2 <= W64; w += 2) {
    const uint64_t c0 = crow[w], c1 = crow[w + 1];
    acc += (uint32_t)__builtin_popcountll(qw[w] & c0) + (uint32_t)__builtin_popcountll(qw[w + 1] & c1);
  }
  if (w < W64) acc += (uint32_t)__builtin_popcountll(qw[w] & crow[w]);
  return (int32_t)acc;
}

template <int M>
__device__ QConst make_qconst(float tau, float Tq, int32_t xq) {
  const float d16 = 1.52587890625e-05f;  // 2^-16 relative slack
  const float d20 = 9.5367431640625e-07f;  // 2^-20
  QConst c;
  c.tau = tau;
  c.Tq = Tq;
  c.xq = xq;
  c.tau_key = 0;
  c.pad1 = 0;
  const float at = fabsf(tau);
  if (M == BS_JACCARD) {
    // js >= tau  =>  T_u <= s / (1 + tau - delta)
    const float den = 1.0f + tau - d16;
    c.A = den > 0.0f ? (1.0f / den) * (1.0f + d20) : FLT_MAX;
    c.B = 0.0f;
    c.C = d20;
  } else if (M == BS_IP) {
    // ip >= tau  =>  T_u <= s - tau (+ slack)
    c.A = 1.0f + d16;
    c.B = 0.0f;
    c.C = -tau + d16 * at + d20;
  } else if (M == BS_HAMMING) {
    // ham <= tau  =>  T_u <= (s + tau) / 2 (+ slack)
    c.A = 0.5f + d16;
    c.B = 0.0f;
    c.C = 0.5f * tau + d16 * at + d20;
  } else {
    // cos >= tau  =>  T_u <= s - tau sqrt(T_q T_c) (+ slack)
    c.A = 1.0f + d16;
    c.B = (-tau + d16 * at) * sqrtf(Tq);
    c.C = d20;
  }
  return c;
}

// ---- pass 1: sample ---------------------------------------------------------
// 1a. Exact keys of every (query, sample row) pair: lanes hold 64 consecutive
// sample rows (every stride-th corpus row, words in VGPRs), queries arrive on
// the scalar unit, and the keys of one query land in 64 consecutive slots.
// W32T: words per row when it is a compile-time constant, else 0 (generic).
template <int M, int W32T, bool LDS_LUT>
__device__ __forceinline__ void sample_scores_body(const TopkArgs& a, int64_t bx, int64_t by) {
  extern __shared__ float lut_s[];
  const float* lut = a.t32;
  if (LDS_LUT) {
    if (a.t32w) {  // small N: every block evaluates T, the first also stores it for the later passes
      for (int x = threadIdx.x; x <= a.N; x += kThreads) {
        const float v = (float)t_value(x, a.N);
        lut_s[x] = v;
        if (bx == 0 && by == 0) a.t32w[x] = v;
      }
    } else {
      copy_words_to_lds(reinterpret_cast<uint32_t*>(lut_s), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
    }
    __syncthreads();
    lut = lut_s;
  }
  const int64_t i = bx * kThreads + threadIdx.x;  // sample index
  const int64_t q_begin = by * a.s_qb;
  const int64_t q_end = q_begin + a.s_qb < a.nQ ? q_begin + a.s_qb : a.nQ;
  const bool i_ok = i < a.S;
  const int64_t row = (i_ok ? i : a.S - 1) * a.stride;
  const int W32 = W32T ? W32T : a.W32;
  const uint32_t* crow = reinterpret_cast<const uint32_t*>(a.C) + (size_t)row * W32;
  const int32_t xc = a.popC[row];
  const float Tc = lut[xc];
  constexpr int R = W32T ? W32T : 2;
  uint32_t cw[R];
  if (W32T) {
#pragma unroll
    for (int w = 0; w < R; ++w) cw[w] = crow[w];
  }
  const uint32_t* Q32 = reinterpret_cast<const uint32_t*>(a.Q);
  const cptr<int32_t> popQ = as_const(a.popQ);
  auto emit = [&](int64_t q, uint32_t acc, int32_t xq) {
    const float sc = score_f32<M>(lut[xq], Tc, lut[xq + xc - (int32_t)acc]);
    if (i_ok) a.skeys[(size_t)q * a.S + i] = score_key<M>(sc);
  };
  if (W32T && W32T <= 32) {
    // query words on the scalar unit, fetched one query ahead into two
    // register sets used in turn (no fetched word is moved; two sets of up
    // to 32 words fit the scalar register file)
    uint32_t qw[2][R];
    int32_t xq[2];
    auto fetch = [&](int b, int64_t q) {
      const cptr<uint32_t> qrow = as_const(Q32 + (size_t)q * W32T);
#pragma unroll
      for (int w = 0; w < R; ++w) qw[b][w] = qrow[w];
      xq[b] = popQ[q];
    };
    auto count = [&](int b) {
      uint32_t acc = 0;
#pragma unroll
      for (int w = 0; w < R; ++w) acc = bcnt_add(qw[b][w] & cw[w], acc);
      return acc;
    };
    if (q_begin < q_end) fetch(0, q_begin);
    for (int64_t q = q_begin; q < q_end; q += 2) {
      if (q + 1 < q_end) fetch(1, q + 1);
      __builtin_amdgcn_sched_barrier(0);
      emit(q, count(0), xq[0]);
      if (q + 1 < q_end) {
        if (q + 2 < q_end) fetch(0, q + 2);
        __builtin_amdgcn_sched_barrier(0);
        emit(q + 1, count(1), xq[1]);
      }
    }
  } else if (W32T) {
    // wider rows: the query streams in pieces of 32 words, each fetched one
    // piece ahead into two register sets used in turn (an even number of
    // pieces per row, so every query starts in set 0)
    constexpr int PS = 32, P = (W32T > 32 ? W32T : 32) / PS;
    uint32_t buf[2][PS];
    if (q_begin < q_end) {
      const cptr<uint32_t> r0 = as_const(Q32 + (size_t)q_begin * W32T);
#pragma unroll
      for (int w = 0; w < PS; ++w) buf[0][w] = r0[w];
    }
    for (int64_t q = q_begin; q < q_end; ++q) {
      const int64_t qn = q + 1 < q_end ? q + 1 : q;
      uint32_t acc = 0;
      int32_t xq = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        uint32_t(&use)[PS] = buf[p & 1];
        uint32_t(&fill)[PS] = buf[(p + 1) & 1];
        const cptr<uint32_t> nr =
            as_const(Q32 + (p + 1 < P ? (size_t)q * W32T + (p + 1) * PS : (size_t)qn * W32T));
#pragma unroll
        for (int w = 0; w < PS; ++w) fill[w] = nr[w];
        if (p == 0) xq = popQ[q];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int w = 0; w < PS; ++w) acc = bcnt_add(use[w] & cw[p * PS + w], acc);
      }
      emit(q, acc, xq);
    }
  } else {
    for (int64_t q = q_begin; q < q_end; ++q) {
      const cptr<uint32_t> qrow = as_const(Q32 + (size_t)q * W32);
      uint32_t acc = 0;
      for (int w = 0; w < W32; w += 2) {
        const uint2 c2 = *reinterpret_cast<const uint2*>(crow + w);
        acc += popc32(qrow[w] & c2.x) + popc32(qrow[w + 1] & c2.y);
      }
      emit(q, acc, popQ[q]);
    }
  }
}

// 1a'. The same for sketches of 256 or 512 words: a block of four waves
// takes 64 sample rows; wave w holds words [w*WS, (w+1)*WS) of its lane's
// row, counts that quarter against each query (scalar), and the partial
// counts meet in LDS every kSplitRows queries.
template <int M, int WS>
__device__ __forceinline__ void sample_split_body(const TopkArgs& a, int64_t bx, int64_t by) {
  extern __shared__ float lut[];  // T[0..N] (N <= 16384)
  __shared__ uint32_t part[kSplitRows][kSplitWaves][kWave];
  copy_words_to_lds(reinterpret_cast<uint32_t*>(lut), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
  __syncthreads();
  constexpr int PS = 32;
  constexpr int P = WS / PS;
  const int lane = threadIdx.x % kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t W32 = kSplitWaves * WS;
  const int64_t i = bx * kWave + lane;  // sample index
  const bool i_ok = i < a.S;
  const int64_t row = (i_ok ? i : a.S - 1) * a.stride;
  uint32_t rw[WS];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.C) + (size_t)row * W32 + wid * WS;
#pragma unroll
    for (int w = 0; w < WS; ++w) rw[w] = src[w];
  }
  const int32_t xc = a.popC[row];
  const float Tc = lut[xc];
  const int64_t q_begin = by * a.s_qb;
  const int64_t q_end = q_begin + a.s_qb < a.nQ ? q_begin + a.s_qb : a.nQ;
  const uint32_t* Q32 = reinterpret_cast<const uint32_t*>(a.Q) + wid * WS;
  for (int64_t q0 = q_begin; q0 < q_end; q0 += kSplitRows) {
    for (int r = 0; r < kSplitRows; ++r) {
      const int64_t q = q0 + r < q_end ? q0 + r : q_end - 1;
      uint32_t acc = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const cptr<uint32_t> qw = as_const(Q32 + (size_t)q * W32 + p * PS);
#pragma unroll
        for (int w = 0; w < PS; ++w) acc = bcnt_add(qw[w] & rw[p * PS + w], acc);
      }
      part[r][wid][lane] = acc;
    }
    __syncthreads();
    for (int r = wid; r < kSplitRows; r += kSplitWaves) {
      const int64_t q = q0 + r;
      if (q >= q_end) break;  // wave-uniform
      int32_t x = 0;
#pragma unroll
      for (int w = 0; w < kSplitWaves; ++w) x += (int32_t)part[r][w][lane];
      const int32_t xq = as_const(a.popQ)[q];
      const float sc = score_f32<M>(lut[xq], Tc, lut[xq + xc - x]);
      if (i_ok) a.skeys[(size_t)q * a.S + i] = score_key<M>(sc);
    }
    __syncthreads();
  }
}

// Compare-exchange into descending order, and Batcher's odd-even merge
// sorting networks for 4 and 8 keys in registers.
__device__ __forceinline__ void cx_desc(uint32_t& x, uint32_t& y) {
  const uint32_t hi = x > y ? x : y, lo = x > y ? y : x;
  x = hi;
  y = lo;
}
__device__ __forceinline__ void sort4_desc(uint32_t (&v)[4]) {
  cx_desc(v[0], v[1]); cx_desc(v[2], v[3]); cx_desc(v[0], v[2]); cx_desc(v[1], v[3]); cx_desc(v[1], v[2]);
}
__device__ __forceinline__ void sort8_desc(uint32_t (&v)[8]) {
  cx_desc(v[0], v[1]); cx_desc(v[2], v[3]); cx_desc(v[4], v[5]); cx_desc(v[6], v[7]);
  cx_desc(v[0], v[2]); cx_desc(v[1], v[3]); cx_desc(v[4], v[6]); cx_desc(v[5], v[7]);
  cx_desc(v[1], v[2]); cx_desc(v[5], v[6]);
  cx_desc(v[0], v[4]); cx_desc(v[1], v[5]); cx_desc(v[2], v[6]); cx_desc(v[3], v[7]);
  cx_desc(v[2], v[4]); cx_desc(v[3], v[5]);
  cx_desc(v[1], v[2]); cx_desc(v[3], v[4]); cx_desc(v[5], v[6]);
}

// The kt-th largest of S <= 2,048 keys in LDS (kt <= 64), exactly. Each wave
// takes 512 keys (8 per lane, sorted in registers) and pops its kt largest
// one at a time: the wave maximum of the lanes' heads, after which the lowest
// lane holding it drops its head. Wave 0 then pops the kt largest of the four
// waves' lists the same way (the kt largest overall are among them). Keys past
// S read as 0, the smallest key, which cannot change the kt-th largest of
// S >= kt keys. scratch: 4 x 64 words of LDS; *out: one LDS word.
constexpr int kSmallKthKeys = 8 * kThreads;
__device__ __forceinline__ uint32_t small_kth(const uint32_t* keys, int S, int kt, uint32_t* scratch, uint32_t* out) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  uint32_t v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = w * 8 * kWave + j * kWave + lane;
    v[j] = i < S ? keys[i] : 0u;
  }
  sort8_desc(v);
  uint32_t mine = 0;  // lane r: the wave's (r + 1)-th largest
  for (int r = 0; r < kt; ++r) {
    const uint32_t m = wave_max_u32(v[0]);
    const int src = __builtin_ctzll(__ballot(v[0] == m));  // some lane holds m
    if (lane == src) {
#pragma unroll
      for (int j = 0; j < 7; ++j) v[j] = v[j + 1];
      v[7] = 0u;
    }
    if (lane == r) mine = m;
  }
  scratch[w * kWave + lane] = lane < kt ? mine : 0u;
  __syncthreads();
  if (w == 0) {
    uint32_t c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = scratch[j * kWave + lane];
    sort4_desc(c);
    uint32_t tau = 0;
    for (int r = 0; r < kt; ++r) {
      const uint32_t m = wave_max_u32(c[0]);
      const int src = __builtin_ctzll(__ballot(c[0] == m));
      if (lane == src) {
        c[0] = c[1];
        c[1] = c[2];
        c[2] = c[3];
        c[3] = 0u;
      }
      tau = m;
    }
    if (lane == 0) *out = tau;
  }
  __syncthreads();
  return *out;
}

// 1b. Per query: tau, the kt-th best sample key (exactly, in registers, for
// samples of at most 2,048 rows and kt <= 64; else a lower bound on it from an
// LDS radix select), the sample rows scoring at least tau, and the per-query
// constants of the scan filter.
template <int M>
__device__ __forceinline__ void sample_select_body(const TopkArgs& a, int64_t q) {
  extern __shared__ uint32_t keys[];  // [S rounded up to 64]
  __shared__ uint32_t hist[2 * kThreads];
  __shared__ uint32_t bprefix;
  __shared__ int64_t bneed;
  __shared__ uint32_t nsel, kmin_s, kmax_s;
  const int32_t xq = a.popQ[q];  // (arrives with the keys)
  copy_words_to_lds(keys, a.skeys + (size_t)q * a.S, a.S);
  if (threadIdx.x == 0) {
    nsel = 0;
    kmin_s = ~0u;
    kmax_s = 0;
  }
  __syncthreads();
  const float Tq = a.t32[xq];  // (used at the end: its load overlaps the selection)
  uint32_t tau_key;
  if (a.S <= kSmallKthKeys && a.kt <= kWave) {
    tau_key = small_kth(keys, (int)a.S, (int)a.kt, hist, &kmin_s);
  } else {
    // tau: the kt-th best sample key resolved to the 16 bits below the highest
    // bit where the keys differ. The lower edge of its bin is a lower bound on
    // it, which is all the filter needs: every row scoring at least tau becomes
    // a candidate, and the final selection is exact.
    uint32_t mn = ~0u, mx = 0;
    for (int64_t i = threadIdx.x; i < a.S; i += kThreads) {
      const uint32_t key = keys[i];
      mn = key < mn ? key : mn;
      mx = key > mx ? key : mx;
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    if (threadIdx.x % kWave == 0) {
      atomicMin(&kmin_s, mn);
      atomicMax(&kmax_s, mx);
    }
    __syncthreads();
    const uint32_t klo = kmin_s, khi = kmax_s;
    const uint32_t diff = klo ^ khi;
    const int hb = diff ? 32 - __clz((int)diff) : 0;
    const uint32_t pmask0 = hb >= 32 ? 0u : ~((1u << hb) - 1u);
    tau_key = radix_select_kth<uint32_t>(keys, a.S, a.kt, hist, &bprefix, &bneed, nullptr, true, hb,
                                         (uint32_t)khi & pmask0, pmask0, hb > 16 ? hb - 16 : 0);
  }
  uint64_t* cq = a.cands + (size_t)q * a.kmax;
  for (int64_t i = threadIdx.x; i < a.S; i += kThreads) {
    const bool win = keys[i] >= tau_key;
    const uint32_t slot = wave_append(win, &nsel);
    if (win) cq[slot] = ((uint64_t)keys[i] << 32) | (uint32_t)~(uint32_t)(i * a.stride);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.cnts[q] = (int32_t)nsel;
    a.qovf[q] = 0;
    QConst c = make_qconst<M>(key_score<M>(tau_key), Tq, xq);
    c.tau_key = tau_key;
    a.qc[q] = c;
  }
}

// ---- pass 2a: per-query integer thresholds ----------------------------------
// For query q and a corpus row of weight x_c, every pair scoring >= tau has
// T(x_u) <= bound(q, x_c) (make_qconst), and since the FP32 table T is
// non-decreasing that means x_u <= X = max{x : T(x) <= bound}, i.e.
//   x_ab >= m[x_c][q] = x_q + x_c - X.
// m is clamped to [0, 65535]: lowering it only admits more candidates.
// Table rows (x_c values) per block of the threshold kernel: 16, or 64 from
// N = 2048 on, where each block's copy of T (4 (N + 1) bytes) would
// otherwise outweigh its work.
__host__ __device__ constexpr int bound_rows_per_block(int32_t N) { return N >= 2048 ? 64 : 16; }

// m[x_c][q] of one query for the table rows xc[r] (r < R, xc[r] <= N + 1),
// with X = max{x in [0, N] : T[x] <= bound} (T non-decreasing), or -1. X is
// first estimated from the inverse of T(x) = ln(1 - x/N) / ln(1 - 1/N),
// x <= N (1 - exp(bound ln(1 - 1/N))), then settled against the table itself,
// which alone decides (so the estimate's rounding cannot change X): each
// round reads T[X] and T[X + 1] and moves X one step down while T[X] > bound,
// or up while T[X + 1] <= bound. The estimate is almost always exact or one
// off; a wave with a row still moving after three rounds runs the search
// below for all its rows (steps depending only on N, every read inside the
// table). Row N + 1, and every row of a query past the batch (q_ok false),
// is 65535: no count of N < 65536 reaches it.
template <int M, int R>
__device__ __forceinline__ void bound_rows(const float* lut, int32_t N, const QConst& k, bool q_ok, const int (&xc)[R],
                                           uint16_t (&m)[R]) {
  float bnd[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float Tc = lut[xc[r] < N ? xc[r] : N];
    float bound = fmaf(k.Tq + Tc, k.A, k.C);
    if (M == BS_COSINE) bound = fmaf(sqrtf(Tc), k.B, bound);
    bnd[r] = bound;
  }
  const float L = log1pf(-1.0f / (float)N);  // < 0
  int X[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float e = (float)N * (1.0f - __expf(bnd[r] * L));
    X[r] = !(e >= 0.0f) ? -1 : (e >= (float)N ? N : (int)e);  // (a NaN bound starts at -1)
  }
  bool moving = true;
  for (int round = 0; round < 4 && moving; ++round) {
    float tx[R], tn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      tx[r] = lut[X[r] > 0 ? X[r] : 0];
      tn[r] = lut[X[r] < N ? X[r] + 1 : N];
    }
    __builtin_amdgcn_sched_barrier(0);
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool down = X[r] >= 0 && !(tx[r] <= bnd[r]);
      const bool up = X[r] < N && tn[r] <= bnd[r];
      if (round < 3) X[r] += (up ? 1 : 0) - (down ? 1 : 0);
      any = any || up || down;
    }
    moving = __ballot(any) != 0;  // wave-uniform
  }
  if (moving) {  // the search, for every row of the wave's lanes
    int base[R];
#pragma unroll
    for (int r = 0; r < R; ++r) base[r] = 0;
    for (int len = N + 1; len > 1;) {  // the count of x <= X lies in [base, base + len]
      const int half = len >> 1;
      float tv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) tv[r] = lut[base[r] + half];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < R; ++r) base[r] = tv[r] <= bnd[r] ? base[r] + half : base[r];
      len -= half;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) X[r] = base[r] + (lut[base[r]] <= bnd[r] ? 1 : 0) - 1;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    m[r] = 65535;
    if (q_ok && xc[r] <= N) {
      const int64_t mm = (int64_t)k.xq + xc[r] - X[r];
      m[r] = (uint16_t)(mm < 0 ? 0 : (mm > 65535 ? 65535 : mm));
    }
  }
}

template <int M, bool LDS_LUT, int BX>
__device__ __forceinline__ void bound_body(const TopkArgs& a, int64_t bx, int64_t by) {
  extern __shared__ float lut_s[];
  const float* lut = a.t32;
  if (LDS_LUT) {
    copy_words_to_lds(reinterpret_cast<uint32_t*>(lut_s), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
    __syncthreads();
    lut = lut_s;
  }
  const int64_t qi = bx * kWave + threadIdx.x % kWave;
  if (qi >= a.nQp) return;  // block-uniform (nQp is a multiple of 64)
  QConst k = {};
  const bool q_ok = qi < a.nQ;
  if (q_ok) k = a.qc[qi];
  constexpr int RW = kThreads / kWave;
  constexpr int RPT = BX / RW;  // table rows per thread
  const int wid = threadIdx.x / kWave;
  int xc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int x = (int)by * BX + wid + r * RW;
    xc[r] = x <= a.N + 1 ? x : a.N + 1;
  }
  uint16_t m[RPT];
  bound_rows<M, RPT>(lut, a.N, k, q_ok, xc, m);
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int x = (int)by * BX + wid + r * RW;
    if (x <= a.N + 1) a.mtab[(size_t)x * a.nQp + qi] = m[r];
  }
}

// ---- pass 2b: filtered scan ----------------------------------------------------
// One wave = QPL groups of 64 queries (one query per lane per group, words in
// VGPRs) x a slab of corpus rows streamed through the scalar unit in pieces
// of PS words, each piece fetched one step ahead of its use. The four waves
// of a block take four query groups of the same slab, so they read the same
// corpus words (scalar-cache hits after the first). W32T: words per row.
template <int W32T, int QPL>
__device__ __forceinline__ void scan_body(const TopkArgs& a, int64_t bid) {
  const int64_t slab = a.slab, nqb4 = a.nqb4;
  constexpr int PS = W32T < 32 ? W32T : 32;  // words per scalar piece
  constexpr int P = W32T / PS;               // pieces per row
  const int lane = threadIdx.x % kWave, wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t sl = bid / nqb4;
  const int64_t qg0 = ((bid % nqb4) * (kThreads / kWave) + wid) * QPL;  // first 64-query group
  const int64_t c_begin = sl * slab;
  const int64_t c_end = c_begin + slab < a.nC ? c_begin + slab : a.nC;
  if (qg0 * kWave >= a.nQ || c_begin >= c_end) return;  // wave-uniform
  const uint32_t* C32 = reinterpret_cast<const uint32_t*>(a.C);
  const cptr<int32_t> popC = as_const(a.popC);

  int64_t q[QPL];
  bool q_ok[QPL];
  uint32_t qw[QPL][W32T];
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    q[j] = (qg0 + j) * kWave + lane;
    q_ok[j] = q[j] < a.nQ;
    const uint32_t* qrow = reinterpret_cast<const uint32_t*>(a.Q) + (size_t)(q_ok[j] ? q[j] : a.nQ - 1) * W32T;
#pragma unroll
    for (int w = 0; w < W32T; ++w) qw[j][w] = qrow[w];
  }
  // threshold-table columns; groups past the last one read group qg0 (masked by q_ok)
  const int64_t ngroups = a.nQp / kWave;
  const uint16_t* mt = a.mtab;
  uint32_t moff[QPL];  // byte offsets of this lane's columns in a table row
#pragma unroll
  for (int j = 0; j < QPL; ++j) moff[j] = (uint32_t)((qg0 + j < ngroups ? qg0 + j : qg0) * kWave + lane) * 2u;
  int cnt[QPL];
  uint64_t* dst[QPL];  // this (query, slab)'s slot range
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    cnt[j] = 0;
    dst[j] = a.cands + (size_t)(q_ok[j] ? q[j] : 0) * a.kmax + a.S + sl;
  }
  // row indices fit 32 bits (nC <= INT32_MAX); next_s is the next sampled
  // row of the slab, -1 once the sample ends
  const int32_t cb = (int32_t)c_begin, ce = (int32_t)c_end, stride = (int32_t)a.stride;
  const int64_t s_end64 = a.S * a.stride < a.nC ? a.S * a.stride : a.nC;
  const uint32_t s_end = (uint32_t)s_end64;
  int32_t next_s;
  {
    const int64_t n = (c_begin + a.stride - 1) / a.stride * a.stride;
    next_s = n < s_end64 ? (int32_t)n : -1;
  }

  // Scalar pipeline: the pieces of consecutive rows land alternately in two
  // register sets (the one in use and the one being fetched), so no fetched
  // word is ever moved; row weights run two rows ahead, threshold columns one.
  uint32_t buf[2][PS];
  {
    const cptr<uint32_t> r0 = as_const(C32 + (size_t)(uint32_t)cb * W32T);
#pragma unroll
    for (int w = 0; w < PS; ++w) buf[0][w] = r0[w];
  }
  // row x of the threshold table as a buffer resource (scalar registers), so
  // a lane's threshold load takes its column offset and no address arithmetic
  auto mrow = [&](int32_t x) {
    const uint16_t* r = mt + (size_t)(uint32_t)x * (uint32_t)a.nQp;
    return __builtin_amdgcn_make_buffer_rsrc((void*)r, (short)0, (int)(a.nQp * 2), 0x00020000);
  };
  auto mload = [&](__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
  };
  int32_t xcur = popC[cb];  // weight of the current row
  uint16_t m[QPL];
  {
    const auto mr = mrow(xcur);
#pragma unroll
    for (int j = 0; j < QPL; ++j) m[j] = mload(mr, moff[j]);
  }
  int32_t x2 = popC[cb + 1 < ce ? cb + 1 : cb];  // weight of the next row

  // one row; PH: register set holding the row's first piece
  auto row = [&](const int32_t c, auto ph) {
    constexpr int PH = decltype(ph)::value;
    const int32_t c1 = c + 1 < ce ? c + 1 : c;
    const int32_t c2 = c1 + 1 < ce ? c1 + 1 : c1;
    uint32_t acc[QPL];
#pragma unroll
    for (int j = 0; j < QPL; ++j) acc[j] = 0;
    int32_t x3 = 0;
    uint16_t mn[QPL];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      uint32_t(&use)[PS] = buf[(PH + p) & 1];
      uint32_t(&fill)[PS] = buf[(PH + p + 1) & 1];
      // fetch the next piece (the next row's first piece after the last one)
      const cptr<uint32_t> nr =
          as_const(C32 + (p + 1 < P ? (size_t)(uint32_t)c * W32T + (p + 1) * PS : (size_t)(uint32_t)c1 * W32T));
#pragma unroll
      for (int w = 0; w < PS; ++w) fill[w] = nr[w];
      if (p == 0) {
        x3 = popC[c2];
        const auto mr = mrow(x2);
#pragma unroll
        for (int j = 0; j < QPL; ++j) mn[j] = mload(mr, moff[j]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < QPL; ++j) {
#pragma unroll
        for (int w = 0; w < PS; ++w) acc[j] = bcnt_add(use[w] & qw[j][p * PS + w], acc[j]);
      }
    }
    const bool in_sample = c == next_s;
    if (in_sample) {
      const uint32_t n = (uint32_t)next_s + (uint32_t)stride;
      next_s = n < s_end ? (int32_t)n : -1;
    }
#pragma unroll
    for (int j = 0; j < QPL; ++j) {
      const bool take = q_ok[j] && !in_sample && acc[j] >= (uint32_t)m[j];
      if (take) {
        if ((uint32_t)cnt[j] < (uint32_t)a.scap) {  // dst[j] walks the query's slot planes
          *dst[j] = raw_entry(acc[j], xcur, c, a.N);
          dst[j] += a.n_slabs;
        }
        ++cnt[j];
      }
      m[j] = mn[j];
    }
    xcur = x2;
    x2 = x3;
  };
  if constexpr (P % 2 == 0) {  // every row starts in set 0
    for (int32_t c = cb; c < ce; ++c) row(c, std::integral_constant<int, 0>());
  } else {  // rows alternate between the sets: two rows per iteration
    for (uint32_t c = (uint32_t)cb; c < (uint32_t)ce; c += 2) {
      row((int32_t)c, std::integral_constant<int, 0>());
      if (c + 1 < (uint32_t)ce) row((int32_t)c + 1, std::integral_constant<int, 1>());
    }
  }
#pragma unroll
  for (int j = 0; j < QPL; ++j) {
    if (q_ok[j]) {
      a.scnt[(size_t)q[j] * a.n_slabs + sl] = cnt[j] < a.scap ? cnt[j] : (int32_t)a.scap;
      if (cnt[j] > a.scap) a.qovf[q[j]] = 1;
    }
  }
}

// Generic widths (N not a power of two, or N > 4096): query words re-read per
// chunk of WC words; correct for every width, tuned for none.
template <int WC>
__device__ __forceinline__ void scan_generic_body(const TopkArgs& a, int64_t bid) {
  const int64_t slab = a.slab, nqb4 = a.nqb4;
  const int lane = threadIdx.x % kWave, wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t sl = bid / nqb4;
  const int64_t qb = (bid % nqb4) * (kThreads / kWave) + wid;
  const int64_t q = qb * kWave + lane;
  const int64_t c_begin = sl * slab;
  const int64_t c_end = c_begin + slab < a.nC ? c_begin + slab : a.nC;
  if (qb * kWave >= a.nQ || c_begin >= c_end) return;
  const bool q_ok = q < a.nQ;
  const int W32 = a.W32;
  const int nchunks = W32 / WC;
  const uint32_t* qrow = reinterpret_cast<const uint32_t*>(a.Q) + (size_t)(q_ok ? q : a.nQ - 1) * W32;
  const uint32_t* C32 = reinterpret_cast<const uint32_t*>(a.C);
  const uint16_t* mt = a.mtab + q;
  int cnt = 0;
  uint64_t* dst = a.cands + (size_t)(q_ok ? q : 0) * a.kmax + a.S + sl;
  int64_t next_s = (c_begin + a.stride - 1) / a.stride * a.stride;
  const int64_t s_end = a.S * a.stride;
  for (int64_t c = c_begin; c < c_end; ++c) {
    uint32_t acc = 0;
    for (int ch = 0; ch < nchunks; ++ch) {
      uint32_t qw[WC];
#pragma unroll
      for (int w = 0; w < WC; ++w) qw[w] = qrow[ch * WC + w];
      const cptr<uint32_t> cr = as_const(C32 + (size_t)c * W32 + ch * WC);
#pragma unroll
      for (int w = 0; w < WC; ++w) acc = bcnt_add(cr[w] & qw[w], acc);
    }
    const int32_t xc = as_const(a.popC)[c];
    const uint16_t m = mt[(size_t)xc * a.nQp];
    const bool in_sample = c == next_s && c < s_end;
    if (c == next_s) next_s += a.stride;
    const bool take = q_ok && !in_sample && acc >= (uint32_t)m;
    if (take) {
      if (cnt < a.scap) dst[(size_t)cnt * a.n_slabs] = raw_entry(acc, xc, c, a.N);
      ++cnt;
    }
  }
  if (q_ok) {
    a.scnt[(size_t)q * a.n_slabs + sl] = cnt < a.scap ? cnt : (int32_t)a.scap;
    if (cnt > a.scap) a.qovf[q] = 1;
  }
}

// Word-split scan for sketches of 256 or 512 words: a block of four waves
// takes one 64-query group and one row slab. Wave w holds words
// [w*WS, (w+1)*WS) of its lane's query and counts that quarter of every row
// (rows on the scalar unit, as above); every kSplitRows rows the partial
// counts meet in LDS and wave w finishes rows w, w+4, ... of the step (sum,
// threshold test, survivor slot in its own quarter of the slab's slots).
template <int WS>
__device__ __forceinline__ void scan_split_body(const TopkArgs& a, int64_t bid) {
  __shared__ uint32_t part[kSplitRows][kSplitWaves][kWave];
  constexpr int PS = 32;  // words per scalar piece
  constexpr int P = WS / PS;
  const int lane = threadIdx.x % kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t ngrp = a.nqb4;
  const int64_t rs = bid / ngrp;  // row slab
  const int64_t g = bid % ngrp;   // query group
  const int64_t c_begin = rs * a.slab;
  const int64_t c_end = c_begin + a.slab < a.nC ? c_begin + a.slab : a.nC;
  // every virtual block has rows and queries: all waves reach every barrier
  const int64_t W32 = kSplitWaves * WS;
  const uint32_t* C32 = reinterpret_cast<const uint32_t*>(a.C) + wid * WS;
  const cptr<int32_t> popC = as_const(a.popC);
  const int64_t q = g * kWave + lane;
  const bool q_ok = q < a.nQ;
  uint32_t qw[WS];
  {
    const uint32_t* qrow = reinterpret_cast<const uint32_t*>(a.Q) + (size_t)(q_ok ? q : a.nQ - 1) * W32 + wid * WS;
#pragma unroll
    for (int w = 0; w < WS; ++w) qw[w] = qrow[w];
  }
  const int64_t ss = rs * kSplitWaves + wid;  // this wave's slot slab
  int cnt = 0;
  uint64_t* dst = a.cands + (size_t)(q_ok ? q : 0) * a.kmax + a.S + ss;
  const uint16_t* mt = a.mtab + q;  // q < nQp
  int64_t next_s = (c_begin + a.stride - 1) / a.stride * a.stride;  // next sampled row at or after the rows seen
  const int64_t s_end = a.S * a.stride;
  // The rows this wave finishes in a block of kSplitRows: with 64-word
  // quarters their weights are fetched one block ahead and their thresholds
  // at the start of the block, so both arrive while the block's counts are
  // formed (with 128-word quarters that measured slower: they are loaded
  // when the rows are finished).
  constexpr int FR = kSplitRows / kSplitWaves;
  constexpr bool PIPE = WS <= 64;
  int32_t xw[FR];
  auto fetch_weights = [&](int64_t b0, int32_t (&x)[FR]) {
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int64_t c = b0 + wid + i * kSplitWaves;
      x[i] = popC[c < c_end ? c : c_end - 1];
    }
  };
  if (PIPE) fetch_weights(c_begin, xw);
  for (int64_t c0 = c_begin; c0 < c_end; c0 += kSplitRows) {
    uint16_t mw[FR];
    int32_t xn[FR];
    if (PIPE) {
#pragma unroll
      for (int i = 0; i < FR; ++i) mw[i] = mt[(size_t)(uint32_t)xw[i] * (uint32_t)a.nQp];
      fetch_weights(c0 + kSplitRows < c_end ? c0 + kSplitRows : c0, xn);
    }
#pragma unroll 2
    for (int r = 0; r < kSplitRows; ++r) {
      const int64_t c = c0 + r < c_end ? c0 + r : c_end - 1;  // rows past the end are not finished
      uint32_t acc = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const cptr<uint32_t> cw = as_const(C32 + (size_t)c * W32 + p * PS);
#pragma unroll
        for (int w = 0; w < PS; ++w) acc = bcnt_add(cw[w] & qw[p * PS + w], acc);
      }
      part[r][wid][lane] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FR; ++i) {
      const int r = wid + i * kSplitWaves;
      const int64_t c = c0 + r;
      if (c >= c_end) break;  // wave-uniform
      uint32_t x = 0;
#pragma unroll
      for (int w = 0; w < kSplitWaves; ++w) x += part[r][w][lane];
      while (next_s < c) next_s += a.stride;
      const bool in_sample = c == next_s && c < s_end;
      const int32_t xc = PIPE ? xw[i] : popC[c];
      const uint32_t m = PIPE ? (uint32_t)mw[i] : (uint32_t)mt[(size_t)(uint32_t)xc * (uint32_t)a.nQp];
      if (q_ok && !in_sample && x >= m) {
        if ((uint32_t)cnt < (uint32_t)a.scap) {  // dst walks the query's slot planes
          *dst = raw_entry(x, xc, c, a.N);
          dst += a.n_slabs;
        }
        ++cnt;
      }
    }
    if (PIPE) {
#pragma unroll
      for (int i = 0; i < FR; ++i) xw[i] = xn[i];
    }
    __syncthreads();
  }
  if (q_ok) {
    a.scnt[(size_t)q * a.n_slabs + ss] = cnt < a.scap ? cnt : (int32_t)a.scap;
    if (cnt > a.scap) a.qovf[q] = 1;
  }
}

template <int M>
__device__ __forceinline__ uint64_t make_key(float sc, uint32_t idx) {
  return ((uint64_t)score_key<M>(sc) << 32) | (uint64_t)(~idx);
}

// Matrix-core scan. The pair counts of 32 queries x 32 corpus rows are one
// product of 0/1 matrices over the N sketch bits (x_ab = sum over bits of
// q_bit * c_bit), formed exactly on the matrix cores with FP4 (E2M1)
// operands. A 256-bit chunk of a row is held by two lanes of the wave, 16
// bytes each (lane l: row l % 32, words 4 (l / 32) .. +3 of the chunk), and
// bit class d (bits 4i + d of every word) becomes an FP4 operand by a mask
// alone: class 0 keeps nibble bit 0 (the value 0.5), class 1 bit 1 (1.0),
// class 2 bit 2 (2.0), and class 3 is shifted down three places (0.5). Each
// class is one v_mfma_scale_f32_32x32x64_f8f6f4 whose block scales make
// every product of two set bits exactly 1.0, so the FP32 accumulators hold
// exact counts (N <= 2^24). A and B take the same bit order, so the product
// is the plain AND-popcount whatever order the unit sums in. The 32 x 32
// shape does twice the work of a 16 x 16 x 128 product per instruction and
// needs a quarter of the accumulator chains for the same tile, which keeps
// the matrix cores far busier at two waves per SIMD.
//
// A wave owns one 64-query group and the rows of its slab in tiles of 64
// rows (2 x 2 products of 32 x 32, 64 accumulators per lane); the four
// waves of a block take four query groups of the same slab. The epilogue
// reads, per lane and row, the bounds m[x_c][q] of its 16 queries, one
// 32-byte run of the table row (for eight or more chunks copied to LDS
// while the tile is multiplied). Survivors are numbered through an LDS
// queue (below), no global atomics.
typedef int bs_v8i __attribute__((ext_vector_type(8)));
typedef float bs_v16f __attribute__((ext_vector_type(16)));

// The scan's accumulators start at 2^23 instead of 0. Every partial sum is
// then an integer in [2^23, 2^24), exact in FP32, and its bit pattern is
// 0x4B000000 + the count: the epilogue compares the count with its bound as
// an integer (the low 16 bits for N < 65536), with no conversion per pair.
constexpr float kCountBias = 8388608.0f;
constexpr uint32_t kCountBiasBits = 0x4B000000u;

template <int D>
__device__ __forceinline__ bs_v8i fp4_class(const uint32_t (&w)[4]) {
  bs_v8i r = {0, 0, 0, 0, 0, 0, 0, 0};  // FP4 operands use the low four words
#pragma unroll
  for (int j = 0; j < 4; ++j)
    r[j] = (int)(D == 0 ? (w[j] & 0x11111111u)
                        : D == 1 ? (w[j] & 0x22222222u) : D == 2 ? (w[j] & 0x44444444u) : ((w[j] >> 3) & 0x11111111u));
  return r;
}

// E8M0 block scale of class D: 2 for the 0.5 classes, 1, 1/2 for the 2.0 class
template <int D>
__device__ __forceinline__ bs_v16f mma_class(bs_v8i a, bs_v8i b, bs_v16f c) {
  constexpr int sc = D == 1 ? 127 : (D == 2 ? 126 : 128);
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, sc, 0, sc);
}

// Blocks are handed to the eight XCDs in turn (block b to XCD b % 8), and each
// XCD has its own L2. This renumbering gives every XCD one contiguous run of
// the `total` blocks (a bijection of [0, total)), so blocks with neighbouring
// numbers share an L2 and run at about the same time. In a persistent grouped
// launch the grid is a multiple of 8, so item-local numbers of one residue
// class still share an XCD.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t total) {
  const int64_t q = total / kXcds, r = total % kXcds;
  const int64_t x = b % kXcds, j = b / kXcds;
  return x * q + (x < r ? x : r) + j;
}

// KCT: 256-bit chunks per row when fixed at compile time (the chunk loop is
// then unrolled, which keeps the accumulators in place), 0 for any width.
template <int KCT>
__device__ __forceinline__ void scan_mma_body(const TopkArgs& a, int64_t vbid) {
  const int lane = threadIdx.x % kWave, wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int c = lane % 32, h = lane / 32;
  // the nqb4 blocks of a slab read the same corpus rows: one L2 for all of them
  const int64_t bid = xcd_contiguous(vbid, a.n_slabs * a.nqb4);
  const int64_t sl = bid / a.nqb4, qgb = bid % a.nqb4;
  const int64_t qg = qgb * (kThreads / kWave) + wid;  // 64-query group
  const int64_t c_begin = sl * a.slab;
  const int64_t c_end = c_begin + a.slab < a.nC ? c_begin + a.slab : a.nC;
  if (qg * kWave >= a.nQ || c_begin >= c_end) return;  // wave-uniform
  const int W32 = a.W32, KC = KCT > 0 ? KCT : W32 / 8;
  const int32_t ntiles = (int32_t)((c_end - c_begin + kMmaRows - 1) / kMmaRows);
  // Operands are read as a uniform base (scalar registers) plus a 32-bit lane
  // offset. A rows: a query of the group (past the batch: the last query);
  // B rows: tile row 32 ct + c (past the slab: its last row).
  const uint32_t rowb = (uint32_t)W32 * 4u;  // bytes per row
  const char* qbase = reinterpret_cast<const char*>(a.Q) + (size_t)qg * kWave * rowb;
  const char* cslab = reinterpret_cast<const char*>(a.C) + (size_t)c_begin * rowb;
  const uint32_t nrows = (uint32_t)(c_end - c_begin);
  // Query order: operand row m of 32-query tile qt is query
  // 32 qt + 16 ((m / 4) % 2) + 4 (m / 8) + m % 4 of the group. The product's
  // rows 8 j + 4 h + r (j, r = 0..3) that lane (h, c) holds are then the
  // consecutive queries 32 qt + 16 h + 4 j + r, so accumulator element e of a
  // lane is query 32 qt + 16 h + e, and its 16 bounds per row are one 32-byte
  // run of a table row.
  uint32_t qoff[2];
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    int64_t q = qg * kWave + 32 * qt + 16 * ((c / 4) % 2) + 4 * (c / 8) + c % 4;
    q = q < a.nQ ? q : a.nQ - 1;
    qoff[qt] = (uint32_t)(q - qg * kWave) * rowb + 16u * h;
  }
  // every operand address is a uniform base (scalar registers) plus a lane
  // offset below 64 rows, so a step forms no address on the vector ALU
  auto load_a = [&](int ch, uint32_t (&qa)[2][4]) {
    const char* qb = qbase + 32u * (uint32_t)ch;
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
      const uint4 v = *reinterpret_cast<const uint4*>(qb + qoff[qt]);
      qa[qt][0] = v.x;
      qa[qt][1] = v.y;
      qa[qt][2] = v.z;
      qa[qt][3] = v.w;
    }
  };
  auto tile_base = [&](int32_t tile) { return cslab + (size_t)(uint32_t)tile * kMmaRows * rowb; };
  // B lane offsets in a tile: row 32 ct + c (past the slab: its last row)
  auto tile_off = [&](int32_t tile, uint32_t (&bo)[2]) {
    const uint32_t left = nrows - (uint32_t)tile * kMmaRows;  // >= 1: tile < ntiles
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint32_t r = 32u * ct + c;
      bo[ct] = (r < left ? r : left - 1) * rowb + 16u * h;
    }
  };
  auto load_b = [&](const char* tb, int ch, const uint32_t (&bo)[2], uint32_t (&cb)[2][4]) {
    const char* bb = tb + 32u * (uint32_t)ch;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint4 v = *reinterpret_cast<const uint4*>(bb + bo[ct]);
      cb[ct][0] = v.x;
      cb[ct][1] = v.y;
      cb[ct][2] = v.z;
      cb[ct][3] = v.w;
    }
  };
  auto load_xc = [&](int32_t tile, int32_t (&xc)[2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      uint32_t r = (uint32_t)tile * kMmaRows + 32u * ct + c;
      r = r < nrows ? r : nrows - 1;
      xc[ct] = a.popC[c_begin + r];
    }
  };
  // Bounds m[x][q] of the tile's rows. A row that must yield no survivor
  // (past the slab, or a sampled row, already scored by the sample pass)
  // takes table row N + 1, which holds 65535 for every query; so do the
  // table's columns of queries past the batch. For N < 65536 a count never
  // reaches 65535, so the compare alone decides; at N = 65536 the epilogue
  // also masks rows and queries explicitly.
  // For four or more chunks the bounds of a tile (64 rows x 128 bytes) are
  // copied into the wave's LDS region by eight 16-byte-per-lane LDS-direct
  // loads issued when the tile starts, so they arrive while it is
  // multiplied. Load j, lane l: row R = 8 j + l / 8 lands at slot s = l % 8
  // and carries piece s ^ (R & 7) of the row (spreads the epilogue's reads
  // over the banks); its table row comes from lane R % 32, which holds it in
  // xb[R / 32]. Shorter tiles read the bounds from the table in the epilogue.
  __shared__ uint4 mlds[kThreads / kWave][kMmaRows * 8];
  uint4* const mw = mlds[wid];
  const uint16_t* const mq = a.mtab + qg * kWave;
  auto bounds_to_lds = [&](const int32_t (&xt)[2]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t R = 8u * j + lane / 8, piece = (lane % 8) ^ (R & 7);
      const int32_t x = __shfl(xt[j / 4], (int)(R % 32));
      const uint16_t* src = mq + (size_t)(uint32_t)x * (size_t)a.nQp + 8 * piece;
      __builtin_amdgcn_global_load_lds(src, mw + 64 * j, 16, 0, 0);
    }
  };
  const uint32_t stride = (uint32_t)a.stride;
  const int64_t s_end64 = a.S * a.stride < a.nC ? a.S * a.stride : a.nC;
  const uint32_t s_end = (uint32_t)s_end64;
  // first sampled row at or after the slab start (rows past s_end are never sampled)
  uint32_t next_s = (uint32_t)((c_begin + a.stride - 1) / a.stride * a.stride);
  // Survivors are first appended to the wave's LDS queue as entries whose
  // low word holds the query (of the group) in its top six bits and the
  // row's offset in the slab below them (a slab holds at most 2^26 rows), at
  // positions from a ballot prefix count (one queue head for the wave). The queue is drained
  // when nearly full and once at the end of the slab: an LDS atomic on the
  // query's counter gives each entry its slot s, stored at
  // cands[q * kmax + S + s * n_slabs + sl]. Slot order within a query does
  // not matter (the select orders candidates by their keys). Draining rarely
  // keeps global stores, and the waits on them, out of the tile loop.
  __shared__ uint64_t sq_lds[kThreads / kWave][kMmaQCap];
  __shared__ uint32_t sc_lds[kThreads / kWave][kWave];
  uint64_t* const squeue = sq_lds[wid];
  uint32_t* const scount = sc_lds[wid];
  scount[lane] = 0u;
  uint64_t* const cbase = a.cands + (size_t)(qg * kWave) * a.kmax + a.S + sl;
  const uint32_t scap = (uint32_t)a.scap;
  const uint32_t nsl = (uint32_t)a.n_slabs;
  uint32_t qn = 0;  // queued entries (wave-uniform)
  auto drain = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t b = 0; b < qn; b += kWave) {
      if (b + (uint32_t)lane < qn) {
        const uint64_t e = squeue[b + lane];
        const uint32_t lo = (uint32_t)e;
        const uint32_t qid = lo >> kMmaSlabRowBits;
        const uint32_t row = (uint32_t)c_begin + (lo & ((1u << kMmaSlabRowBits) - 1u));
        const uint32_t slot = atomicAdd(&scount[qid], 1u);
        if (slot < scap) cbase[(size_t)qid * a.kmax + (size_t)slot * nsl] = (e & 0xFFFFFFFF00000000ull) | row;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    qn = 0;
  };
  // At N = 65536 a count can reach the 65535 of the masked bounds: lanes of
  // queries past the batch and of rows to skip are masked out of every
  // ballot there.
  const bool explicit_mask = a.N >= 65536;
  const int32_t nrem = (int32_t)(a.nQ - qg * kWave < kWave ? a.nQ - qg * kWave : kWave);
  auto qvalid = [&](int qt, int e) -> uint64_t {
    const uint64_t lo = 32 * qt + e < nrem ? 0xffffffffull : 0ull;
    const uint64_t hi = 32 * qt + 16 + e < nrem ? 0xffffffff00000000ull : 0ull;
    return lo | hi;
  };
  const int32_t xskip = a.N + 1;  // the table row of 65535s

  // software pipeline: the operands of the next (tile, chunk) step load while
  // the current one is multiplied; the row weights of the next tile load
  // during the current tile's epilogue
  // with at most two chunks the query words stay in registers for the whole slab
  constexpr bool HOLD = KCT > 0 && KCT <= kMmaHoldChunks;
  uint32_t qh[HOLD ? KCT : 1][2][4];
  if constexpr (HOLD) {
#pragma unroll
    for (int ch = 0; ch < KCT; ++ch) load_a(ch, qh[ch]);
  }
  uint32_t qa[2][4], cb[2][4];
  if constexpr (!HOLD) load_a(0, qa);
  uint32_t boff[2];
  tile_off(0, boff);
  load_b(tile_base(0), 0, boff, cb);
  int32_t xc[2];
  load_xc(0, xc);
  // With four or more chunks a tile is long enough to hide the copy of its
  // bounds, issued by the first step after its operand loads. The epilogue
  // waits for the copy with vmcnt(VM_AFTER): the vector memory operations
  // issued after it are the operand loads of the later steps (two per step,
  // four without held query words), and they complete in order (each step
  // also waits for all earlier loads before issuing its own, which covers
  // the copy from the second step on). Width-generic code (KCT = 0) waits
  // for everything.
  constexpr bool LDSB = KCT == 0 || KCT >= 4;
  constexpr int VM_AFTER0 = (KCT > 0 ? KCT - 1 : 0) * (HOLD ? 2 : 4);
  constexpr int VM_AFTER = VM_AFTER0 > 63 ? 63 : VM_AFTER0;
  constexpr int VM_WAIT = (VM_AFTER & 0xF) | ((VM_AFTER >> 4) << 14) | (0x7 << 4) | (0xF << 8);
  for (int32_t tile = 0; tile < ntiles; ++tile) {
    // rows of this tile that yield no survivor: past the slab, or sampled
    const uint32_t r0 = (uint32_t)(c_begin + (int64_t)tile * kMmaRows);
    const uint32_t r_hi = (uint32_t)(c_begin + (int64_t)tile * kMmaRows + kMmaRows < c_end
                                         ? c_begin + (int64_t)tile * kMmaRows + kMmaRows
                                         : c_end);
    uint64_t smask = 0;
    while (next_s < r_hi && next_s < s_end) {
      smask |= 1ull << (next_s - r0);
      next_s += stride;
    }
    int32_t xb[2];  // the bound table row of each of the lane's two rows
    bool row_ok[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint32_t R = 32u * ct + c;
      row_ok[ct] = r0 + R < r_hi && !((smask >> R) & 1);
      xb[ct] = row_ok[ct] ? xc[ct] : xskip;
    }
    // the previous epilogue's reads of the bounds region are done (their
    // values were used); the first step then starts this tile's bounds on
    // their way into it
    if constexpr (LDSB) __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    if constexpr (HOLD) {  // class operands formed anew per tile (hoisted, they would take 32 registers per chunk)
#pragma unroll
      for (int ch = 0; ch < (HOLD ? KCT : 1); ++ch)
#pragma unroll
        for (int qt = 0; qt < 2; ++qt)
          asm volatile("" : "+v"(qh[ch][qt][0]), "+v"(qh[ch][qt][1]), "+v"(qh[ch][qt][2]), "+v"(qh[ch][qt][3]));
    }
    bs_v16f acc[2][2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int qt = 0; qt < 2; ++qt)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[ct][qt][e] = kCountBias;
    // the last step loads the next tile's first chunk (the last tile's last
    // step reloads itself: in bounds, unused)
    const char* const tb = tile_base(tile);
    const bool more = tile + 1 < ntiles;
    const char* const tbn = more ? tile_base(tile + 1) : tb;
    uint32_t boffn[2];
    tile_off(more ? tile + 1 : tile, boffn);
    auto step = [&](int ch, const char* nb, int nch, const uint32_t (&nbo)[2], bool first) {
      uint32_t qn4[2][4], cn[2][4];
      // The step's operands (loaded during the previous step) are complete
      // before the next ones are issued: without this wait the compiler
      // waits for everything, the loads just issued included, at the step's
      // first use of its operands.
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      if constexpr (!HOLD) load_a(nch, qn4);
      load_b(nb, nch, nbo, cn);
      if (LDSB && first) bounds_to_lds(xb);
      // keep the next step's loads ahead of this step's products (left to
      // itself the scheduler sinks them to the end of the step, and the
      // next step then waits for their whole round trip)
      __builtin_amdgcn_sched_barrier(0);
      auto klass = [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        bs_v8i A[2];
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) A[qt] = HOLD ? fp4_class<D>(qh[HOLD ? ch : 0][qt]) : fp4_class<D>(qa[qt]);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const bs_v8i B = fp4_class<D>(cb[ct]);
#pragma unroll
          for (int qt = 0; qt < 2; ++qt) acc[ct][qt] = mma_class<D>(A[qt], B, acc[ct][qt]);
        }
      };
      klass(std::integral_constant<int, 0>());
      klass(std::integral_constant<int, 1>());
      klass(std::integral_constant<int, 2>());
      klass(std::integral_constant<int, 3>());
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          if constexpr (!HOLD) qa[u][w] = qn4[u][w];
          cb[u][w] = cn[u][w];
        }
    };
    constexpr int KU = HOLD ? KCT : 1;
#pragma unroll KU
    for (int ch = 0; ch + 1 < KC; ++ch) step(ch, tb, ch + 1, boff, ch == 0);
    step(KC - 1, tbn, more ? 0 : KC - 1, boffn, KC == 1);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) boff[ct] = boffn[ct];
    if constexpr (LDSB) {
      if constexpr (KCT > 0) __builtin_amdgcn_s_waitcnt(VM_WAIT);  // this tile's bounds are in LDS
      else __builtin_amdgcn_s_waitcnt(0x0F70);                     // vmcnt(0)
    }
    // the next tile's row weights load during this tile's epilogue
    int32_t xcur[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) xcur[ct] = xc[ct];
    load_xc(tile + 1 < ntiles ? tile + 1 : tile, xc);
    // the epilogue, with explicit row and query masks (EM) only at N = 65536
    auto epilogue = [&](auto em_tag) {
      constexpr bool EM = decltype(em_tag)::value;
  #pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const uint32_t R = 32u * ct + c;
        const uint64_t rowm = EM ? __builtin_amdgcn_ballot_w64(row_ok[ct]) : ~0ull;
        // queue entry of a survivor: high word as in raw_entry, x_c << 16 |
        // x_ab (x_ab alone at N = 65536); low word its query 16 h + 32 qt + e
        // of the group above the row's offset in the slab
        uint32_t hi_t = a.N < 65536 ? (uint32_t)xcur[ct] << 16 : 0u;
        uint32_t lo_t = ((uint32_t)tile * kMmaRows + R) | (16u * h) << kMmaSlabRowBits;
        // formed anew per tile: hoisted out of the tile loop, the per-query
        // values would take 64 registers
        asm volatile("" : "+v"(lo_t), "+v"(hi_t));
  #pragma unroll
        for (int qt = 0; qt < 2; ++qt) {
          // bounds of queries 32 qt + 16 h .. + 15 for this row: pieces 4 qt + 2 h and + 1
          const uint32_t p0 = 4u * qt + 2u * h;
          uint4 mg[2];
          if constexpr (LDSB) {
            mg[0] = mw[R * 8 + (p0 ^ (R & 7))];
            mg[1] = mw[R * 8 + ((p0 + 1) ^ (R & 7))];
          } else {
            const uint4* mrow = reinterpret_cast<const uint4*>(mq + 8 * p0 + (size_t)(uint32_t)xb[ct] * (size_t)a.nQp);
            mg[0] = mrow[0];
            mg[1] = mrow[1];
          }
  #pragma unroll
          for (int e = 0; e < 16; ++e) {
            if (e % 4 == 0) {
              __builtin_amdgcn_sched_barrier(0);  // four queries at a time: short live ranges
              // room for four full ballots (one check per four queries keeps
              // the drain's code out of every query's path)
              if (qn > (uint32_t)(kMmaQCap - 4 * kWave)) drain();
            }
            const uint4 m4 = mg[e / 8];
            const uint32_t mw32 = (e % 8) / 2 == 0 ? m4.x : (e % 8) / 2 == 1 ? m4.y : (e % 8) / 2 == 2 ? m4.z : m4.w;
            const uint32_t m = e % 2 == 0 ? (mw32 & 0xffffu) : (mw32 >> 16);
            // the accumulator's bits are 0x4B000000 + x_ab (x_ab < 2^16 for
            // N < 65536: its low half)
            const uint32_t bits = __float_as_uint(acc[ct][qt][e]);
            const uint32_t x = EM ? bits - kCountBiasBits : (bits & 0xffffu);
            const bool pass = x >= m;
            uint64_t bal = __builtin_amdgcn_ballot_w64(pass);
            if (EM) bal &= rowm & qvalid(qt, e);
            if (bal) {  // wave-uniform
              const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
              if (EM ? ((bal >> lane) & 1) != 0 : pass)
                (squeue + qn)[pos] = ((uint64_t)(hi_t | x) << 32) | (lo_t + ((uint32_t)(32 * qt + e) << kMmaSlabRowBits));
              qn += (uint32_t)__popcll(bal);
            }
          }
        }
      }
    };
    if (explicit_mask) epilogue(std::true_type());
    else epilogue(std::false_type());
  }
  drain();
  // lane l reports query qg*64 + l
  const uint32_t n = scount[lane];
  const int64_t q = qg * kWave + lane;
  if (q < a.nQ) {
    a.scnt[(size_t)q * a.n_slabs + sl] = (int32_t)(n < scap ? n : scap);
    if (n > scap) a.qovf[q] = 1;
  }
}

// Sample pass on the matrix cores (the widths and batches the matrix-core
// scan takes): the exact score of every query against each of the S sampled
// rows (row i * stride) as a selection key in skeys[q][i], from the same
// FP4 products as the scan. A block takes 64 queries x 64 sampled rows and
// each of its four waves one 32 x 32 product (query tile wid / 2, row tile
// wid % 2); the counts become FP32 scores exactly as in the other sample
// kernels.
template <int M, int KCT, bool LDS_LUT>
__device__ __forceinline__ void sample_mma_body(const TopkArgs& a, int64_t bx, int64_t by) {
  extern __shared__ float lut_s[];
  const int lane = threadIdx.x % kWave, wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int c = lane % 32, h = lane / 32;
  const int64_t q0 = by * kWave + 32 * (wid / 2);  // the wave's 32 queries
  const int64_t i0 = bx * kWave + 32 * (wid % 2);  // the wave's 32 sampled rows
  const bool live = q0 < a.nQ && i0 < a.S;          // wave-uniform
  const int W32 = a.W32, KC = KCT > 0 ? KCT : W32 / 8;
  const uint32_t rowb = (uint32_t)W32 * 4u;
  // operand row c holds query q0 + 16 ((c / 4) % 2) + 4 (c / 8) + c % 4, so
  // accumulator element e of lane (h, c) is query q0 + 16 h + e (as in the
  // scan). Indices are clamped, so a wave past the batch loads in bounds.
  int64_t qr = q0 + 16 * ((c / 4) % 2) + 4 * (c / 8) + c % 4;
  qr = qr < a.nQ ? qr : a.nQ - 1;
  const int64_t irow = i0 + c;
  const int64_t crow = (irow < a.S ? irow : a.S - 1) * a.stride;
  const char* qp = reinterpret_cast<const char*>(a.Q) + (size_t)qr * rowb + 16u * h;
  const char* cp = reinterpret_cast<const char*>(a.C) + (size_t)crow * rowb + 16u * h;
  // every load first (the first G chunks of both operands and the row
  // weights), then T, so that building T overlaps the loads' round trip
  constexpr int G = 4;  // chunks loaded as one batch
  uint4 av[G], bv[G];
#pragma unroll
  for (int j = 0; j < G; ++j)
    if (j < KC) {
      av[j] = *reinterpret_cast<const uint4*>(qp + 32u * j);
      bv[j] = *reinterpret_cast<const uint4*>(cp + 32u * j);
    }
  const int32_t xc = a.popC[crow];
  // the weights of the 16 queries of the lane's accumulator elements (query
  // q0 + 16 h + e), loaded directly: two distinct addresses per load
  int32_t xqe[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t q = q0 + 16 * h + e;
    xqe[e] = a.popQ[q < a.nQ ? q : a.nQ - 1];
  }
  const float* lut = a.t32;
  if (LDS_LUT) {
    if (a.t32w) {  // small N: every block evaluates T, the first also stores it for the later passes
      // TV entries per thread evaluated side by side (independent FP64 chains)
      constexpr int TV = 5;
      for (int x0 = threadIdx.x; x0 <= a.N; x0 += TV * kThreads) {
        float v[TV];
#pragma unroll
        for (int j = 0; j < TV; ++j) {
          const int x = x0 + j * kThreads;
          v[j] = x <= a.N ? (float)t_value(x, a.N) : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < TV; ++j) {
          const int x = x0 + j * kThreads;
          if (x <= a.N) {
            lut_s[x] = v[j];
            if (bx == 0 && by == 0) a.t32w[x] = v[j];
          }
        }
      }
    } else {
      copy_words_to_lds(reinterpret_cast<uint32_t*>(lut_s), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
    }
    __syncthreads();
    lut = lut_s;
  }
  if (!live) return;  // no barrier follows
  bs_v16f acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
  for (int c0 = 0; c0 < KC; c0 += G) {
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (c0 + j < KC) {
        const uint32_t aw[4] = {av[j].x, av[j].y, av[j].z, av[j].w}, bw[4] = {bv[j].x, bv[j].y, bv[j].z, bv[j].w};
        acc = mma_class<0>(fp4_class<0>(aw), fp4_class<0>(bw), acc);
        acc = mma_class<1>(fp4_class<1>(aw), fp4_class<1>(bw), acc);
        acc = mma_class<2>(fp4_class<2>(aw), fp4_class<2>(bw), acc);
        acc = mma_class<3>(fp4_class<3>(aw), fp4_class<3>(bw), acc);
      }
    if (c0 + G < KC) {  // the next batch of chunks (wide sketches)
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (c0 + G + j < KC) {
          av[j] = *reinterpret_cast<const uint4*>(qp + 32u * (c0 + G + j));
          bv[j] = *reinterpret_cast<const uint4*>(cp + 32u * (c0 + G + j));
        }
    }
  }
  const float Tc = lut[xc];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int32_t xq = xqe[e];
    const float sc = score_f32<M>(lut[xq], Tc, lut[xq + xc - (int32_t)acc[e]]);
    const int64_t q = q0 + 16 * h + e;
    if (irow < a.S && q < a.nQ) a.skeys[(size_t)q * a.S + irow] = score_key<M>(sc);
  }
}

// Row-lane scan for batches of at most 64 queries. Each wave owns one slab:
// a run of 64-row tiles. Lane l holds row (tile + l) in VGPRs; the queries
// arrive in turn on the scalar unit, so the corpus is read from HBM exactly
// once with every lane busy. The filter is the predicate the threshold table
// encodes, T(x_u) <= bound(q, x_c), evaluated directly with T in LDS. A
// query's survivors in the slab are numbered by a wave prefix count (ballot);
// lane j of the counter register holds query j's running count. Survivors
// are stored as final selection keys (the score is at hand here).
template <int M, int W32T>
__device__ __forceinline__ void scan_rows_body(const TopkArgs& a, int64_t bid) {
  extern __shared__ float lut[];  // T[0..N]
  copy_words_to_lds(reinterpret_cast<uint32_t*>(lut), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
  __syncthreads();
  constexpr int PS = W32T < 32 ? W32T : 32;  // query words per scalar piece
  const int lane = threadIdx.x % kWave;
  const int64_t sl = bid * (kThreads / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (sl >= a.n_slabs) return;  // wave-uniform; no block barrier follows
  const int64_t r_begin = sl * a.slab;
  const int64_t r_end = r_begin + a.slab < a.nC ? r_begin + a.slab : a.nC;
  const int nQ = (int)a.nQ;
  const uint32_t stride = (uint32_t)a.stride;
  const uint32_t S = (uint32_t)a.S;
  const int32_t N = a.N;
  const uint32_t* Q32 = reinterpret_cast<const uint32_t*>(a.Q);
  const cptr<QConst> qc = as_const(a.qc);
  const cptr<int32_t> popQ = as_const(a.popQ);
  int cntv = 0;  // lane j: survivors of query j in this slab so far
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kWave) {
    const int64_t r = r0 + lane;
    const bool ok = r < r_end;
    const int64_t rr = ok ? r : r_end - 1;
    uint32_t row[W32T];
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a.C) + (size_t)rr * W32T;
      if (W32T >= 4) {
#pragma unroll
        for (int w = 0; w < W32T; w += 4) {
          const uint4 v = *reinterpret_cast<const uint4*>(src + w);
          row[w] = v.x;
          row[w + 1] = v.y;
          row[w + 2] = v.z;
          row[w + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int w = 0; w < W32T; ++w) row[w] = src[w];
      }
    }
    int32_t xc = a.popC[rr];
    xc = xc < 0 ? 0 : (xc > N ? N : xc);
    const float Tc = lut[xc];
    const float sTc = M == BS_COSINE ? sqrtf(Tc) : 0.0f;
    const uint32_t ur = (uint32_t)rr;
    const uint32_t si = ur / stride;
    const bool live = ok && !(ur == si * stride && si < S);  // sampled rows were ranked by the sample pass
    for (int q = 0; q < nQ; ++q) {
      uint32_t acc = 0;
#pragma unroll
      for (int p = 0; p < W32T / PS; ++p) {
        const cptr<uint32_t> qw = as_const(Q32 + (size_t)q * W32T + p * PS);
#pragma unroll
        for (int w = 0; w < PS; ++w) acc = bcnt_add(row[p * PS + w] & qw[w], acc);
      }
      float bound = fmaf(qc[q].Tq + Tc, qc[q].A, qc[q].C);
      if (M == BS_COSINE) bound = fmaf(sTc, qc[q].B, bound);
      int32_t xu = popQ[q] + xc - (int32_t)acc;
      xu = xu < 0 ? 0 : (xu > N ? N : xu);
      const float Tu = lut[xu];
      const bool take = live && Tu <= bound;
      const uint64_t bal = __ballot(take);
      if (bal) {
        const int base = __builtin_amdgcn_readlane(cntv, q);
        if (take) {
          const int slot = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          if (slot < a.scap) {
            const float sc = score_f32<M>(lut[popQ[q]], Tc, Tu);
            a.cands[(size_t)q * a.kmax + a.S + (size_t)slot * a.n_slabs + sl] = make_key<M>(sc, (uint32_t)rr);
          }
        }
        if (lane == q) cntv += __popcll(bal);
      }
    }
  }
  if (lane < nQ) {
    a.scnt[(size_t)lane * a.n_slabs + sl] = cntv < a.scap ? cntv : (int32_t)a.scap;
    if (cntv > a.scap) a.qovf[lane] = 1;
  }
}

// ---- pass 3: exact selection of each query's candidates -----------------------

// The k best of n unique keys (1 <= k <= n) into sel[0..k), unordered. The
// radix select runs on xf(key) (an order-preserving map), whose bits at and
// above hb equal those of prefix0 for every key. Returns the radix select's
// prefix: the winners are exactly the keys with (xf(key) & *pmask_out) >=
// prefix. Block-wide; ends with a barrier.
template <typename Xf = KeyIdentity>
__device__ uint64_t select_top(const uint64_t* keys, int64_t n, int64_t k, int hb, uint64_t prefix0, uint64_t* sel,
                               uint32_t* hist, uint64_t* bprefix, int64_t* bneed, uint32_t* nsel,
                               uint64_t* pmask_out, Xf xf = Xf()) {
  const uint64_t pmask0 = hb >= 64 ? 0 : ~((((uint64_t)1) << hb) - 1);
  uint64_t pmask = 0;
  const uint64_t kth = radix_select_kth<uint64_t, Xf>(keys, n, k, hist, bprefix, bneed, &pmask, true, hb,
                                                      prefix0 & pmask0, pmask0, 0, xf, true);
  if (threadIdx.x == 0) *nsel = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const uint64_t key = keys[i];
    const bool win = (xf(key) & pmask) >= kth;  // exactly k keys: the keys are unique
    const uint32_t slot = wave_append(win, nsel);
    if (win) sel[slot] = key;
  }
  __syncthreads();
  *pmask_out = pmask;
  return kth;
}

// Radix start for keys spanning [lo, hi]: the highest bit in which they can
// differ (the bits above are common to all).
__device__ __forceinline__ int range_top_bit(uint64_t lo, uint64_t hi) {
  const uint64_t diff = lo ^ hi;
  return diff ? 64 - __clzll((long long)diff) : 0;
}

// A candidate key (score key << 32 | ~row) as a shorter key of the same
// order: (score key - the smallest score key) << b, then (2^b - 1 - row),
// with 2^b > every row. Ties of the score are broken by the row in the low b
// bits, so the radix select resolves no bits that no key uses.
struct KeyCompress {
  uint32_t base;  // smallest score key
  int b;          // row bits
  uint32_t mask;  // 2^b - 1
  __device__ uint64_t operator()(uint64_t key) const {
    return ((uint64_t)((uint32_t)(key >> 32) - base) << b) | (uint64_t)(mask - ~(uint32_t)key);
  }
};

// The k best of n unique keys, written best first as row indices (and
// scores) of query q. Each winner's place is the number of winners above it,
// counted by its own thread over broadcast LDS reads of the winners, two keys
// per read and four independent counts (no sorting network, no barrier
// between steps).
template <int M, typename Xf = KeyIdentity>
__device__ void select_and_write(const uint64_t* keys, int64_t n, int64_t q, const TopkArgs& a, int hb,
                                 uint64_t prefix0, uint64_t* sel, uint32_t* hist, uint64_t* bprefix, int64_t* bneed,
                                 uint32_t* nsel, Xf xf = Xf()) {
  uint64_t pmask;
  select_top<Xf>(keys, n, a.k, hb, prefix0, sel, hist, bprefix, bneed, nsel, &pmask, xf);
  const int k = a.k;
  const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(sel);  // sel is 16-byte aligned (LDS base)
  for (int w = threadIdx.x; w < k; w += kThreads) {
    const uint64_t kw = sel[w];
    uint32_t r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    int j = 0;
#pragma unroll 4
    for (; j + 4 <= k; j += 4) {
      const ulonglong2 x = s2[j / 2], y = s2[j / 2 + 1];
      r0 += x.x > kw ? 1u : 0u;
      r1 += x.y > kw ? 1u : 0u;
      r2 += y.x > kw ? 1u : 0u;
      r3 += y.y > kw ? 1u : 0u;
    }
    for (; j < k; ++j) r0 += sel[j] > kw ? 1u : 0u;
    const uint32_t r = r0 + r1 + r2 + r3;
    a.out_idx[q * a.k + r] = (int32_t)(~(uint32_t)kw);
    if (a.out_score) a.out_score[q * a.k + r] = key_score<M>((uint32_t)(kw >> 32));
  }
  __syncthreads();
}

// Whole-corpus selection of query q by its own block, for a query whose
// candidate list cannot be trusted (a slab had more survivors than slots, or
// fewer than k candidates reach tau). Every corpus row is scored; the keys
// that can still be among the k best wait in an LDS buffer of
// kpad + kFbRowsPerThread * 256 keys, which is cut back to its k best
// whenever the next step's rows might not fit. After a cut only keys >= the
// cut's prefix can still be among the k best (k keys already are), so each cut
// raises the bar for the rows after it. Keys are unique (every key is
// nonzero), so the result equals one selection over all nC keys.
// LDS: sel[kpad], the buffer, the query's words.
template <int M>
__device__ void fallback_query(const TopkArgs& a, int64_t q, uint64_t* sm, uint32_t* hist, uint64_t* bprefix,
                               int64_t* bneed, uint32_t* nsel, uint32_t* wsum, uint32_t* total_s) {
  constexpr int R = kFbRowsPerThread;
  const int t = threadIdx.x;
  const int W64 = a.W32 / 2;
  uint64_t* sel = sm;
  uint64_t* buf = sm + a.kpad;
  const int64_t cap = (int64_t)a.kpad + (int64_t)R * kThreads;
  uint64_t* qw = buf + cap;
  const uint64_t* qrow = a.Q + (size_t)q * W64;
  for (int w = t; w < W64; w += kThreads) qw[w] = qrow[w];
  const int32_t xq = a.popQ[q];
  const float Tq = a.t32[xq];
  __syncthreads();
  int64_t cur = 0;   // keys in the buffer (block-uniform)
  uint64_t thr = 0;  // keys below thr cannot be among the k best
  for (int64_t base = 0; base < a.nC; base += (int64_t)R * kThreads) {
    if (cur + (int64_t)R * kThreads > cap) {  // block-uniform: cut the buffer back to its k best
      uint64_t pmask, lo, hi;
      block_key_range(buf, cur, &lo, &hi);
      thr = select_top(buf, cur, a.k, range_top_bit(lo, hi), hi, sel, hist, bprefix, bneed, nsel, &pmask);
      for (int i = t; i < a.k; i += kThreads) buf[i] = sel[i];
      cur = a.k;
      __syncthreads();
    }
    uint64_t key[R];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t i = base + (int64_t)j * kThreads + t;
      key[j] = 0;
      if (i < a.nC) {
        const int32_t xab = and_popcount_row(qw, a.C + (size_t)i * W64, W64);
        const int32_t xc = a.popC[i];
        key[j] = make_key<M>(score_f32<M>(Tq, a.t32[xc], a.t32[xq + xc - xab]), (uint32_t)i);
      }
      c += (key[j] != 0 && key[j] >= thr) ? 1u : 0u;
    }
    const uint32_t incl = block_incl_scan(c, wsum);
    if (t == kThreads - 1) *total_s = incl;
    uint32_t o = (uint32_t)cur + incl - c;
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (key[j] != 0 && key[j] >= thr) buf[o++] = key[j];
    __syncthreads();
    cur += *total_s;
  }
  uint64_t lo, hi;
  block_key_range(buf, cur, &lo, &hi);
  select_and_write<M>(buf, cur, q, a, range_top_bit(lo, hi), hi, sel, hist, bprefix, bneed, nsel);
}

template <int M>
__device__ __forceinline__ uint64_t cand_key(uint64_t e, int32_t xq, float Tq, const float* lut, const TopkArgs& a) {
  const uint32_t idx = (uint32_t)e;
  int32_t xab, xc;
  if (a.N < 65536) {  // x_c travels in the entry: no gather from popC
    xab = (int32_t)((e >> 32) & 0xFFFFu);
    xc = (int32_t)(e >> 48);
  } else {
    xab = (int32_t)(e >> 32);
    xc = a.popC[idx];
  }
  return make_key<M>(score_f32<M>(Tq, lut[xc], lut[xq + xc - xab]), idx);
}

// Select of query q. Slot entries of the query-lane scans are raw
// (x_c, x_ab, row) and are scored here (RAW); the row-lane scan and the
// sample pass store final keys. PER: slabs per thread (n_slabs <= 256 * PER).
template <int M, bool RAW, bool LUT, int PER>
__device__ __forceinline__ void select_query(const TopkArgs& a, int64_t q) {
  // sel[kpad], keys[lds_keys], then (LUT) T[0..N] as floats; or, for the
  // whole-corpus fallback, the layout of fallback_query
  extern __shared__ uint64_t sm[];
  __shared__ uint32_t hist[2 * kThreads];
  __shared__ uint32_t wsum[kThreads / kWave];
  __shared__ uint64_t bprefix;
  __shared__ int64_t bneed;
  __shared__ uint32_t nsel;
  __shared__ uint32_t total_s;
  __shared__ uint32_t above_s;
  __shared__ uint32_t smin_s, smax_s;
  constexpr int RE = 6;  // scan entries per thread read in one round (more: one by one after)
  const int t = threadIdx.x;
  uint64_t* region = a.cands + (size_t)q * a.kmax;  // S sample slots, then the slot planes
  const uint64_t* slots = region + a.S;
  // 1. first round of loads: the query's constants, the overflow flag, the
  // slab counts, the first 256 sample candidates, T into LDS. Thread t owns
  // slabs t, t + 256, ..., so the count loads are one coalesced run per wave.
  const float Tq = a.qc[q].Tq;
  const int32_t xq = a.qc[q].xq;
  const uint32_t tau_key = a.qc[q].tau_key;
  const int32_t qovf = a.qovf[q];
  const int64_t ns = a.cnts[q];
  const int32_t* sc = a.scnt + (size_t)q * a.n_slabs;
  const uint64_t s0 = t < a.S ? region[t] : 0;
  uint32_t cnt[PER], part = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = (int64_t)u * kThreads + t;
    cnt[u] = i < a.n_slabs ? (uint32_t)sc[i] : 0u;
  }
  float* lut_s = reinterpret_cast<float*>(sm + a.kpad + a.lds_keys);
  if (LUT) copy_words_to_lds(reinterpret_cast<uint32_t*>(lut_s), reinterpret_cast<const uint32_t*>(a.t32), a.N + 1);
  const float* lut = LUT ? lut_s : a.t32;
  if (t == 0) {
    above_s = 0;
    smin_s = ~0u;
    smax_s = 0;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) part += cnt[u];
  const uint32_t incl = block_incl_scan(part, wsum);  // (its barriers also publish T)
  if (t == kThreads - 1) total_s = incl;
  __syncthreads();
  if (qovf) {  // block-uniform: a slab overflowed its slots
    fallback_query<M>(a, q, sm, hist, &bprefix, &bneed, &nsel, wsum, &total_s);
    return;
  }
  const int64_t n = ns + total_s;
  uint64_t* sel = sm;
  // keys at or above tau (the check below) and the range of score keys,
  // noted as the keys are written
  const uint64_t thr = a.kt < a.k ? (uint64_t)tau_key << 32 : 0;
  uint32_t above = 0, smin = ~0u, smax = 0;
  auto note = [&](uint64_t key) {
    above += key >= thr ? 1u : 0u;
    const uint32_t sk = (uint32_t)(key >> 32);
    smin = sk < smin ? sk : smin;
    smax = sk > smax ? sk : smax;
  };
  auto key_of = [&](uint64_t e) { return RAW ? cand_key<M>(e, xq, Tq, lut, a) : e; };
  uint64_t* keys;
  if (n <= a.lds_keys) {
    // 2a. into LDS, in two steps so that every thread handles about the same
    // number of entries (slab counts vary). First each thread writes, at the
    // position of every entry of its slabs (from the count's scan), where the
    // entry lives: (slot, slab). Then, after a barrier, thread t reads
    // positions ns + t, ns + t + 256, ...: their entries arrive in one round
    // of loads, are scored, and replace their own map words.
    keys = sm + a.kpad;
    uint32_t o = (uint32_t)ns + incl - part;  // the thread's first position in the count's scan
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const uint32_t slab = (uint32_t)(u * kThreads + t);
      for (uint32_t c = 0; c < cnt[u]; ++c) keys[o + c] = ((uint64_t)c << 32) | slab;
      o += cnt[u];
    }
    for (int64_t i = t; i < ns; i += kThreads) {
      const uint64_t key = i < kThreads ? s0 : region[i];
      keys[i] = key;
      note(key);
    }
    __syncthreads();
    const uint32_t nsc = total_s;  // scan entries
    auto fetch = [&](uint32_t e) {
      const uint64_t m = keys[ns + e];
      return slots[(size_t)(m >> 32) * a.n_slabs + (uint32_t)m];
    };
    uint64_t v[RE];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const uint32_t e = (uint32_t)(r * kThreads + t);
      v[r] = e < nsc ? fetch(e) : 0;
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
      const uint32_t e = (uint32_t)(r * kThreads + t);
      if (e < nsc) {
        const uint64_t key = key_of(v[r]);
        keys[ns + e] = key;
        note(key);
      }
    }
    for (uint32_t e = RE * kThreads + t; e < nsc; e += kThreads) {
      const uint64_t key = key_of(fetch(e));
      keys[ns + e] = key;
      note(key);
    }
  } else {
    // 2b. in place, one slot plane at a time (keys in plane order). Plane
    // c's keys go to [ns + E, ns + E + n_c) with E the entries of planes
    // below c: E <= c * n_slabs and n_c <= n_slabs, so they stay below plane
    // c + 1's sources, and every read of plane c comes before a write of it.
    keys = region;
    auto slot = [&](uint32_t c, int u) { return slots[(size_t)c * a.n_slabs + (size_t)u * kThreads + t]; };
    uint32_t cm = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) cm = cnt[u] > cm ? cnt[u] : cm;
    const uint32_t cmax = block_max_u32(cm, wsum);
    uint32_t E = (uint32_t)ns;
    for (uint32_t c = 0; c < cmax; ++c) {
      uint32_t m = 0;
#pragma unroll
      for (int u = 0; u < PER; ++u) m += cnt[u] > c ? 1u : 0u;
      const uint32_t pincl = block_incl_scan(m, wsum);
      if (t == kThreads - 1) total_s = pincl;
      uint64_t w[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) w[u] = cnt[u] > c ? slot(c, u) : 0;
      __syncthreads();
      uint32_t o = E + pincl - m;
#pragma unroll
      for (int u = 0; u < PER; ++u)
        if (cnt[u] > c) {
          const uint64_t key = key_of(w[u]);
          keys[o++] = key;
          note(key);
        }
      E += total_s;
    }
    for (int64_t i = t; i < ns; i += kThreads) note(region[i]);  // the sample keys stay in place
  }
  smin = wave_min_u32(smin);
  smax = wave_max_u32(smax);
  above = wave_sum_u32(above);
  if (t % kWave == 0) {
    atomicMin(&smin_s, smin);
    atomicMax(&smax_s, smax);
    atomicAdd(&above_s, above);
  }
  __syncthreads();
  // tau check: with at least k candidates scoring >= tau the true k-th best
  // score is >= tau, and every row scoring >= tau is a candidate (with
  // kt = k, tau is a lower bound by construction and thr = 0 counts all)
  if (above_s < (uint32_t)a.k) {  // block-uniform
    fallback_query<M>(a, q, sm, hist, &bprefix, &bneed, &nsel, wsum, &total_s);
    return;
  }
  KeyCompress xf;
  xf.base = smin_s;
  xf.b = a.nC > 1 ? 32 - __clz((int)(uint32_t)(a.nC - 1)) : 0;
  xf.mask = (uint32_t)((1ull << xf.b) - 1);
  const uint32_t span = smax_s - smin_s;
  const int hb = xf.b + (span ? 32 - __clz((int)span) : 0);
  select_and_write<M>(keys, n, q, a, hb, 0, sel, hist, &bprefix, &bneed, &nsel, xf);
}

// ---- grouped launches ---------------------------------------------------------
// Every stage kernel runs a list of virtual blocks: block vb of the launch
// belongs to item i with voff[i] <= vb < voff[i + 1] and is that item's local
// block vb - voff[i]. A launch of one item carries its arguments inline
// (items == null). With fewer hardware blocks than virtual blocks the grid is
// persistent: each block walks vb = blockIdx.x, + gridDim.x, ...; every body
// returns only at points where the whole block or a whole wave is done with
// block barriers, and a barrier separates consecutive virtual blocks.
struct GroupArgs {
  const TopkArgs* items;  // [n] argument blocks in device memory, or null
  const int64_t* voff;    // [n + 1]
  int64_t total;          // virtual blocks
  int32_t n;
  TopkArgs one;           // the single item when items is null
};

__device__ __forceinline__ int64_t group_item(const GroupArgs& g, int64_t vb, TopkArgs& a) {
  if (!g.items) {
    a = g.one;
    return vb;
  }
  const cptr<int64_t> off = as_const(g.voff);
  int lo = 0, hi = g.n - 1;  // last item whose first block is <= vb (items with no blocks are skipped)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= vb) lo = mid;
    else hi = mid - 1;
  }
  a = load_args(g.items + lo);
  return vb - off[lo];
}

// ONE: a single item, one hardware block per virtual block (no loop, no
// argument lookup: the leanest code for the hot loops' register budget).
#define BS_GROUP_LOOP(BODY)                                           \
  if (ONE) {                                                          \
    const TopkArgs& a = g.one;                                        \
    const int64_t lb = blockIdx.x;                                    \
    BODY;                                                             \
    return;                                                           \
  }                                                                   \
  for (int64_t vb = blockIdx.x; vb < g.total; vb += gridDim.x) {      \
    if (vb != (int64_t)blockIdx.x) __syncthreads();                   \
    TopkArgs a;                                                       \
    const int64_t lb = group_item(g, vb, a);                          \
    BODY;                                                             \
  }

template <bool ONE, int M, int W32T, bool LDS_LUT>
__global__ __launch_bounds__(kThreads) void topk_sample_scores_kernel(GroupArgs g) {
  BS_GROUP_LOOP((sample_scores_body<M, W32T, LDS_LUT>(a, lb % a.s_rblocks, lb / a.s_rblocks)))
}
template <bool ONE, int M, int WS>
__global__ __launch_bounds__(kThreads) void topk_sample_split_kernel(GroupArgs g) {
  BS_GROUP_LOOP((sample_split_body<M, WS>(a, lb % a.s_rblocks, lb / a.s_rblocks)))
}
template <bool ONE, int M, int KCT, bool LDS_LUT>
__global__ __launch_bounds__(kThreads) void topk_sample_mma_kernel(GroupArgs g) {
  BS_GROUP_LOOP((sample_mma_body<M, KCT, LDS_LUT>(a, lb % a.s_rblocks, lb / a.s_rblocks)))
}
template <bool ONE, int M>
__global__ __launch_bounds__(kThreads) void topk_sample_select_kernel(GroupArgs g) {
  BS_GROUP_LOOP((sample_select_body<M>(a, lb)))
}
template <bool ONE, int M, bool LDS_LUT, int BX>
__global__ __launch_bounds__(kThreads) void topk_bound_kernel(GroupArgs g) {
  BS_GROUP_LOOP((bound_body<M, LDS_LUT, BX>(a, lb % (a.nQp / kWave), lb / (a.nQp / kWave))))
}
template <bool ONE, int W32T, int QPL>
__global__ __launch_bounds__(kThreads) void topk_scan_kernel(GroupArgs g) {
  BS_GROUP_LOOP((scan_body<W32T, QPL>(a, lb)))
}
template <bool ONE, int WC>
__global__ __launch_bounds__(kThreads) void topk_scan_generic_kernel(GroupArgs g) {
  BS_GROUP_LOOP((scan_generic_body<WC>(a, lb)))
}
template <bool ONE, int WS>
__global__ __launch_bounds__(kThreads) void topk_scan_split_kernel(GroupArgs g) {
  BS_GROUP_LOOP((scan_split_body<WS>(a, lb)))
}
template <bool ONE, int KCT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void topk_scan_mma_kernel(GroupArgs g) {
  BS_GROUP_LOOP((scan_mma_body<KCT>(a, lb)))
}
template <bool ONE, int M, int W32T>
__global__ __launch_bounds__(kThreads) void topk_scan_rows_kernel(GroupArgs g) {
  BS_GROUP_LOOP((scan_rows_body<M, W32T>(a, lb)))
}
template <bool ONE, int M, bool RAW, bool LUT, int PER>
__global__ __launch_bounds__(kThreads) void topk_select_kernel(GroupArgs g) {
  BS_GROUP_LOOP((select_query<M, RAW, LUT, PER>(a, lb)))
}
#undef BS_GROUP_LOOP

enum Stage { kStSample = 0, kStSampleSelect, kStBound, kStScan, kStSelect, kStages };
const char* const kStageTimer[kStages] = {"topk_sample", "topk_sample_select", "topk_bound", "topk_scan",
                                          "topk_select"};

// The select kernel keeps T in LDS when it scores raw survivors and T is small.
bool select_lut(const TopkArgs& a) { return a.sel_lut != 0; }

// Virtual blocks of one item in one stage (0: the stage does not run).
int64_t stage_blocks(const TopkArgs& a, int st) {
  const bool scan = a.S < a.nC;
  switch (st) {
    case kStSample: return a.s_rblocks * a.s_nqb;
    case kStSampleSelect: return a.nQ;
    case kStBound: {
      const int bx = bound_rows_per_block(a.N);
      return (scan && !a.rows) ? (a.nQp / kWave) * ((a.N + 2 + bx - 1) / bx) : 0;
    }
    case kStScan:
      if (!scan) return 0;
      if (a.rows) return (a.n_slabs + kThreads / kWave - 1) / (kThreads / kWave);
      if (a.mma) return a.n_slabs * a.nqb4;
      if (a.split) return (a.n_slabs / kSplitWaves) * a.nqb4;
      return a.n_slabs * a.nqb4;
    case kStSelect: return a.nQ;
    default: return 0;
  }
}

// Dynamic LDS bytes of one item in one stage.
size_t stage_lds(const TopkArgs& a, int st) {
  const bool lds_lut = a.N < 16384;  // T (rounded up to 64 words) within 64 KB
  switch (st) {
    case kStSample: return (lds_lut || (a.split && !a.mma)) ? (size_t)round_up64(a.N + 1) * 4 : 0;
    case kStSampleSelect: return (size_t)round_up64(a.S) * 4;
    case kStBound: return lds_lut ? (size_t)round_up64(a.N + 1) * 4 : 0;
    case kStScan: return a.rows ? (size_t)round_up64(a.N + 1) * 4 : 0;
    case kStSelect: {  // also room for the whole-corpus fallback (selected keys, key buffer, query words)
      const size_t sel = (size_t)a.kpad * 8 + (size_t)a.lds_keys * 8 + (select_lut(a) ? (size_t)round_up64(a.N + 1) * 4 : 0);
      const size_t fb = ((size_t)2 * a.kpad + (size_t)kFbRowsPerThread * kThreads + (size_t)(a.W32 / 2)) * 8;
      return sel > fb ? sel : fb;
    }
    default: return 0;
  }
}

// The kernel of a stage for the variant of `a` (its width, scan mode, queries per lane).
template <bool ONE, int M>
const void* stage_kernel(const TopkArgs& a, int st) {
  const int W32 = a.W32;
  const bool lds_lut = a.N < 16384;  // T (rounded up to 64 words) within 64 KB
  const bool pow2 = (W32 & (W32 - 1)) == 0;
  switch (st) {
    case kStSample:
      if (a.mma) {
        if (!lds_lut) return (const void*)topk_sample_mma_kernel<ONE, M, 0, false>;
        switch (W32 / 8) {  // 256-bit chunks per row
          case 1: return (const void*)topk_sample_mma_kernel<ONE, M, 1, true>;
          case 2: return (const void*)topk_sample_mma_kernel<ONE, M, 2, true>;
          case 4: return (const void*)topk_sample_mma_kernel<ONE, M, 4, true>;
          case 8: return (const void*)topk_sample_mma_kernel<ONE, M, 8, true>;
          case 16: return (const void*)topk_sample_mma_kernel<ONE, M, 16, true>;
          default: return (const void*)topk_sample_mma_kernel<ONE, M, 0, true>;
        }
      }
      if (a.split)
        return W32 == 256 ? (const void*)topk_sample_split_kernel<ONE, M, 64>
                          : (const void*)topk_sample_split_kernel<ONE, M, 128>;
#define BS_SAMPLE(w) \
  return lds_lut ? (const void*)topk_sample_scores_kernel<ONE, M, w, true> : (const void*)topk_sample_scores_kernel<ONE, M, w, false>
      switch (W32) {
        case 2: BS_SAMPLE(2);
        case 4: BS_SAMPLE(4);
        case 8: BS_SAMPLE(8);
        case 16: BS_SAMPLE(16);
        case 32: BS_SAMPLE(32);
        case 64: BS_SAMPLE(64);
        case 128: BS_SAMPLE(128);
        default: BS_SAMPLE(0);
      }
#undef BS_SAMPLE
    case kStSampleSelect: return (const void*)topk_sample_select_kernel<ONE, M>;
    case kStBound:
      if (bound_rows_per_block(a.N) == 64)
        return lds_lut ? (const void*)topk_bound_kernel<ONE, M, true, 64> : (const void*)topk_bound_kernel<ONE, M, false, 64>;
      return lds_lut ? (const void*)topk_bound_kernel<ONE, M, true, 16> : (const void*)topk_bound_kernel<ONE, M, false, 16>;
    case kStScan:
      if (a.rows) {
        switch (W32) {
          case 2: return (const void*)topk_scan_rows_kernel<ONE, M, 2>;
          case 4: return (const void*)topk_scan_rows_kernel<ONE, M, 4>;
          case 8: return (const void*)topk_scan_rows_kernel<ONE, M, 8>;
          case 16: return (const void*)topk_scan_rows_kernel<ONE, M, 16>;
          case 32: return (const void*)topk_scan_rows_kernel<ONE, M, 32>;
          case 64: return (const void*)topk_scan_rows_kernel<ONE, M, 64>;
          default: return (const void*)topk_scan_rows_kernel<ONE, M, 128>;
        }
      }
      if (a.mma) {
        switch (W32 / 8) {  // 256-bit chunks per row
          case 1: return (const void*)topk_scan_mma_kernel<ONE, 1>;
          case 2: return (const void*)topk_scan_mma_kernel<ONE, 2>;
          case 4: return (const void*)topk_scan_mma_kernel<ONE, 4>;
          case 8: return (const void*)topk_scan_mma_kernel<ONE, 8>;
          case 16: return (const void*)topk_scan_mma_kernel<ONE, 16>;
          default: return (const void*)topk_scan_mma_kernel<ONE, 0>;
        }
      }
      if (a.split) return W32 == 256 ? (const void*)topk_scan_split_kernel<ONE, 64> : (const void*)topk_scan_split_kernel<ONE, 128>;
      if (pow2 && W32 <= 128) {
        const int q = (int)a.qpl;
        switch (W32) {
          case 2: return q == 4 ? (const void*)topk_scan_kernel<ONE, 2, 4> : q == 2 ? (const void*)topk_scan_kernel<ONE, 2, 2> : (const void*)topk_scan_kernel<ONE, 2, 1>;
          case 4: return q == 4 ? (const void*)topk_scan_kernel<ONE, 4, 4> : q == 2 ? (const void*)topk_scan_kernel<ONE, 4, 2> : (const void*)topk_scan_kernel<ONE, 4, 1>;
          case 8: return q == 4 ? (const void*)topk_scan_kernel<ONE, 8, 4> : q == 2 ? (const void*)topk_scan_kernel<ONE, 8, 2> : (const void*)topk_scan_kernel<ONE, 8, 1>;
          case 16: return q == 4 ? (const void*)topk_scan_kernel<ONE, 16, 4> : q == 2 ? (const void*)topk_scan_kernel<ONE, 16, 2> : (const void*)topk_scan_kernel<ONE, 16, 1>;
          case 32: return q == 2 ? (const void*)topk_scan_kernel<ONE, 32, 2> : (const void*)topk_scan_kernel<ONE, 32, 1>;
          case 64: return (const void*)topk_scan_kernel<ONE, 64, 1>;
          default: return (const void*)topk_scan_kernel<ONE, 128, 1>;
        }
      } else {
        int WC = 64;
        while (W32 % WC) WC >>= 1;
        switch (WC) {
          case 2: return (const void*)topk_scan_generic_kernel<ONE, 2>;
          case 4: return (const void*)topk_scan_generic_kernel<ONE, 4>;
          case 8: return (const void*)topk_scan_generic_kernel<ONE, 8>;
          case 16: return (const void*)topk_scan_generic_kernel<ONE, 16>;
          case 32: return (const void*)topk_scan_generic_kernel<ONE, 32>;
          default: return (const void*)topk_scan_generic_kernel<ONE, 64>;
        }
      }
    case kStSelect: {
      const bool wide = a.sel_per > 4;
      if (a.rows)
        return wide ? (const void*)topk_select_kernel<ONE, M, false, false, 8>
                    : (const void*)topk_select_kernel<ONE, M, false, false, 4>;
      if (select_lut(a))
        return wide ? (const void*)topk_select_kernel<ONE, M, true, true, 8>
                    : (const void*)topk_select_kernel<ONE, M, true, true, 4>;
      return wide ? (const void*)topk_select_kernel<ONE, M, true, false, 8>
                  : (const void*)topk_select_kernel<ONE, M, true, false, 4>;
    }
    default: return nullptr;
  }
}

const void* stage_kernel_m(bool one, int measure, const TopkArgs& a, int st) {
  if (one) {
    switch (measure) {
      case BS_IP: return stage_kernel<true, BS_IP>(a, st);
      case BS_HAMMING: return stage_kernel<true, BS_HAMMING>(a, st);
      case BS_JACCARD: return stage_kernel<true, BS_JACCARD>(a, st);
      default: return stage_kernel<true, BS_COSINE>(a, st);
    }
  }
  switch (measure) {
    case BS_IP: return stage_kernel<false, BS_IP>(a, st);
    case BS_HAMMING: return stage_kernel<false, BS_HAMMING>(a, st);
    case BS_JACCARD: return stage_kernel<false, BS_JACCARD>(a, st);
    default: return stage_kernel<false, BS_COSINE>(a, st);
  }
}

bs_status launch_group_kernel(const void* fn, const GroupArgs& g, int64_t grid, size_t lds, hipStream_t s) {
  if (grid < 1 || grid > INT32_MAX) return BS_ERR_ARG;
  void* args[] = {const_cast<GroupArgs*>(&g)};
  const hipError_t e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kThreads), args, lds, s);
  return e == hipSuccess ? BS_OK : BS_ERR_HIP;
}

// Blocks of `fn` that fit one CU at `lds` bytes (at least 1).
int64_t blocks_per_cu(const void* fn, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kThreads, lds) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

// Plan -> argument block. ws: the item's scratch; the LUT comes from the item.
void fill_args(TopkArgs& a, const Plan& p, const TopkItem& it, char* ws) {
  a.Q = it.Q;
  a.C = it.C;
  a.t32 = it.t32;
  a.t32w = nullptr;
  a.popQ = it.popQ;
  a.popC = it.popC;
  a.skeys = reinterpret_cast<uint32_t*>(ws + p.off_skeys);
  a.qc = reinterpret_cast<QConst*>(ws + p.off_qc);
  a.cnts = reinterpret_cast<int32_t*>(ws + p.off_cnts);
  a.cands = reinterpret_cast<uint64_t*>(ws + p.off_cands);
  a.scnt = reinterpret_cast<int32_t*>(ws + p.off_scnt);
  a.qovf = reinterpret_cast<int32_t*>(ws + p.off_qovf);
  a.mtab = reinterpret_cast<uint16_t*>(ws + p.off_mtab);
  a.out_idx = it.out_idx;
  a.out_score = it.out_score;
  a.nQ = it.nQ;
  a.nQp = (it.nQ + 63) / 64 * 64;
  a.nC = it.nC;
  a.S = p.S;
  a.stride = p.stride;
  a.n_slabs = p.n_slabs;
  a.slab = p.slab;
  a.nqb4 = p.nqb4;
  a.scap = p.scap;
  a.kmax = p.kmax;
  a.lds_keys = p.lds_keys;
  a.s_rblocks = p.s_rblocks;
  a.s_nqb = p.s_nqb;
  a.s_qb = p.s_qb;
  a.N = it.N;
  a.W32 = it.N / 32;
  a.k = it.k;
  a.kt = (int32_t)p.kt;
  int kpad = 1;
  while (kpad < it.k) kpad <<= 1;
  a.kpad = kpad;
  a.qpl = (int32_t)p.qpl;
  a.rows = p.rows ? 1 : 0;
  a.split = p.split ? 1 : 0;
  a.mma = p.mma ? 1 : 0;
  a.sel_lut = p.sel_lut ? 1 : 0;
  a.sel_per = p.n_slabs <= 4 * kThreads ? 4 : 8;
}

}  // namespace

// Overrides for tests of the overflow paths (negative = automatic). Each
// host thread has its own: a test's setting never reaches calls that other
// threads make (a server's, say).
static thread_local int64_t g_scap_override = -1;
static thread_local int64_t g_ldskeys_override = -1;
static thread_local int64_t g_taurank_override = -1;
static thread_local int32_t g_mma_override = -1;

// ---- group plans ----------------------------------------------------------------
struct TopkGroup {
  int32_t measure = 0;
  bool persistent = true;
  std::vector<TopkArgs> args;                   // per item (host copy)
  std::vector<std::vector<int32_t>> classes;    // item indices per kernel-variant class
  struct Launch {                               // one stage of one class
    int32_t cls, st;
    const void* fn;
    GroupArgs g;
    int64_t grid;
    size_t lds;
  };
  std::vector<Launch> launches;                 // stage-major order
};

bs_status topk_item_check(const TopkItem& it, int32_t measure) {
  if (it.nQ < 0 || it.nQ > INT32_MAX || it.nC < 1 || it.nC > INT32_MAX || !valid_width(it.N) || it.k < 1 ||
      it.k > BS_MAX_K || it.k > it.nC || measure < 0 || measure > 3)
    return BS_ERR_ARG;
  if (!it.C || !it.popC || !it.t32 || ((!it.Q || !it.popQ || !it.out_idx) && it.nQ > 0)) return BS_ERR_NULL;
  return BS_OK;
}

size_t topk_item_workspace(int64_t nQ, int64_t nC, int32_t N, int32_t k, const TopkTune& tune) {
  return make_plan(nQ, nC, N, k, tune).total;
}

size_t topk_group_meta_bytes(int32_t n_items) {
  if (n_items < 0) return 0;
  // argument blocks, then one offset table per (stage, class); at most one class per item
  return align256((size_t)n_items * sizeof(TopkArgs)) +
         (size_t)kStages * (size_t)n_items * align256(((size_t)n_items + 1) * sizeof(int64_t));
}

bs_status topk_group_create(const TopkItem* items, const TopkTune* tunes, int32_t n, int32_t measure,
                            void* const* item_ws, void* meta, size_t meta_bytes, bool persistent,
                            TopkGroup** out) {
  if (!out) return BS_ERR_NULL;
  *out = nullptr;
  if (n < 0 || measure < 0 || measure > 3) return BS_ERR_ARG;
  if (n > 0 && (!items || !item_ws || !meta)) return BS_ERR_NULL;
  if (meta_bytes < topk_group_meta_bytes(n) || (reinterpret_cast<uintptr_t>(meta) & 255)) return BS_ERR_WORKSPACE;
  for (int32_t i = 0; i < n; ++i) {
    const bs_status st = topk_item_check(items[i], measure);
    if (st != BS_OK) return st;
    if (!item_ws[i] || (reinterpret_cast<uintptr_t>(item_ws[i]) & 255)) return BS_ERR_WORKSPACE;
  }
  std::unique_ptr<TopkGroup> G(new TopkGroup);
  G->measure = measure;
  G->persistent = persistent;
  G->args.resize(n);
  const TopkTune dflt;
  for (int32_t i = 0; i < n; ++i) {
    const Plan p = make_plan(items[i].nQ, items[i].nC, items[i].N, items[i].k, tunes ? tunes[i] : dflt);
    fill_args(G->args[i], p, items[i], static_cast<char*>(item_ws[i]));
  }
  // classes: items that share every kernel variant (width, scan mode, queries per lane, select LUT
  // and slabs per thread)
  for (int32_t i = 0; i < n; ++i) {
    if (G->args[i].nQ == 0) continue;
    int32_t c = -1;
    for (size_t j = 0; j < G->classes.size(); ++j) {
      const TopkArgs& r = G->args[G->classes[j][0]];
      if (r.N == G->args[i].N && r.rows == G->args[i].rows && r.mma == G->args[i].mma && r.qpl == G->args[i].qpl &&
          r.sel_lut == G->args[i].sel_lut && r.sel_per == G->args[i].sel_per)
        c = (int32_t)j;
    }
    if (c < 0) {
      G->classes.emplace_back();
      c = (int32_t)G->classes.size() - 1;
    }
    G->classes[c].push_back(i);
  }
  int lds_max = 0, n_cu = 0;
  device_limits(&lds_max, &n_cu);
  if (n_cu < 1) n_cu = 1;
  // upload: argument blocks, then the offset tables
  char* m = static_cast<char*>(meta);
  const size_t args_bytes = align256((size_t)n * sizeof(TopkArgs));
  const size_t tab_bytes = align256(((size_t)n + 1) * sizeof(int64_t));
  std::vector<char> host(topk_group_meta_bytes(n), 0);
  if (n > 0) memcpy(host.data(), G->args.data(), (size_t)n * sizeof(TopkArgs));
  for (int st = 0; st < kStages; ++st) {
    for (size_t c = 0; c < G->classes.size(); ++c) {
      const std::vector<int32_t>& ci = G->classes[c];
      // the class's items, in item order, as a contiguous sub-array of argument blocks is not
      // guaranteed, so each class gets its own copy of the blocks after the offsets
      const size_t at = args_bytes + ((size_t)st * n + c) * tab_bytes;
      int64_t* off = reinterpret_cast<int64_t*>(host.data() + at);
      int64_t total = 0;
      size_t lds = 0;
      for (size_t j = 0; j < ci.size(); ++j) {
        off[j] = total;
        total += stage_blocks(G->args[ci[j]], st);
        const size_t l = stage_lds(G->args[ci[j]], st);
        lds = l > lds ? l : lds;
      }
      off[ci.size()] = total;
      if (total == 0) continue;
      if (lds > (size_t)65536) return BS_ERR_ARG;  // never with the limits above
      TopkGroup::Launch L;
      L.cls = (int32_t)c;
      L.st = st;
      L.fn = stage_kernel_m(false, measure, G->args[ci[0]], st);
      L.g.items = nullptr;
      L.g.voff = reinterpret_cast<const int64_t*>(m + at);
      L.g.total = total;
      L.g.n = (int32_t)ci.size();
      L.g.one = G->args[ci[0]];
      L.lds = lds;
      L.grid = total;
      if (persistent) {
        const int64_t cap = blocks_per_cu(L.fn, lds) * n_cu;
        if (L.grid > cap) L.grid = cap;
      }
      G->launches.push_back(L);
    }
  }
  // per-class argument blocks: the class's items packed in class order
  // (stored in the first class-sized run of the argument region)
  std::vector<TopkArgs> packed;
  std::vector<size_t> class_base(G->classes.size());
  for (size_t c = 0; c < G->classes.size(); ++c) {
    class_base[c] = packed.size();
    for (int32_t i : G->classes[c]) packed.push_back(G->args[i]);
  }
  if (!packed.empty()) memcpy(host.data(), packed.data(), packed.size() * sizeof(TopkArgs));
  for (TopkGroup::Launch& L : G->launches)
    L.g.items = reinterpret_cast<const TopkArgs*>(m) + class_base[L.cls];
  if (!host.empty() && hipMemcpy(meta, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return BS_ERR_HIP;
  *out = G.release();
  return BS_OK;
}

bs_status topk_group_launch(const TopkGroup* g, hipStream_t s, int32_t cls) {
  if (!g) return BS_ERR_NULL;
  for (const TopkGroup::Launch& L : g->launches) {
    if (cls >= 0 && L.cls != cls) continue;
    ScopedTiming timing(kStageTimer[L.st], s);
    const bs_status st = launch_group_kernel(L.fn, L.g, L.grid, L.lds, s);
    if (st != BS_OK) return st;
  }
  return BS_OK;
}

int32_t topk_group_classes(const TopkGroup* g) { return g ? (int32_t)g->classes.size() : 0; }

int32_t topk_group_class_items(const TopkGroup* g, int32_t cls, int32_t* items, int32_t cap) {
  if (!g || cls < 0 || cls >= (int32_t)g->classes.size()) return 0;
  const std::vector<int32_t>& ci = g->classes[cls];
  for (int32_t j = 0; j < (int32_t)ci.size() && j < cap; ++j) items[j] = ci[j];
  return (int32_t)ci.size();
}

void topk_group_destroy(TopkGroup* g) { delete g; }

}  // namespace bs

extern "C" size_t bs_topk_workspace_size(int64_t nQ, int64_t nC, int32_t N, int32_t k) {
  using namespace bs;
  if (nQ < 0 || nC < 1 || !valid_width(N) || k < 1 || k > BS_MAX_K || k > nC) return 0;
  TopkTune tune;
  tune.mma = g_mma_override;
  return make_plan(nQ, nC, N, k, tune).total;
}

extern "C" int bs_debug_set_topk_limits(int64_t slab_capacity, int64_t lds_keys) {
  bs::g_scap_override = slab_capacity < 0 ? -1 : slab_capacity;
  bs::g_ldskeys_override = lds_keys < 0 ? -1 : lds_keys;
  return 0;
}

extern "C" int64_t bs_topk_sample_size(int64_t nC) { return nC < 1 ? 0 : bs::sample_rows(nC); }

extern "C" int bs_debug_set_topk_mma(int32_t on) {
  bs::g_mma_override = on == 0 ? 0 : -1;
  return 0;
}

extern "C" int bs_debug_set_topk_tau_rank(int64_t rank) {
  bs::g_taurank_override = rank < 1 ? -1 : rank;
  return 0;
}

extern "C" bs_status bs_topk(const uint64_t* Q, const int32_t* popQ, int64_t nQ, const uint64_t* C,
                             const int32_t* popC, int64_t nC, int32_t N, int32_t measure, int32_t k,
                             int32_t* out_idx, float* out_score, void* workspace, size_t workspace_bytes,
                             void* stream) {
  using namespace bs;
  if (nQ < 0 || nC < 1 || nC > INT32_MAX || !valid_width(N) || k < 1 || k > BS_MAX_K || k > nC ||
      measure < 0 || measure > 3)
    return BS_ERR_ARG;
  if (!C || ((!Q || !out_idx) && nQ > 0)) return BS_ERR_NULL;
  if (nQ > INT32_MAX) return BS_ERR_ARG;
  TopkTune tune;
  tune.mma = g_mma_override;
  Plan p = make_plan(nQ, nC, N, k, tune);
  if (!workspace || workspace_bytes < p.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return BS_ERR_WORKSPACE;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  if (nQ == 0) return BS_OK;
  if (g_scap_override >= 0 && g_scap_override < p.scap) {  // fewer slots within the same layout size
    p.scap = g_scap_override;
    p.kmax = p.S + p.n_slabs * p.scap;
  }
  if (g_ldskeys_override >= 0 && g_ldskeys_override < p.lds_keys) p.lds_keys = g_ldskeys_override;
  if (g_taurank_override >= 1 && g_taurank_override < p.kt) p.kt = g_taurank_override;
  char* ws = static_cast<char*>(workspace);
  TopkItem it;
  it.Q = Q;
  it.popQ = popQ ? popQ : reinterpret_cast<const int32_t*>(ws + p.off_popq);
  it.nQ = nQ;
  it.C = C;
  it.popC = popC ? popC : reinterpret_cast<const int32_t*>(ws + p.off_popc);
  it.nC = nC;
  it.N = N;
  it.k = k;
  it.out_idx = out_idx;
  it.out_score = out_score;
  it.t32 = reinterpret_cast<const float*>(ws + p.off_t32);
  TopkArgs a;
  fill_args(a, p, it, ws);
  if (N <= 1024 && !p.split) a.t32w = reinterpret_cast<float*>(ws + p.off_t32);
  hipStream_t s = as_stream(stream);
  // up to N = 1024 the sample pass evaluates T itself (one launch fewer)
  if (a.t32w == nullptr || !popQ || !popC) {
    ScopedTiming timing("topk_prep", s);
    if (a.t32w == nullptr) launch_lut(N, nullptr, reinterpret_cast<float*>(ws + p.off_t32), s);
    if (!popQ) launch_row_popcount(Q, nQ, N, reinterpret_cast<int32_t*>(ws + p.off_popq), s);
    if (!popC) launch_row_popcount(C, nC, N, reinterpret_cast<int32_t*>(ws + p.off_popc), s);
  }
  st = launch_status();
  if (st != BS_OK) return st;
  // one item: arguments inline, one hardware block per virtual block
  for (int stg = 0; stg < kStages; ++stg) {
    const int64_t total = stage_blocks(a, stg);
    if (total == 0) continue;
    GroupArgs g;
    g.items = nullptr;
    g.voff = nullptr;
    g.total = total;
    g.n = 1;
    g.one = a;
    ScopedTiming timing(kStageTimer[stg], s);
    st = launch_group_kernel(stage_kernel_m(true, measure, a, stg), g, total, stage_lds(a, stg), s);
    if (st != BS_OK) return st;
  }
  return BS_OK;
}
