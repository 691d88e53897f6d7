// Query-vs-corpus top-k by estimated similarity on gfx950.
//
// For every query sketch and every corpus sketch the pair count
// x_ab = |q_s AND c_s| (Algorithm 1, second step) is formed on the vector ALU
// and turned into the FP32 score of the chosen measure (Algorithms 1-4, the
// canonical form documented in binsketch.h). The k best corpus rows per query
// are returned ordered by (score, then smaller index). The paper ranks by a
// similarity threshold (Section 4.2); a fixed k is the serving form of it.
//
// Selection without a global sort, in three launches plus a rare fallback:
//  1. sample: per query (one block), score a strided sample of S corpus rows,
//     find the k-th best score tau among them by an LDS radix select, append
//     the sample rows scoring >= tau to the query's candidate list, and store
//     per-query constants for the filter below. The k-th best over the whole
//     corpus is >= tau, so every true top-k row scores >= tau.
//  2. scan: every other (query, corpus row) pair. Lanes hold corpus rows in
//     VGPRs, query words arrive on the scalar unit. Instead of evaluating the
//     score (an IEEE division per pair) the kernel tests a conservative bound
//     on T(x_u) that every pair scoring >= tau satisfies; survivors (a few
//     percent) are staged per wave in LDS and appended 64 at a time with one
//     vector atomic per lane.
//  3. select: per query, exact scores of the candidates as unique 64-bit keys
//     (score key, then inverted index), an exact radix select of the k-th key
//     and a bitonic sort of the k winners.
//  4. fallback: a query whose candidate list overflowed its capacity (e.g.
//     massive exact ties) is recomputed over the whole corpus by a few blocks
//     and selected the same way. Results never depend on which path ran.
#include <float.h>

#include "bs_common.h"

namespace bs {

void launch_lut(int32_t N, double* t64, float* t32, hipStream_t s);
void launch_row_popcount(const uint64_t* X, int64_t n, int32_t N, int32_t* pop, hipStream_t s);

namespace {

constexpr int kThreads = 256;
constexpr int kSampleMax = 4096;     // rows scored in the sample pass
constexpr int kSelectLdsKeys = 4096; // candidate keys selected in LDS (else in place)
constexpr int kStage = 128;          // per-wave staging entries in the scan pass
constexpr int kFallbackBlocks = 16;

struct QConst {  // per-query constants written by the sample pass
  float tau;     // k-th best sample score
  float Tq;      // T(|q_s|)
  float A, B, C; // filter bound: T(x_u) <= fma(sqrtTc, B, fma(s, A, C))
  int32_t xq;    // |q_s|
  int32_t pad0, pad1;
};

struct Plan {
  int64_t S, stride, cap, F;
  size_t off_t32, off_popq, off_popc, off_qc, off_cnt, off_cand, off_scratch, total;
};

Plan make_plan(int64_t nQ, int64_t nC, int32_t N, int32_t k) {
  Plan p;
  p.S = nC < kSampleMax ? nC : kSampleMax;
  p.stride = p.S > 0 ? nC / p.S : 1;
  if (p.S == nC) {
    p.cap = nC;
  } else {
    const int64_t per = (nC + p.S - 1) / p.S;
    int64_t cap = 4 * (int64_t)k * per;
    cap = (cap + 255) / 256 * 256;
    if (cap < p.S) cap = p.S;
    if (cap > nC) cap = nC;
    p.cap = cap;
  }
  p.F = nQ < kFallbackBlocks ? nQ : kFallbackBlocks;
  size_t o = 0;
  p.off_t32 = o;
  o += align256((size_t)(N + 1) * 4);
  p.off_popq = o;
  o += align256((size_t)nQ * 4);
  p.off_popc = o;
  o += align256((size_t)nC * 4);
  p.off_qc = o;
  o += align256((size_t)nQ * sizeof(QConst));
  p.off_cnt = o;
  o += align256((size_t)nQ * 4);
  p.off_cand = o;
  o += align256((size_t)nQ * (size_t)p.cap * 8);
  p.off_scratch = o;
  o += align256((size_t)p.F * (size_t)nC * 8);
  p.total = o;
  return p;
}

template <int M>
__device__ __forceinline__ float score_f32(float Ta, float Tb, float Tu) {
  const float s = Ta + Tb;
  const float ip = s - Tu;
  if (M == BS_IP) return ip;
  const float ham = s - (ip + ip);
  if (M == BS_HAMMING) return ham;
  if (M == BS_JACCARD) {
    const float den = ip + ham;
    return den == 0.0f ? 0.0f : ip / den;
  }
  const float pr = Ta * Tb;
  return pr == 0.0f ? 0.0f : ip / sqrtf(pr);
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

// Block-wide (256 threads) inclusive scan over thread order.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(v, off);
    if (lane >= off) v += t;
  }
  if (lane == kWave - 1) wsum[wid] = v;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wid; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

// The k-th largest of n keys (1 <= k <= n), by MSB-first radix select over
// 8-bit digits. `keys` may point to LDS or global memory. Block-wide call.
template <typename K>
__device__ K radix_select_kth(const K* keys, int64_t n, int64_t k, uint32_t* hist, uint32_t* wsum,
                              K* bcast_prefix, int64_t* bcast_need) {
  K prefix = 0, pmask = 0;
  int64_t need = k;
  for (int shift = (int)sizeof(K) * 8 - 8; shift >= 0; shift -= 8) {
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
      const K key = keys[i];
      if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    // thread t looks at bin 255 - t; inclusive scan = count of keys in bins >= 255 - t
    const uint32_t b = 255u - threadIdx.x;
    const uint32_t h = hist[b];
    const uint32_t incl = block_incl_scan(h, wsum);
    const uint32_t excl = incl - h;
    if ((int64_t)excl < need && (int64_t)incl >= need) {
      *bcast_prefix = prefix | ((K)b << shift);
      *bcast_need = need - (int64_t)excl;
    }
    __syncthreads();
    prefix = *bcast_prefix;
    need = *bcast_need;
    pmask |= ((K)255) << shift;
    __syncthreads();
  }
  return prefix;
}

// Descending bitonic sort of n (power of two, <= 2 * kThreads * 8) keys in LDS.
__device__ void bitonic_sort_desc(uint64_t* v, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += kThreads) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool desc = ((lo & size) == 0);
        const uint64_t a = v[lo], b = v[hi];
        if (desc ? (a < b) : (a > b)) {
          v[lo] = b;
          v[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

struct TopkArgs {
  const uint64_t* __restrict__ Q;  // [nQ][W64]
  const uint64_t* __restrict__ C;  // [nC][W64]
  const float* __restrict__ t32;   // T(0..N)
  const int32_t* __restrict__ popQ;
  const int32_t* __restrict__ popC;
  QConst* __restrict__ qc;
  int32_t* __restrict__ cnt;       // [nQ]
  uint64_t* __restrict__ cand;     // [nQ][cap]
  uint64_t* __restrict__ scratch;  // [F][nC]
  int32_t* __restrict__ out_idx;   // [nQ][k]
  float* __restrict__ out_score;   // [nQ][k] or null
  int64_t nQ, nC, S, stride, cap;
  int32_t N, W32, k, kpad;
};

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
  c.pad0 = c.pad1 = 0;
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
template <int M>
__global__ __launch_bounds__(kThreads) void topk_sample_kernel(TopkArgs a) {
  extern __shared__ uint64_t smem64[];
  const int W64 = a.W32 / 2;
  uint64_t* qw = smem64;                                   // [W64]
  uint32_t* keys = reinterpret_cast<uint32_t*>(qw + W64);  // [S]
  int32_t* xabs = reinterpret_cast<int32_t*>(keys + a.S);  // [S]
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kThreads / kWave];
  __shared__ uint32_t bprefix;
  __shared__ int64_t bneed;
  __shared__ uint32_t nsel;
  const int64_t q = blockIdx.x;
  const uint64_t* qrow = a.Q + (size_t)q * W64;
  for (int w = threadIdx.x; w < W64; w += kThreads) qw[w] = qrow[w];
  if (threadIdx.x == 0) nsel = 0;
  const int32_t xq = a.popQ[q];
  const float Tq = a.t32[xq];
  __syncthreads();
  for (int64_t i = threadIdx.x; i < a.S; i += kThreads) {
    const int64_t row = i * a.stride;
    const int32_t xab = and_popcount_row(qw, a.C + (size_t)row * W64, W64);
    const int32_t xc = a.popC[row];
    const float sc = score_f32<M>(Tq, a.t32[xc], a.t32[xq + xc - xab]);
    keys[i] = score_key<M>(sc);
    xabs[i] = xab;
  }
  __syncthreads();
  const uint32_t tau_key = radix_select_kth<uint32_t>(keys, a.S, a.k, hist, wsum, &bprefix, &bneed);
  uint64_t* cq = a.cand + (size_t)q * a.cap;
  for (int64_t i = threadIdx.x; i < a.S; i += kThreads) {
    if (keys[i] >= tau_key) {
      const uint32_t slot = atomicAdd(&nsel, 1u);
      cq[slot] = ((uint64_t)(uint32_t)xabs[i] << 32) | (uint32_t)(i * a.stride);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.cnt[q] = (int32_t)nsel;
    a.qc[q] = make_qconst<M>(key_score<M>(tau_key), Tq, xq);
  }
}

// ---- pass 2: filtered scan ----------------------------------------------------
struct Staged {
  int32_t q, row, xab;
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Append the first `n` (<= 64) staged entries: one vector atomic per lane.
__device__ __forceinline__ void flush_stage(Staged* st, int n, int lane, const TopkArgs& a) {
  if (lane < n) {
    const Staged e = st[lane];
    const int32_t slot = atomicAdd(a.cnt + e.q, 1);
    if (slot < a.cap) a.cand[(size_t)e.q * a.cap + slot] = ((uint64_t)(uint32_t)e.xab << 32) | (uint32_t)e.row;
  }
}

template <int WC, int M>
__global__ __launch_bounds__(kThreads) void topk_scan_kernel(TopkArgs a, int64_t n_ctiles, int64_t nqb,
                                                             int64_t qb_size) {
  extern __shared__ float lut[];  // [N+1], then per-wave staging
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  // XCD-aware tile order: blocks are dealt round-robin to the 8 XCDs, so
  // give each XCD a contiguous range of (corpus tile, query block) pairs;
  // the query blocks of one corpus tile then share that XCD's L2.
  const int64_t nblocks = n_ctiles * nqb;
  const int64_t per_xcd = (nblocks + 7) / 8;
  const int64_t bid = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (bid >= nblocks) return;
  const int64_t ct = bid / nqb, qb = bid % nqb;
  const int64_t q_begin = qb * qb_size;
  const int64_t q_end = q_begin + qb_size < a.nQ ? q_begin + qb_size : a.nQ;

  const int Np1 = a.N + 1;
  for (int x = threadIdx.x; x < Np1; x += kThreads) lut[x] = a.t32[x];
  Staged* stage = reinterpret_cast<Staged*>(lut + ((Np1 + 3) & ~3)) + (size_t)wid * kStage;
  __syncthreads();

  const int64_t row = ct * kThreads + threadIdx.x;
  const bool in_sample = (row % a.stride == 0) && (row / a.stride < a.S);
  const bool valid = row < a.nC && !in_sample;
  const int64_t rr = row < a.nC ? row : a.nC - 1;
  const int W32 = a.W32;
  const int nchunks = W32 / WC;
  const uint32_t* crow = reinterpret_cast<const uint32_t*>(a.C) + (size_t)rr * W32;
  const uint32_t* Q32 = reinterpret_cast<const uint32_t*>(a.Q);
  const int32_t xc = a.popC[rr];
  const float Tc = lut[xc];
  const float sqTc = (M == BS_COSINE) ? sqrtf(Tc) : 0.0f;

  uint32_t cw[WC];
  if (nchunks == 1) {
#pragma unroll
    for (int w = 0; w < WC; ++w) cw[w] = crow[w];
  }
  int fill = 0;  // wave-uniform count of staged entries
  for (int64_t q = q_begin; q < q_end; ++q) {
    uint32_t acc = 0;
    for (int c = 0; c < nchunks; ++c) {
      if (nchunks != 1) {
#pragma unroll
        for (int w = 0; w < WC; ++w) cw[w] = crow[c * WC + w];
      }
      const cptr<uint32_t> qrow = as_const(Q32 + (size_t)q * W32 + c * WC);
#pragma unroll
      for (int w = 0; w < WC; ++w) acc += popc32(qrow[w] & cw[w]);
    }
    const cptr<QConst> k = as_const<QConst>(a.qc) + q;
    const int32_t xu = k->xq + xc - (int32_t)acc;
    const float Tu = lut[xu];
    const float s = k->Tq + Tc;
    float bound = fmaf(s, k->A, k->C);
    if (M == BS_COSINE) bound = fmaf(sqTc, k->B, bound);
    const bool take = valid && Tu <= bound;
    const uint64_t mask = __ballot(take);
    if (mask) {
      const int pos = fill + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      if (take) stage[pos] = Staged{(int32_t)q, (int32_t)row, (int32_t)acc};
      fill += __builtin_popcountll(mask);
      if (fill >= kWave) {
        wave_sync_lds();
        flush_stage(stage, kWave, lane, a);
        wave_sync_lds();
        Staged rest = {0, 0, 0};
        if (lane < fill - kWave) rest = stage[kWave + lane];
        wave_sync_lds();
        if (lane < fill - kWave) stage[lane] = rest;
        fill -= kWave;
        wave_sync_lds();
      }
    }
  }
  wave_sync_lds();
  flush_stage(stage, fill, lane, a);
}

// ---- pass 3: exact selection of each query's candidates -----------------------
template <int M>
__device__ __forceinline__ uint64_t make_key(float sc, uint32_t idx) {
  return ((uint64_t)score_key<M>(sc) << 32) | (uint64_t)(~idx);
}

template <int M>
__device__ void select_and_write(const uint64_t* keys, int64_t n, int64_t q, const TopkArgs& a,
                                 uint64_t* sel, uint32_t* hist, uint32_t* wsum, uint64_t* bprefix,
                                 int64_t* bneed, uint32_t* nsel) {
  const uint64_t kth = radix_select_kth<uint64_t>(keys, n, a.k, hist, wsum, bprefix, bneed);
  if (threadIdx.x == 0) *nsel = 0;
  for (int t = threadIdx.x; t < a.kpad; t += kThreads) sel[t] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const uint64_t key = keys[i];
    if (key >= kth) {  // exactly k keys: the keys are unique
      const uint32_t slot = atomicAdd(nsel, 1u);
      if (slot < (uint32_t)a.kpad) sel[slot] = key;
    }
  }
  __syncthreads();
  bitonic_sort_desc(sel, a.kpad);
  for (int t = threadIdx.x; t < a.k; t += kThreads) {
    const uint64_t key = sel[t];
    a.out_idx[q * a.k + t] = (int32_t)(~(uint32_t)key);
    if (a.out_score) a.out_score[q * a.k + t] = key_score<M>((uint32_t)(key >> 32));
  }
  __syncthreads();
}

template <int M>
__global__ __launch_bounds__(kThreads) void topk_select_kernel(TopkArgs a) {
  extern __shared__ uint64_t sm[];  // sel[kpad], then keys[kSelectLdsKeys]
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kThreads / kWave];
  __shared__ uint64_t bprefix;
  __shared__ int64_t bneed;
  __shared__ uint32_t nsel;
  const int64_t q = blockIdx.x;
  const int64_t n = a.cnt[q];
  if (n > a.cap) return;  // overflowed: the fallback kernel owns this query
  uint64_t* sel = sm;
  uint64_t* cq = a.cand + (size_t)q * a.cap;
  uint64_t* keys = n <= kSelectLdsKeys ? sm + a.kpad : cq;
  const int32_t xq = a.popQ[q];
  const float Tq = a.t32[xq];
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const uint64_t e = cq[i];
    const uint32_t idx = (uint32_t)e;
    const int32_t xab = (int32_t)(e >> 32);
    const int32_t xc = a.popC[idx];
    const float sc = score_f32<M>(Tq, a.t32[xc], a.t32[xq + xc - xab]);
    keys[i] = make_key<M>(sc, idx);
  }
  __syncthreads();
  select_and_write<M>(keys, n, q, a, sel, hist, wsum, &bprefix, &bneed, &nsel);
}

// ---- fallback: whole-corpus selection for overflowed queries ----------------
template <int M>
__global__ __launch_bounds__(kThreads) void topk_fallback_kernel(TopkArgs a) {
  extern __shared__ uint64_t sm[];  // sel[kpad], then qw[W64]
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kThreads / kWave];
  __shared__ uint64_t bprefix;
  __shared__ int64_t bneed;
  __shared__ uint32_t nsel;
  const int W64 = a.W32 / 2;
  uint64_t* sel = sm;
  uint64_t* qw = sm + a.kpad;
  uint64_t* keys = a.scratch + (size_t)blockIdx.x * a.nC;
  for (int64_t q = blockIdx.x; q < a.nQ; q += gridDim.x) {
    if (a.cnt[q] <= a.cap) continue;
    const uint64_t* qrow = a.Q + (size_t)q * W64;
    for (int w = threadIdx.x; w < W64; w += kThreads) qw[w] = qrow[w];
    const int32_t xq = a.popQ[q];
    const float Tq = a.t32[xq];
    __syncthreads();
    for (int64_t i = threadIdx.x; i < a.nC; i += kThreads) {
      const int32_t xab = and_popcount_row(qw, a.C + (size_t)i * W64, W64);
      const int32_t xc = a.popC[i];
      const float sc = score_f32<M>(Tq, a.t32[xc], a.t32[xq + xc - xab]);
      keys[i] = make_key<M>(sc, (uint32_t)i);
    }
    __syncthreads();
    select_and_write<M>(keys, a.nC, q, a, sel, hist, wsum, &bprefix, &bneed, &nsel);
  }
}

template <int M>
bs_status run_topk(TopkArgs a, const Plan& p, hipStream_t s) {
  const int W64 = a.W32 / 2;
  // 1. sample
  {
    const size_t lds = (size_t)W64 * 8 + (size_t)p.S * 8;
    ScopedTiming timing("topk_sample", s);
    hipLaunchKernelGGL((topk_sample_kernel<M>), dim3((unsigned)a.nQ), dim3(kThreads), lds, s, a);
  }
  // 2. scan the rest of the corpus
  if (p.S < a.nC) {
    const int64_t n_ctiles = (a.nC + kThreads - 1) / kThreads;
    // query blocks: enough (tile, block) pairs for ~16 blocks per CU
    int64_t nqb = (4096 + n_ctiles - 1) / n_ctiles;
    if (nqb > a.nQ) nqb = a.nQ;
    if (nqb < 1) nqb = 1;
    const int64_t qb_size = (a.nQ + nqb - 1) / nqb;
    nqb = (a.nQ + qb_size - 1) / qb_size;
    const int64_t nblocks = n_ctiles * nqb;
    const int64_t grid = (nblocks + 7) / 8 * 8;
    if (grid > INT32_MAX) return BS_ERR_ARG;
    const size_t lds = (size_t)((a.N + 1 + 3) & ~3) * 4 + (size_t)(kThreads / kWave) * kStage * sizeof(Staged);
    int WC = 64;
    while (a.W32 % WC) WC >>= 1;
    ScopedTiming timing("topk_scan", s);
#define BS_SCAN_CASE(wc)                                                                          \
  case wc:                                                                                        \
    hipLaunchKernelGGL((topk_scan_kernel<wc, M>), dim3((unsigned)grid), dim3(kThreads), lds, s, a, \
                       n_ctiles, nqb, qb_size);                                                   \
    break;
    switch (WC) {
      BS_SCAN_CASE(2)
      BS_SCAN_CASE(4)
      BS_SCAN_CASE(8)
      BS_SCAN_CASE(16)
      BS_SCAN_CASE(32)
      BS_SCAN_CASE(64)
      default:
        return BS_ERR_ARG;
    }
#undef BS_SCAN_CASE
  }
  // 3. select
  {
    const size_t lds = (size_t)a.kpad * 8 + (size_t)kSelectLdsKeys * 8;
    ScopedTiming timing("topk_select", s);
    hipLaunchKernelGGL((topk_select_kernel<M>), dim3((unsigned)a.nQ), dim3(kThreads), lds, s, a);
  }
  // 4. fallback for overflowed queries (exits at once when none overflowed)
  if (p.S < a.nC) {
    const size_t lds = (size_t)a.kpad * 8 + (size_t)W64 * 8;
    ScopedTiming timing("topk_fallback", s);
    hipLaunchKernelGGL((topk_fallback_kernel<M>), dim3((unsigned)p.F), dim3(kThreads), lds, s, a);
  }
  return launch_status();
}

}  // namespace

// Capacity override for tests of the overflow path (0 = automatic).
static int64_t g_cap_override = 0;

}  // namespace bs

extern "C" size_t bs_topk_workspace_size(int64_t nQ, int64_t nC, int32_t N, int32_t k) {
  using namespace bs;
  if (nQ < 0 || nC < 1 || !valid_width(N) || k < 1 || k > BS_MAX_K || k > nC) return 0;
  return make_plan(nQ, nC, N, k).total;
}

extern "C" int bs_debug_set_topk_capacity(int64_t cap) {
  bs::g_cap_override = cap < 0 ? 0 : cap;
  return 0;
}

extern "C" bs_status bs_topk(const uint64_t* Q, int64_t nQ, const uint64_t* C, int64_t nC, int32_t N,
                             int32_t measure, int32_t k, int32_t* out_idx, float* out_score,
                             void* workspace, size_t workspace_bytes, void* stream) {
  using namespace bs;
  if (nQ < 0 || nC < 1 || nC > INT32_MAX || !valid_width(N) || k < 1 || k > BS_MAX_K || k > nC ||
      measure < 0 || measure > 3)
    return BS_ERR_ARG;
  if (!C || ((!Q || !out_idx) && nQ > 0)) return BS_ERR_NULL;
  if (nQ > INT32_MAX) return BS_ERR_ARG;
  Plan p = make_plan(nQ, nC, N, k);
  if (!workspace || workspace_bytes < p.total || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return BS_ERR_WORKSPACE;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  if (nQ == 0) return BS_OK;
  if (g_cap_override > 0 && g_cap_override >= p.S && g_cap_override < p.cap) p.cap = g_cap_override;
  char* ws = static_cast<char*>(workspace);
  TopkArgs a;
  a.Q = Q;
  a.C = C;
  a.t32 = reinterpret_cast<const float*>(ws + p.off_t32);
  a.popQ = reinterpret_cast<const int32_t*>(ws + p.off_popq);
  a.popC = reinterpret_cast<const int32_t*>(ws + p.off_popc);
  a.qc = reinterpret_cast<QConst*>(ws + p.off_qc);
  a.cnt = reinterpret_cast<int32_t*>(ws + p.off_cnt);
  a.cand = reinterpret_cast<uint64_t*>(ws + p.off_cand);
  a.scratch = reinterpret_cast<uint64_t*>(ws + p.off_scratch);
  a.out_idx = out_idx;
  a.out_score = out_score;
  a.nQ = nQ;
  a.nC = nC;
  a.S = p.S;
  a.stride = p.stride;
  a.cap = p.cap;
  a.N = N;
  a.W32 = N / 32;
  a.k = k;
  int kpad = 1;
  while (kpad < k) kpad <<= 1;
  a.kpad = kpad;
  hipStream_t s = as_stream(stream);
  {
    ScopedTiming timing("topk_prep", s);
    launch_lut(N, nullptr, reinterpret_cast<float*>(ws + p.off_t32), s);
    launch_row_popcount(Q, nQ, N, reinterpret_cast<int32_t*>(ws + p.off_popq), s);
    launch_row_popcount(C, nC, N, reinterpret_cast<int32_t*>(ws + p.off_popc), s);
  }
  st = launch_status();
  if (st != BS_OK) return st;
  switch (measure) {
    case BS_IP:
      return run_topk<BS_IP>(a, p, s);
    case BS_HAMMING:
      return run_topk<BS_HAMMING>(a, p, s);
    case BS_JACCARD:
      return run_topk<BS_JACCARD>(a, p, s);
    default:
      return run_topk<BS_COSINE>(a, p, s);
  }
}
