// BinSketch compression on gfx950 (Section 3, Definition "BinSketch"):
// sketch bit j of row r is the OR of a[i] over all i with pi(i) = j, i.e. it
// is set iff some set index i of row r has pi[i] == j. Only the set indices
// are touched, one pass over the CSR data (Section 3, the cost paragraph
// after the definition).
//
// Kernel design
//   * One wavefront owns a window of G consecutive rows (G * N/32 32-bit
//     words of LDS, ~2 KB). It streams the window's whole nnz range
//     [indptr[r0], indptr[r0+G]) with coalesced, non-temporal 4-byte loads,
//     U loads in flight per lane, so row boundaries cost nothing in the
//     memory stream and short rows do not idle lanes.
//   * Each element's window row is found without a search: the row starts
//     inside the current chunk are walked on the scalar path and every lane
//     increments its row for each start it has passed (two VALU ops per row
//     start, ~1 start per 230 elements at the benchmark's mean row length).
//   * pi[idx] is gathered through the cache hierarchy (the table is read by
//     every wave and stays resident in L2), then ds_or_b32 sets the bit in the
//     LDS copy of the row's sketch. OR is idempotent and commutative, so the
//     LDS atomics give the same bits in any order (no race in the result).
//   * The window's sketches are contiguous in the output, so they leave LDS
//     as one coalesced run of 64-bit non-temporal stores; popcounts are summed
//     per row in LDS on the way out.
#include <string.h>

#include <memory>
#include <type_traits>
#include <vector>

#include "bs_common.h"
#include "sketch_group.h"

namespace bs {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kUnroll = 8;              // element loads in flight per lane
constexpr int kStageWords = 512;        // LDS sketch words per wave (2 KB)
constexpr int kMaxRowsPerWave = 32;     // G <= 32 so G+1 row pointers fit one wave

struct SketchArgs {
  const int32_t* __restrict__ indptr;
  const int32_t* __restrict__ indices;
  const int32_t* __restrict__ pi;
  const uint16_t* __restrict__ pi16;  // the map as 16-bit targets (validated), or null
  uint32_t* __restrict__ out32;  // [n_rows][W32]
  int32_t* __restrict__ pop;     // [n_rows] or null
  int32_t* __restrict__ err;     // [1] or null
  int64_t n_rows;
  int64_t nnz;
  int64_t d;
  int32_t N;
  int32_t W32;     // N / 32
  int32_t G;       // rows per wave
  int32_t stride;  // LDS words per wave: G*W32 + G
};

// One window of G rows by one wave; `sk` is the wave's LDS stage
// (a.stride words). Wave-level synchronisation only.
__device__ __forceinline__ void sketch_window(const SketchArgs& a, int64_t wave, uint32_t* sk) {
  const int lane = threadIdx.x % kWave;
  const int64_t r0 = wave * a.G;
  if (r0 >= a.n_rows) return;
  const int g = (int)(a.n_rows - r0 < a.G ? a.n_rows - r0 : a.G);
  const int W32 = a.W32;
  uint32_t* cnt = sk + (size_t)a.G * W32;

  // Row pointers of the window: lane l holds indptr[r0 + l] for l <= g.
  const int32_t p = (lane <= g) ? a.indptr[r0 + lane] : 0;
  const int32_t prev = __shfl_up(p, 1);
  const bool bad = (lane <= g) &&
                   (p < 0 || (int64_t)p > a.nnz || (lane >= 1 && p < prev) || (r0 == 0 && lane == 0 && p != 0));
  const bool window_bad = __ballot(bad) != 0;

  for (int w = lane; w < g * W32; w += kWave) sk[w] = 0u;
  if (lane < g) cnt[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  uint32_t errbits = window_bad ? (uint32_t)BS_FLAG_INDPTR : 0u;
  if (!window_bad) {
    const int64_t e0 = __builtin_amdgcn_readfirstlane(p);
    const int64_t e1 = __builtin_amdgcn_readlane(p, g);
    int cur = 0;  // window row of element `base` (wave-uniform)
    int64_t nxt = (g > 1) ? (int64_t)__builtin_amdgcn_readlane(p, 1) : INT64_MAX;
    const uint32_t d32 = (uint32_t)a.d;
    const uint32_t N32 = (uint32_t)a.N;
    for (int64_t base = e0; base < e1; base += (int64_t)kWave * kUnroll) {
      int32_t idx[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = base + u * kWave + lane;
        idx[u] = (k < e1) ? __builtin_nontemporal_load(a.indices + k) : -1;
      }
      int32_t j[kUnroll];
      bool in[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = base + u * kWave + lane;
        const bool live = k < e1;
        in[u] = live && (uint32_t)idx[u] < d32;
        if (live && !in[u]) errbits |= BS_FLAG_INDEX;
        j[u] = in[u] ? (a.pi16 ? (int32_t)a.pi16[idx[u]] : a.pi[idx[u]]) : 0;
      }
      int rowv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) rowv[u] = cur;
      const int64_t end = base + (int64_t)kWave * kUnroll;
      while (nxt < end) {  // row starts inside this chunk (wave-uniform loop)
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) rowv[u] += (base + u * kWave + lane >= nxt) ? 1 : 0;
        ++cur;
        nxt = (cur + 1 < g) ? (int64_t)__builtin_amdgcn_readlane(p, cur + 1) : INT64_MAX;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (in[u]) {
          if ((uint32_t)j[u] < N32) {
            atomicOr(&sk[rowv[u] * W32 + (j[u] >> 5)], 1u << (j[u] & 31));
          } else {
            errbits |= BS_FLAG_MAP;
          }
        }
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // The window's sketches are contiguous in the output: one coalesced run.
  const int W64 = W32 / 2;
  const uint64_t* s64 = reinterpret_cast<const uint64_t*>(sk);
  uint64_t* o64 = reinterpret_cast<uint64_t*>(a.out32 + (size_t)r0 * W32);
  for (int w = lane; w < g * W64; w += kWave) {
    const uint64_t v = s64[w];
    __builtin_nontemporal_store(v, o64 + w);
    if (a.pop) atomicAdd(&cnt[w / W64], (uint32_t)__builtin_popcountll(v));
  }
  if (a.pop) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < g) a.pop[r0 + lane] = (int32_t)cnt[lane];
  }
  if (a.err && errbits) atomicOr(a.err, (int32_t)errbits);
  // the stage may be reused by this wave's next window
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kWavesPerBlock * kWave) void sketch_csr_kernel(SketchArgs a) {
  extern __shared__ uint32_t lds[];
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  sketch_window(a, (int64_t)blockIdx.x * kWavesPerBlock + wid, lds + (size_t)wid * a.stride);
}

// Many independent sketch problems (different maps, widths and sizes) in one
// launch: the windows of all items form one list; wave w of the grid takes
// windows w, w + (waves in the grid), ... and finds each window's item by a
// binary search over the items' first-window offsets.
__device__ __forceinline__ SketchArgs load_sketch_args(const SketchArgs* p) {
  const cptr<SketchArgs> c = as_const(p);
  SketchArgs a;
  a.indptr = c->indptr;
  a.indices = c->indices;
  a.pi = c->pi;
  a.pi16 = c->pi16;
  a.out32 = c->out32;
  a.pop = c->pop;
  a.err = c->err;
  a.n_rows = c->n_rows;
  a.nnz = c->nnz;
  a.d = c->d;
  a.N = c->N;
  a.W32 = c->W32;
  a.G = c->G;
  a.stride = c->stride;
  return a;
}

// The maps of a group as 16-bit targets (N <= 65536): half the bytes of
// the 32-bit table, so a 10^6-entry map (2 MB) stays in L2 while the grid
// works through its problem. Values outside [0, N) are reported (BS_FLAG_MAP,
// as when the map is packed for LDS) and stored as 0. Virtual blocks of 1024
// entries, four per thread.
struct PackItem {
  const int32_t* pi;
  uint16_t* out;
  int64_t d;
  int32_t N;
  int32_t* err;
};

__global__ __launch_bounds__(256) void pack16_group_kernel(const PackItem* items, const int64_t* boff, int32_t n,
                                                         int64_t total) {
  const cptr<int64_t> off = as_const(boff);
  for (int64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= vb) lo = mid;
      else hi = mid - 1;
    }
    const cptr<PackItem> it = as_const(items + lo);
    const int32_t* pi = it->pi;
    uint16_t* out = it->out;
    const int64_t d = it->d;
    const uint32_t N = (uint32_t)it->N;
    int32_t* err = it->err;
    const int64_t e0 = ((vb - off[lo]) * 256 + threadIdx.x) * 4;
    if (e0 >= d) continue;
    uint32_t v[4];
    if (e0 + 4 <= d && (reinterpret_cast<uintptr_t>(pi) & 15) == 0) {
      const int4 q = *reinterpret_cast<const int4*>(pi + e0);
      v[0] = (uint32_t)q.x;
      v[1] = (uint32_t)q.y;
      v[2] = (uint32_t)q.z;
      v[3] = (uint32_t)q.w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = e0 + u < d ? (uint32_t)pi[e0 + u] : 0u;
    }
    bool bad = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (v[u] >= N) {
        bad = true;
        v[u] = 0;
      }
    }
    if (bad && err) atomicOr(err, (int32_t)BS_FLAG_MAP);
    if (e0 + 4 <= d && (reinterpret_cast<uintptr_t>(out) & 7) == 0) {
      const uint64_t w = (uint64_t)v[0] | ((uint64_t)v[1] << 16) | ((uint64_t)v[2] << 32) | ((uint64_t)v[3] << 48);
      *reinterpret_cast<uint64_t*>(out + e0) = w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u < d) out[e0 + u] = (uint16_t)v[u];
    }
  }
}

__global__ __launch_bounds__(kWavesPerBlock * kWave) void sketch_group_kernel(const SketchArgs* items,
                                                                            const int64_t* woff, int32_t n,
                                                                            int64_t total, int32_t wave_words) {
  extern __shared__ uint32_t lds[];
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  uint32_t* sk = lds + (size_t)wid * wave_words;
  const cptr<int64_t> off = as_const(woff);
  const int64_t step = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + wid; w < total; w += step) {
    int lo = 0, hi = n - 1;  // last item whose first window is <= w
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= w) lo = mid;
      else hi = mid - 1;
    }
    const SketchArgs a = load_sketch_args(items + lo);
    sketch_window(a, w - off[lo], sk);
  }
}

// ---- map-in-LDS variant ---------------------------------------------------
// When pi fits in LDS bit-packed (ceil(log2 N) bits per entry), it is packed
// once per call into the caller's workspace, and a persistent grid of one
// 16-wave block per CU copies it into LDS, so every gather is an LDS read
// plus a funnel shift instead of a 128-byte L2 line fill for 4 useful bytes.
// Each wave then owns a contiguous range of rows, processed in windows of G
// rows exactly as above.
constexpr int kBigBlockWaves = 16;
constexpr int kMaxParts = BS_SKETCH_MAX_PARTS;  // CSR matrices sketched by one launch
constexpr int kUnrollLds = 16;  // element loads in flight per lane

// LDS byte addresses as plain integers, so that an address is one
// shift-and-add from an index (the LDS base of the dynamic allocation is a
// link-time constant the compiler cannot fold into the offset).
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_addr(const uint32_t* p) {
  return (uint32_t)(uintptr_t)(const lds_u32*)p;
}
__device__ __forceinline__ lds_u32* lds_ptr(uint32_t a) { return (lds_u32*)(uintptr_t)a; }

struct SketchLdsArgs {
  SketchArgs s[kMaxParts];  // the CSR matrices (parts) of the call; one map, one width
  int32_t n_parts;
  int32_t wave_off[kMaxParts + 1];  // part i is sketched by waves [wave_off[i], wave_off[i + 1])
  const uint32_t* __restrict__ packed;  // bit-packed map (table_words - 1 words)
  int32_t bits;         // bits per packed map entry
  int32_t table_words;  // packed map words in LDS (including one pad word)
  int64_t n_windows;
};

// Bit-pack pi: entry e occupies bits [e*bits, (e+1)*bits) of the packed
// words, so the 32 entries of group g fill exactly words [g*bits, (g+1)*bits).
// One thread per group: no division and no atomics. Out-of-range values are
// reported and stored as 0, so the packed table always holds valid targets.
__global__ void pack_map_kernel(const int32_t* __restrict__ pi, int64_t d, int32_t N, int32_t bits,
                                uint32_t* __restrict__ packed, int32_t* __restrict__ err) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_groups = (d + 31) / 32;
  if (gi >= n_groups) return;
  const int64_t e0 = gi * 32;
  uint32_t v[32];
  if (e0 + 32 <= d && (reinterpret_cast<uintptr_t>(pi) & 15) == 0) {  // eight 16-byte loads
    const int4* src = reinterpret_cast<const int4*>(pi + e0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int4 q = src[u];
      v[4 * u] = (uint32_t)q.x;
      v[4 * u + 1] = (uint32_t)q.y;
      v[4 * u + 2] = (uint32_t)q.z;
      v[4 * u + 3] = (uint32_t)q.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = e0 + u < d ? (uint32_t)pi[e0 + u] : 0u;
  }
  uint64_t acc = 0;
  int fill = 0;
  uint32_t* dst = packed + gi * bits;
  bool bad = false;
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    uint32_t x = v[u];
    if (x >= (uint32_t)N) {
      bad = true;
      x = 0;
    }
    acc |= (uint64_t)x << fill;
    fill += bits;
    if (fill >= 32) {
      *dst++ = (uint32_t)acc;
      acc >>= 32;
      fill -= 32;
    }
  }
  if (bad && err) atomicOr(err, (int32_t)BS_FLAG_MAP);
}

// RA: index chunks aligned to each wave's element run (short windows) rather
// than to each window's start (see the index-stream comment below).
template <bool RA>
__global__ __launch_bounds__(kBigBlockWaves * kWave) void sketch_csr_lds_kernel(SketchLdsArgs A) {
  extern __shared__ uint32_t lds[];
  const int bits = A.bits;
  uint32_t* table = lds;
  uint32_t* stage_base = lds + A.table_words;

  uint32_t errbits = 0;
  // The packed map (built by pack_map_kernel) goes to LDS 16 bytes per load,
  // every load of a thread in flight at once (one round trip for up to
  // 128 KB); then the pad word read past the last entry is cleared.
  {
    constexpr int CB = 8;
    const int n16 = (A.table_words - 1) / 4;  // whole 16-byte chunks of the packed words
    const uint4* src = reinterpret_cast<const uint4*>(A.packed);
    uint4* dst = reinterpret_cast<uint4*>(table);
    for (int t0 = threadIdx.x; t0 < n16; t0 += (int)blockDim.x * CB) {
      uint32_t v[CB][4];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int t = t0 + c * (int)blockDim.x;
        const uint4 q = src[t < n16 ? t : 0];
        v[c][0] = q.x;
        v[c][1] = q.y;
        v[c][2] = q.z;
        v[c][3] = q.w;
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int t = t0 + c * (int)blockDim.x;
        if (t < n16) dst[t] = make_uint4(v[c][0], v[c][1], v[c][2], v[c][3]);
      }
    }
    for (int t = n16 * 4 + threadIdx.x; t < A.table_words - 1; t += blockDim.x) table[t] = A.packed[t];
    if (threadIdx.x == 0) table[A.table_words - 1] = 0u;
  }
  __syncthreads();

  // 2. each wave owns a contiguous range of rows of one part, in windows of G
  // rows. The part is picked by constant-index selects (no dynamic indexing
  // of the argument block).
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t gwv = (int64_t)blockIdx.x * kBigBlockWaves + wid;
  SketchArgs a = A.s[0];
  int64_t w_lo = 0, w_hi = A.wave_off[1];
#pragma unroll
  for (int i = 1; i < kMaxParts; ++i) {
    if (i < A.n_parts && gwv >= A.wave_off[i]) {
      a = A.s[i];
      w_lo = A.wave_off[i];
      w_hi = A.wave_off[i + 1];
    }
  }
  const int W32 = a.W32;
  uint32_t* sk = stage_base + (size_t)wid * a.stride;
  uint32_t* cnt = sk + (size_t)a.G * W32;
  const uint32_t d32 = (uint32_t)a.d;
  // Rows split by set bits, not by count: wave w takes the rows that start
  // in [w*nnz/W, (w+1)*nnz/W) of the element stream (W waves), found by a
  // 32-ary search of indptr (lanes 0-31 for the start, 32-63 for the end).
  // With a monotone indptr the ranges partition the rows; a range whose end
  // comes before its start can only come from a malformed indptr and is
  // reported.
  const int64_t total_waves = w_hi - w_lo;  // waves of this part
  const int64_t wv = gwv - w_lo;
  int64_t rw0, rw1;
  {
    const int half = lane >> 5, hl = lane & 31;
    const int64_t T = (wv + half) * a.nnz / total_waves;  // < 2^52: no overflow
    int64_t lo = 0, hi = a.n_rows;  // the first row r with indptr[r] >= T lies in [lo, hi]
    if (wv + half == 0) hi = 0;
    if (wv + half >= total_waves) lo = a.n_rows;
    while (__ballot(hi > lo) != 0) {  // at most five rounds: the interval shrinks 32-fold
      const int64_t step = hi > lo ? (hi - lo + 31) / 32 : 1;
      const int64_t pos = lo + hl * step;
      const bool probe = pos < hi;
      const int32_t v = probe ? a.indptr[pos] : 0;
      const uint64_t m = __ballot(probe && (int64_t)v < T);
      const int k = __popc(half ? (uint32_t)(m >> 32) : (uint32_t)m);  // probes below T
      if (hi > lo) {
        if (k == 0) {
          hi = lo;
        } else {
          const int64_t nlo = lo + (k - 1) * step + 1, nhi = lo + k * step;
          lo = nlo;
          hi = nhi < hi ? nhi : hi;
        }
      }
    }
    const uint32_t lo_l = (uint32_t)lo, lo_h = (uint32_t)((uint64_t)lo >> 32);
    rw0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo_h, 0) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(lo_l, 0));
    rw1 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo_h, 32) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(lo_l, 32));
  }
  uint32_t range_err = rw1 < rw0 ? (uint32_t)BS_FLAG_INDPTR : 0u;
  if (rw1 < rw0) rw1 = rw0;

  int32_t p_next = 0;
  if (rw0 < rw1) {
    const int g0 = (int)(rw1 - rw0 < a.G ? rw1 - rw0 : a.G);
    p_next = (lane <= g0) ? a.indptr[rw0 + lane] : 0;
  }
  // The wave's elements are one contiguous run (its rows are consecutive), so
  // the index stream is software-pipelined in 1,024-element chunks: while one
  // is processed, the next one's loads are in flight. With RA (windows
  // shorter than two chunks on average: wide sketches leave room for few
  // rows) the chunks are aligned to the run's start: a chunk that straddles
  // windows is loaded once and serves each of them (the slices outside a
  // window are skipped, the lanes outside it masked), so every index is
  // fetched once. Otherwise the chunks start at each window's start, which
  // re-fetches part of a chunk per window but processes no chunk twice (the
  // kernel is then bound by LDS, not by the fetch). Prefetch positions are
  // clamped into [0, nnz), so a malformed indptr can only waste a prefetch,
  // never read out of bounds; a chunk whose start differs from the
  // prefetched one reloads.
  const int64_t nnz = a.nnz;
  const int64_t wave_end = rw0 < rw1 ? (int64_t)a.indptr[rw1] : 0;  // prefetch bound only
  // Element positions fit 32 bits (nnz <= INT32_MAX), so every position and
  // row-start comparison below is a scalar 32-bit operation.
  constexpr uint32_t CH = kWave * kUnrollLds;  // elements per chunk
  uint32_t nidx[kUnrollLds], idx[kUnrollLds];
  uint32_t pf_base = UINT32_MAX;   // start of the chunk whose indices are in flight (nidx)
  uint32_t cur_base = UINT32_MAX;  // start of the chunk in idx
  uint32_t run0 = 0;               // the wave's first element: run-aligned chunks start at run0 + k CH
  auto prefetch = [&](uint32_t b) {
    pf_base = b;
    if ((int64_t)b + (int64_t)kWave * kUnrollLds <= nnz) {
      const int32_t* src = a.indices + b + lane;
#pragma unroll
      for (int u = 0; u < kUnrollLds; ++u) nidx[u] = (uint32_t)__builtin_nontemporal_load(src + u * kWave);
    } else {
      const uint32_t last = (uint32_t)(nnz - 1);
#pragma unroll
      for (int u = 0; u < kUnrollLds; ++u) {
        const uint32_t pos = b + (uint32_t)(u * kWave + lane);
        nidx[u] = (uint32_t)__builtin_nontemporal_load(a.indices + (pos < last ? pos : last));
      }
    }
  };
  if (rw0 < rw1 && nnz > 0) {
    const int32_t b = __builtin_amdgcn_readfirstlane(p_next);
    run0 = b < 0 ? 0u : (uint32_t)b;
    prefetch(run0);
  }
  const uint32_t row_bytes = (uint32_t)W32 * 4u;
  const uint32_t sk_b = lds_addr(sk), table_b = lds_addr(table);
  const uint32_t dmax = d32 - 1u;
  const uint32_t wbits = (uint32_t)bits - 5u;  // bits of a target's word index (N >= 64)
  // Largest index loaded. Every loaded element lies in [0, nnz) (tail loads
  // are clamped there), so an index outside [0, d) anywhere in the input is
  // reported, as with a per-element check.
  uint32_t imax = 0;
  for (int64_t r0 = rw0; r0 < rw1; r0 += a.G) {
    const int g = (int)(rw1 - r0 < a.G ? rw1 - r0 : a.G);
    const int32_t p = p_next;
    {  // row pointers of the next window, in flight while this one runs
      const int64_t r1 = r0 + a.G;
      const int gn = (int)(rw1 - r1 < a.G ? rw1 - r1 : a.G);
      p_next = (r1 < rw1 && lane <= gn) ? a.indptr[r1 + lane] : 0;
    }
    const int32_t prev = __shfl_up(p, 1);
    const bool bad = (lane <= g) && (p < 0 || (int64_t)p > a.nnz || (lane >= 1 && p < prev) ||
                                     (r0 == 0 && lane == 0 && p != 0));
    const bool window_bad = __ballot(bad) != 0;
    for (int w = lane; w < g * W32; w += kWave) sk[w] = 0u;
    if (lane < g) cnt[lane] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (window_bad) errbits |= BS_FLAG_INDPTR;
    if (!window_bad) {
      const uint32_t e0 = (uint32_t)__builtin_amdgcn_readfirstlane(p);
      const uint32_t e1 = (uint32_t)__builtin_amdgcn_readlane(p, g);
      // lanes 1 .. g-1 of p hold the window's row starts after the first
      const uint64_t starts = __ballot(lane >= 1 && lane < g);
      uint32_t c_prev = 0;  // row starts before the current slice
      // the run-aligned chunk holding e0 (a window starting before the run,
      // possible only with a malformed indptr, takes its own chunk), or e0
      const uint32_t base0 = RA && e0 >= run0 ? run0 + (e0 - run0) / CH * CH : e0;
      for (uint32_t base = base0; base < e1; base += CH) {
        // Element u of lane l sits at base + u*64 + l; the window holds
        // positions [e0, e1). A chunk inside the window has no per-element
        // branches; otherwise the 64-element slices outside the window are
        // skipped with a uniform branch and the lanes of the partial slices
        // masked. An index outside [0, d) is flagged and clamped (the output
        // is then undefined) so the table read stays inside LDS.
        if (!RA || cur_base != base) {
          if (pf_base != base) prefetch(base);
#pragma unroll
          for (int u = 0; u < kUnrollLds; ++u) idx[u] = nidx[u];
          cur_base = base;
          // the next chunk: the run's next, or (window-aligned) this window's
          // next or else the next window's start
          const uint32_t next = (RA || e1 - base > CH) ? base + CH : e1;
          if ((int64_t)next < wave_end) prefetch(next);
          else pf_base = UINT32_MAX;
        }
        const uint32_t lo_off = RA && e0 > base ? e0 - base : 0u;  // first window position in the chunk
        auto chunk = [&](auto full_tag) {
          constexpr bool FULL = decltype(full_tag)::value;
          const uint32_t rem = FULL ? CH : (e1 - base < CH ? e1 - base : CH);
          // Stage-row LDS byte address of each lane's element in slice u: the
          // row starts up to the slice's last element are counted with one
          // ballot; each start inside the slice moves the lanes at and past
          // it one row on (rows are longer than a slice on average, so this
          // is rarely more than one step). Slices are taken in order.
          auto slice_rows = [&](int u) {
            const uint32_t s0 = base + (uint32_t)(u * kWave);
            const uint32_t c_hi = (uint32_t)__popcll(__ballot((uint32_t)p <= s0 + (kWave - 1)) & starts);
            uint32_t ro = sk_b + c_prev * row_bytes;
            if (c_hi != c_prev) {  // wave-uniform; starts c_prev+1 .. c_hi lie in the slice
              uint32_t i = c_prev;
              do {
                ++i;
                ro += (uint32_t)lane >= (uint32_t)__builtin_amdgcn_readlane(p, i) - s0 ? row_bytes : 0u;
              } while (i != c_hi);
            }
            c_prev = c_hi;
            return ro;
          };
          // table word pairs, half a chunk at a time: addresses, then 16 reads
          // in flight, then use (half keeps the registers within budget while
          // the next chunk's loads are outstanding)
          constexpr int H = kUnrollLds / 2;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (!FULL && (uint32_t)(h * H * kWave) >= rem) break;  // wave-uniform: the rest is past the end
            if (!FULL && (uint32_t)((h + 1) * H * kWave) <= lo_off) continue;  // wave-uniform: before the window
            uint32_t bp[H], lo[H], hi[H];
#pragma unroll
            for (int v = 0; v < H; ++v) {
              const int u = h * H + v;
              imax = idx[u] > imax ? idx[u] : imax;
              bp[v] = __umul24(idx[u] < dmax ? idx[u] : dmax, (uint32_t)bits);
            }
#pragma unroll
            for (int v = 0; v < H; ++v) {
              const int u = h * H + v;
              // wave-uniform: no table read for a slice outside the window
              if (!FULL && ((uint32_t)((u + 1) * kWave) <= lo_off || (uint32_t)(u * kWave) >= rem)) continue;
              const lds_u32* tw = lds_ptr(table_b + ((bp[v] >> 5) << 2));
              lo[v] = tw[0];
              hi[v] = tw[1];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int v = 0; v < H; ++v) {
              const int u = h * H + v;
              if (!FULL && (uint32_t)(u * kWave) >= rem) break;  // wave-uniform
              // wave-uniform: a slice before the window (it holds no row start)
              if (!FULL && (uint32_t)((u + 1) * kWave) <= lo_off) continue;
              const uint32_t ro = slice_rows(u);
              // target in the low `bits` bits of t (higher bits are the next
              // entries): word t[bits-1:5] of the row, bit t[4:0]
              const uint32_t t = __builtin_amdgcn_alignbit(hi[v], lo[v], bp[v]);
              const uint32_t addr = ro + (__builtin_amdgcn_ubfe(t, 5, wbits) << 2);
              const uint32_t pos = (uint32_t)(u * kWave + lane);
              if (FULL || (pos < rem && pos >= lo_off))
                __atomic_fetch_or(lds_ptr(addr), 1u << (t & 31), __ATOMIC_RELAXED);
            }
          }
        };
        if (lo_off == 0 && e1 - base >= CH) chunk(std::true_type());
        else chunk(std::false_type());
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int W64 = W32 / 2;
    const uint64_t* s64 = reinterpret_cast<const uint64_t*>(sk);
    uint64_t* o64 = reinterpret_cast<uint64_t*>(a.out32 + (size_t)r0 * W32);
    for (int w = lane; w < g * W64; w += kWave) {
      const uint64_t v = s64[w];
      __builtin_nontemporal_store(v, o64 + w);
      if (a.pop) atomicAdd(&cnt[w / W64], (uint32_t)__builtin_popcountll(v));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (a.pop && lane < g) a.pop[r0 + lane] = (int32_t)cnt[lane];
  }
  if (imax > dmax) errbits |= BS_FLAG_INDEX;
  errbits |= range_err;
  if (a.err && errbits) atomicOr(a.err, (int32_t)errbits);
}

}  // namespace
}  // namespace bs

namespace bs {
namespace {
// Packed-map geometry for (d, N); table_words includes one pad word.
inline int map_bits(int32_t N) {
  int bits = 1;
  while ((1LL << bits) < (long long)N) ++bits;
  return bits;
}
inline int64_t map_table_words(int64_t d, int32_t N) { return (d + 31) / 32 * map_bits(N) + 1; }
}  // namespace
}  // namespace bs

namespace bs {

bs_status sketch_item_check(const SketchItem& it) {
  if (it.n_rows < 0 || it.nnz < 0 || it.nnz > INT32_MAX || it.d < 1 || it.d > INT32_MAX || !valid_width(it.N))
    return BS_ERR_ARG;
  if (!it.indptr || !it.pi || (!it.indices && it.nnz > 0) || (!it.sketches && it.n_rows > 0)) return BS_ERR_NULL;
  return BS_OK;
}

struct SketchGroup {
  const SketchArgs* items = nullptr;
  const int64_t* woff = nullptr;
  int32_t n = 0;
  int64_t total = 0;
  int32_t wave_words = 0;
  int64_t grid = 0;
  const PackItem* packs = nullptr;  // maps to pack to 16 bits first
  const int64_t* poff = nullptr;
  int32_t n_packs = 0;
  int64_t pack_blocks = 0;
  int64_t pack_grid = 0;
};

size_t sketch_group_meta_bytes(int32_t n) {
  if (n < 0) return 0;
  return align256((size_t)n * sizeof(SketchArgs)) + align256(((size_t)n + 1) * sizeof(int64_t)) +
         align256((size_t)n * sizeof(PackItem)) + align256(((size_t)n + 1) * sizeof(int64_t));
}

bs_status sketch_group_create(const SketchItem* items, int32_t n, void* meta, size_t meta_bytes, bool persistent,
                              SketchGroup** out) {
  if (!out) return BS_ERR_NULL;
  *out = nullptr;
  if (n < 0) return BS_ERR_ARG;
  if (n > 0 && (!items || !meta)) return BS_ERR_NULL;
  if (meta_bytes < sketch_group_meta_bytes(n) || (reinterpret_cast<uintptr_t>(meta) & 255)) return BS_ERR_WORKSPACE;
  std::vector<SketchArgs> args(n);
  std::vector<int64_t> woff((size_t)n + 1);
  std::vector<PackItem> packs;
  std::vector<int64_t> poff(1, 0);
  int64_t total = 0;
  int32_t wave_words = 1;
  for (int32_t i = 0; i < n; ++i) {
    const bs_status st = sketch_item_check(items[i]);
    if (st != BS_OK) return st;
    SketchArgs& a = args[i];
    a.indptr = items[i].indptr;
    a.indices = items[i].indices;
    a.pi = items[i].pi;
    a.pi16 = items[i].pi16;
    if (items[i].pi16) {  // each packed map once (items may share one)
      bool seen = false;
      for (const PackItem& pk : packs) seen = seen || pk.out == items[i].pi16;
      if (!seen) {
        packs.push_back(PackItem{items[i].pi, items[i].pi16, items[i].d, items[i].N, items[i].err});
        poff.push_back(poff.back() + (items[i].d + 1023) / 1024);
      }
    }
    a.out32 = reinterpret_cast<uint32_t*>(items[i].sketches);
    a.pop = items[i].popcounts;
    a.err = items[i].err;
    a.n_rows = items[i].n_rows;
    a.nnz = items[i].nnz;
    a.d = items[i].d;
    a.N = items[i].N;
    a.W32 = items[i].N / 32;
    int G = kStageWords / a.W32;
    a.G = G < 1 ? 1 : (G > kMaxRowsPerWave ? kMaxRowsPerWave : G);
    a.stride = a.G * a.W32 + a.G;
    wave_words = a.stride > wave_words ? a.stride : wave_words;
    woff[i] = total;
    total += (a.n_rows + a.G - 1) / a.G;
  }
  woff[n] = total;
  std::unique_ptr<SketchGroup> g(new SketchGroup);
  char* m = static_cast<char*>(meta);
  std::vector<char> host(sketch_group_meta_bytes(n), 0);
  const size_t args_bytes = align256((size_t)n * sizeof(SketchArgs));
  const size_t woff_bytes = align256(((size_t)n + 1) * sizeof(int64_t));
  const size_t packs_bytes = align256((size_t)n * sizeof(PackItem));
  if (n > 0) memcpy(host.data(), args.data(), (size_t)n * sizeof(SketchArgs));
  memcpy(host.data() + args_bytes, woff.data(), woff.size() * sizeof(int64_t));
  if (!packs.empty()) memcpy(host.data() + args_bytes + woff_bytes, packs.data(), packs.size() * sizeof(PackItem));
  memcpy(host.data() + args_bytes + woff_bytes + packs_bytes, poff.data(), poff.size() * sizeof(int64_t));
  if (!host.empty() && hipMemcpy(meta, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return BS_ERR_HIP;
  g->items = reinterpret_cast<const SketchArgs*>(m);
  g->woff = reinterpret_cast<const int64_t*>(m + args_bytes);
  g->packs = reinterpret_cast<const PackItem*>(m + args_bytes + woff_bytes);
  g->poff = reinterpret_cast<const int64_t*>(m + args_bytes + woff_bytes + packs_bytes);
  g->n_packs = (int32_t)packs.size();
  g->pack_blocks = poff.back();
  g->n = n;
  g->total = total;
  g->wave_words = wave_words;
  const int64_t blocks = (total + kWavesPerBlock - 1) / kWavesPerBlock;
  g->grid = blocks;
  if (persistent && blocks > 0) {
    int lds_max = 0, n_cu = 0;
    device_limits(&lds_max, &n_cu);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)sketch_group_kernel, kWavesPerBlock * kWave,
                                                      (size_t)kWavesPerBlock * wave_words * 4) != hipSuccess ||
        nb < 1)
      nb = 1;
    const int64_t cap = (int64_t)nb * (n_cu > 0 ? n_cu : 1);
    if (g->grid > cap) g->grid = cap;
  }
  g->pack_grid = g->pack_blocks;
  if (persistent) {
    int lds_max = 0, n_cu = 0;
    device_limits(&lds_max, &n_cu);
    const int64_t cap = (int64_t)8 * (n_cu > 0 ? n_cu : 1);
    if (g->pack_grid > cap) g->pack_grid = cap;
  }
  *out = g.release();
  return BS_OK;
}

bs_status sketch_group_launch(const SketchGroup* g, hipStream_t s) {
  if (!g) return BS_ERR_NULL;
  if (g->total == 0) return BS_OK;
  if (g->grid > INT32_MAX || g->pack_grid > INT32_MAX) return BS_ERR_ARG;
  if (g->pack_blocks > 0) {
    ScopedTiming timing("sketch_pack16", s);
    hipLaunchKernelGGL(pack16_group_kernel, dim3((unsigned)g->pack_grid), dim3(256), 0, s, g->packs, g->poff,
                       g->n_packs, g->pack_blocks);
  }
  ScopedTiming timing("sketch_group", s);
  hipLaunchKernelGGL(sketch_group_kernel, dim3((unsigned)g->grid), dim3(kWavesPerBlock * kWave),
                     (size_t)kWavesPerBlock * g->wave_words * 4, s, g->items, g->woff, g->n, g->total,
                     g->wave_words);
  return launch_status();
}

void sketch_group_destroy(SketchGroup* g) { delete g; }

}  // namespace bs

extern "C" size_t bs_sketch_workspace_size(int64_t d, int32_t N) {
  using namespace bs;
  if (d < 1 || d > INT32_MAX || !valid_width(N)) return 0;
  return align256((size_t)map_table_words(d, N) * 4);
}

namespace bs {
namespace {

// Waves per part in proportion to its set bits plus rows; a part with rows
// always gets at least one. wave_off[i] is the first wave of part i.
void split_waves(const bs_sketch_part* parts, int32_t n_parts, int64_t total, int32_t* wave_off) {
  int64_t wt[kMaxParts] = {}, w[kMaxParts] = {}, wsum = 0, used = 0;
  for (int i = 0; i < n_parts; ++i) {
    wt[i] = parts[i].n_rows > 0 ? parts[i].nnz + parts[i].n_rows : 0;
    wsum += wt[i];
  }
  for (int i = 0; i < n_parts; ++i) {
    if (wt[i] == 0) continue;
    w[i] = total * wt[i] / wsum;
    if (w[i] < 1) w[i] = 1;
    used += w[i];
  }
  while (used > total) {  // total >= the parts with rows, so a part with two or more waves exists
    int j = -1;
    for (int i = 0; i < n_parts; ++i)
      if (w[i] > 1 && (j < 0 || w[i] > w[j])) j = i;
    --w[j];
    --used;
  }
  while (used < total) {  // the rest to the parts with the most weight per wave
    int j = -1;
    for (int i = 0; i < n_parts; ++i)
      if (wt[i] > 0 && (j < 0 || wt[i] * w[j] > wt[j] * w[i])) j = i;
    ++w[j];
    ++used;
  }
  wave_off[0] = 0;
  for (int i = 0; i < kMaxParts; ++i) wave_off[i + 1] = wave_off[i] + (int32_t)(i < n_parts ? w[i] : 0);
}

// packed: the workspace already holds pi packed by bs_sketch_prepare_map
// (no pack launch; pi's values were checked then).
bs_status sketch_parts_impl(const bs_sketch_part* parts, int32_t n_parts, const int32_t* pi, int64_t d, int32_t N,
                            int32_t* err_flag, void* workspace, size_t workspace_bytes, void* stream,
                            bool packed = false) {
  if (n_parts < 1 || n_parts > kMaxParts || d < 1 || d > INT32_MAX || !valid_width(N)) return BS_ERR_ARG;
  if (!parts) return BS_ERR_NULL;
  for (int i = 0; i < n_parts; ++i)
    if (parts[i].n_rows < 0 || parts[i].nnz < 0 || parts[i].nnz > INT32_MAX) return BS_ERR_ARG;
  if (!pi) return BS_ERR_NULL;
  for (int i = 0; i < n_parts; ++i)
    if (!parts[i].indptr || (!parts[i].indices && parts[i].nnz > 0) || (!parts[i].sketches && parts[i].n_rows > 0))
      return BS_ERR_NULL;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  int64_t rows_total = 0;
  for (int i = 0; i < n_parts; ++i) rows_total += parts[i].n_rows;
  if (rows_total == 0) return BS_OK;

  auto part_args = [&](const bs_sketch_part& pt, int32_t G) {
    SketchArgs a;
    a.indptr = pt.indptr;
    a.indices = pt.indices;
    a.pi = pi;
    a.pi16 = nullptr;
    a.out32 = reinterpret_cast<uint32_t*>(pt.sketches);
    a.pop = pt.popcounts;
    a.err = err_flag;
    a.n_rows = pt.n_rows;
    a.nnz = pt.nnz;
    a.d = d;
    a.N = N;
    a.W32 = N / 32;
    a.G = G;
    a.stride = G * a.W32 + G;
    return a;
  };

  // Map-in-LDS path when the bit-packed map leaves room for staging.
  int lds_max = 0, n_cu = 0;
  device_limits(&lds_max, &n_cu);
  const int bits = map_bits(N);
  const int64_t table_words = map_table_words(d, N);
  const int64_t W32 = N / 32;
  const int64_t table_bytes = table_words * 4;
  const int64_t stage_bytes_per_wave = ((int64_t)lds_max - table_bytes) / kBigBlockWaves;
  int64_t Gl = stage_bytes_per_wave / (4 * (W32 + 1));
  if (Gl > 16) Gl = 16;
  const bool have_ws = workspace && workspace_bytes >= (size_t)table_words * 4 &&
                       (reinterpret_cast<uintptr_t>(workspace) & 15) == 0;
  if (have_ws && n_cu > 0 && Gl >= 1 && table_words < (INT64_C(1) << 26)) {
    SketchLdsArgs L;
    memset(&L, 0, sizeof(L));
    L.n_parts = n_parts;
    L.n_windows = 0;
    for (int i = 0; i < n_parts; ++i) {
      L.s[i] = part_args(parts[i], (int32_t)Gl);
      L.n_windows += (parts[i].n_rows + Gl - 1) / Gl;
    }
    L.bits = bits;
    L.packed = static_cast<const uint32_t*>(workspace);
    L.table_words = (int32_t)table_words;
    const size_t lds = (size_t)table_bytes + (size_t)kBigBlockWaves * L.s[0].stride * 4;
    // one block per CU; fewer when there is less than one window per wave
    int64_t grid = (L.n_windows + kBigBlockWaves - 1) / kBigBlockWaves;
    if (grid > n_cu) grid = n_cu;
    if (grid < 1) grid = 1;
    if ((size_t)lds <= (size_t)lds_max) {
      split_waves(parts, n_parts, grid * kBigBlockWaves, L.wave_off);
      // short windows (on average under two index chunks): run-aligned chunks
      int64_t rows = 0, nnz = 0;
      for (int i = 0; i < n_parts; ++i) {
        rows += parts[i].n_rows;
        nnz += parts[i].nnz;
      }
      const bool ra = nnz * Gl < INT64_C(2) * kWave * kUnrollLds * rows;
      const void* fn = ra ? (const void*)sketch_csr_lds_kernel<true> : (const void*)sketch_csr_lds_kernel<false>;
      if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (!packed) {
        const int64_t n_groups = (d + 31) / 32;
        ScopedTiming timing("sketch_pack", as_stream(stream));
        hipLaunchKernelGGL(pack_map_kernel, dim3((unsigned)((n_groups + 255) / 256)), dim3(256), 0,
                           as_stream(stream), pi, d, N, bits, static_cast<uint32_t*>(workspace), err_flag);
      }
      ScopedTiming timing("sketch_csr", as_stream(stream));
      if (ra)
        hipLaunchKernelGGL(sketch_csr_lds_kernel<true>, dim3((unsigned)grid), dim3(kBigBlockWaves * kWave), lds,
                           as_stream(stream), L);
      else
        hipLaunchKernelGGL(sketch_csr_lds_kernel<false>, dim3((unsigned)grid), dim3(kBigBlockWaves * kWave), lds,
                           as_stream(stream), L);
      return launch_status();
    }
  }

  // map gathered through L2: one launch per part
  int G = kStageWords / (N / 32);
  G = G < 1 ? 1 : (G > kMaxRowsPerWave ? kMaxRowsPerWave : G);
  for (int i = 0; i < n_parts; ++i) {
    if (parts[i].n_rows == 0) continue;
    const SketchArgs a = part_args(parts[i], G);
    const int64_t waves = (a.n_rows + a.G - 1) / a.G;
    const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > INT32_MAX) return BS_ERR_ARG;
    const size_t lds_bytes = (size_t)kWavesPerBlock * a.stride * sizeof(uint32_t);
    ScopedTiming timing("sketch_csr", as_stream(stream));
    hipLaunchKernelGGL(sketch_csr_kernel, dim3((unsigned)blocks), dim3(kWavesPerBlock * kWave), lds_bytes,
                       as_stream(stream), a);
    st = launch_status();
    if (st != BS_OK) return st;
  }
  return BS_OK;
}

}  // namespace
}  // namespace bs

extern "C" bs_status bs_sketch(const int32_t* indptr, const int32_t* indices, int64_t n_rows,
                               int64_t nnz, const int32_t* pi, int64_t d, int32_t N,
                               uint64_t* sketches, int32_t* popcounts, int32_t* err_flag,
                               void* workspace, size_t workspace_bytes, void* stream) {
  const bs_sketch_part part = {indptr, indices, n_rows, nnz, sketches, popcounts};
  return bs::sketch_parts_impl(&part, 1, pi, d, N, err_flag, workspace, workspace_bytes, stream);
}

extern "C" bs_status bs_sketch_parts(const bs_sketch_part* parts, int32_t n_parts, const int32_t* pi, int64_t d,
                                     int32_t N, int32_t* err_flag, void* workspace, size_t workspace_bytes,
                                     void* stream) {
  return bs::sketch_parts_impl(parts, n_parts, pi, d, N, err_flag, workspace, workspace_bytes, stream);
}

extern "C" bs_status bs_sketch_prepare_map(const int32_t* pi, int64_t d, int32_t N, int32_t* err_flag, void* map,
                                           size_t map_bytes, void* stream) {
  using namespace bs;
  if (d < 1 || d > INT32_MAX || !valid_width(N)) return BS_ERR_ARG;
  if (!pi) return BS_ERR_NULL;
  if (!map || map_bytes < bs_sketch_workspace_size(d, N) || (reinterpret_cast<uintptr_t>(map) & 15))
    return BS_ERR_WORKSPACE;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  const int64_t n_groups = (d + 31) / 32;
  ScopedTiming timing("sketch_pack", as_stream(stream));
  hipLaunchKernelGGL(pack_map_kernel, dim3((unsigned)((n_groups + 255) / 256)), dim3(256), 0, as_stream(stream), pi,
                     d, N, map_bits(N), static_cast<uint32_t*>(map), err_flag);
  return launch_status();
}

extern "C" bs_status bs_sketch_parts_prepared(const bs_sketch_part* parts, int32_t n_parts, const int32_t* pi,
                                              int64_t d, int32_t N, const void* map, size_t map_bytes,
                                              int32_t* err_flag, void* stream) {
  using namespace bs;
  if (!map || map_bytes < bs_sketch_workspace_size(d, N) || (reinterpret_cast<uintptr_t>(map) & 15))
    return (d < 1 || d > INT32_MAX || !valid_width(N)) ? BS_ERR_ARG : BS_ERR_WORKSPACE;
  return sketch_parts_impl(parts, n_parts, pi, d, N, err_flag, const_cast<void*>(map), map_bytes, stream, true);
}
