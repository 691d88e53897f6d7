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
#include "bs_common.h"

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

__global__ __launch_bounds__(kWavesPerBlock * kWave) void sketch_csr_kernel(SketchArgs a) {
  extern __shared__ uint32_t lds[];
  const int wid = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  const int64_t r0 = wave * a.G;
  if (r0 >= a.n_rows) return;
  const int g = (int)(a.n_rows - r0 < a.G ? a.n_rows - r0 : a.G);
  const int W32 = a.W32;
  uint32_t* sk = lds + (size_t)wid * a.stride;
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
        j[u] = in[u] ? a.pi[idx[u]] : 0;
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
}

}  // namespace
}  // namespace bs

extern "C" bs_status bs_sketch(const int32_t* indptr, const int32_t* indices, int64_t n_rows,
                               int64_t nnz, const int32_t* pi, int64_t d, int32_t N,
                               uint64_t* sketches, int32_t* popcounts, int32_t* err_flag,
                               void* stream) {
  using namespace bs;
  if (n_rows < 0 || nnz < 0 || nnz > INT32_MAX || d < 1 || d > INT32_MAX || !valid_width(N))
    return BS_ERR_ARG;
  if (!indptr || !pi || (!indices && nnz > 0) || (!sketches && n_rows > 0)) return BS_ERR_NULL;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  if (n_rows == 0) return BS_OK;

  SketchArgs a;
  a.indptr = indptr;
  a.indices = indices;
  a.pi = pi;
  a.out32 = reinterpret_cast<uint32_t*>(sketches);
  a.pop = popcounts;
  a.err = err_flag;
  a.n_rows = n_rows;
  a.nnz = nnz;
  a.d = d;
  a.N = N;
  a.W32 = N / 32;
  int G = kStageWords / a.W32;
  a.G = G < 1 ? 1 : (G > kMaxRowsPerWave ? kMaxRowsPerWave : G);
  a.stride = a.G * a.W32 + a.G;
  const int64_t waves = (n_rows + a.G - 1) / a.G;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > INT32_MAX) return BS_ERR_ARG;
  const size_t lds_bytes = (size_t)kWavesPerBlock * a.stride * sizeof(uint32_t);
  ScopedTiming timing("sketch_csr", as_stream(stream));
  hipLaunchKernelGGL(sketch_csr_kernel, dim3((unsigned)blocks), dim3(kWavesPerBlock * kWave),
                     lds_bytes, as_stream(stream), a);
  return launch_status();
}
