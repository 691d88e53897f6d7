// All-pairs sketch inner products and estimates on gfx950.
//
// <a_s, b_s> = |a_s AND b_s| (Algorithm 1, second step) is bit work, not a
// floating-point contraction, so it runs on the vector ALU: per 32-bit word
// pair one v_and_b32 and one v_bcnt_u32_b32 (which also accumulates).
//
// Mapping: one lane per B row, whose words sit in VGPRs; the A rows are
// wave-uniform, so their words are fetched by the scalar unit (s_load) and
// feed the VALU as SGPR operands at no vector-memory or LDS cost. Lanes of a
// wave hold consecutive B rows, so every output row segment is a coalesced
// 64-lane store.
//
// Estimator epilogue (Algorithms 1-4, canonical form): with
// T(x) = ln(1 - x/N) / ln(1 - 1/N) tabulated for x = 0..N (T(N) := T(N-1),
// the saturation clamp), and x_u = x_a + x_b - x_ab = |a_s OR b_s|,
//   s = T(x_a) + T(x_b),  ip = s - T(x_u),  ham = s - 2 ip,
//   js = ip / (ip + ham),  cos = ip / sqrt(T(x_a) T(x_b)).
#include <mutex>

#include "bs_common.h"

namespace bs {

// T(x) for x in [0, N] in FP64 and FP32 (the FP32 table is the FP64 value
// rounded once). Both forms log1p(-x/N) and log(1-x/N) take the logarithm of
// the same exactly representable number when N is a power of two.
__global__ void build_lut_kernel(int32_t N, double* __restrict__ t64, float* __restrict__ t32) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > N) return;
  const double v = t_value(x, N);
  if (t64) t64[x] = v;
  if (t32) t32[x] = (float)v;
}

// popcount of each row of X[n][W32] (32-bit words).
__global__ void row_popcount_kernel(const uint32_t* __restrict__ X, int64_t n, int32_t W32,
                                    int32_t* __restrict__ pop) {
  // one wave per row: lanes sum strided words, then a wave reduction
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= n) return;
  const uint32_t* x = X + (size_t)row * W32;
  uint32_t c = 0;
  for (int w = lane; w < W32; w += kWave) c += popc32(x[w]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) pop[row] = (int32_t)c;
}

// out[i] = |A[ia[i]] AND B[ib[i]]| for listed pairs (one thread per pair).
__global__ void pair_list_kernel(const uint64_t* __restrict__ A, int64_t nA, const int32_t* __restrict__ ia,
                                 const uint64_t* __restrict__ B, int64_t nB, const int32_t* __restrict__ ib,
                                 int64_t n, int32_t W64, int32_t* __restrict__ out, int32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = ia[i], q = ib[i];
  if (p < 0 || p >= nA || q < 0 || q >= nB) {  // out-of-range row: reported, output 0
    out[i] = 0;
    if (err) atomicOr(err, 1);
    return;
  }
  const uint64_t* a = A + (size_t)p * W64;
  const uint64_t* b = B + (size_t)q * W64;
  uint32_t c = 0;
  for (int w = 0; w < W64; ++w) c += (uint32_t)__builtin_popcountll(a[w] & b[w]);
  out[i] = (int32_t)c;
}

void launch_lut(int32_t N, double* t64, float* t32, hipStream_t s) {
  const int threads = 256;
  hipLaunchKernelGGL(build_lut_kernel, dim3((N + 1 + threads - 1) / threads), dim3(threads), 0, s, N,
                     t64, t32);
}

void launch_row_popcount(const uint64_t* X, int64_t n, int32_t N, int32_t* pop, hipStream_t s) {
  if (n <= 0) return;
  const int rows_per_block = 4;
  hipLaunchKernelGGL(row_popcount_kernel, dim3((unsigned)((n + rows_per_block - 1) / rows_per_block)),
                     dim3(rows_per_block * kWave), 0, s, reinterpret_cast<const uint32_t*>(X), n, N / 32,
                     pop);
}

namespace {

constexpr int kPairThreads = 256;

struct DenseArgs {
  const uint32_t* __restrict__ A;  // [nA][W32]
  const uint32_t* __restrict__ B;  // [nB][W32]
  const int32_t* __restrict__ popA;
  const int32_t* __restrict__ popB;
  const double* __restrict__ t64;  // T(0..N) (mode 1)
  const float* __restrict__ t32;   // T(0..N) rounded to float (mode 2)
  int32_t* __restrict__ xab_out;   // [nA][nB] (mode 0)
  float* __restrict__ f32;         // [nA][nB] (mode 2): one measure, FP32
  double* __restrict__ ip;         // [nA][nB] (mode 1), each may be null
  double* __restrict__ ham;
  double* __restrict__ js;
  double* __restrict__ cs;
  int64_t nA, nB;
  int32_t W32;
  int32_t a_per_block;
};

// WC: 32-bit words of B held in VGPRs per chunk; TA: A rows per tile.
// MODE 0: counts x_ab; 1: FP64 estimates (any of the four planes); 2: the
// FP32 score of measure M (the value bs_topk ranks by).
template <int WC, int TA, int MODE, int M>
__global__ __launch_bounds__(kPairThreads) void pair_dense_kernel(DenseArgs a) {
  constexpr bool EST = MODE != 0;
  const int64_t b = (int64_t)blockIdx.x * kPairThreads + threadIdx.x;
  const bool b_ok = b < a.nB;
  const int64_t bb = b_ok ? b : a.nB - 1;
  const int64_t a_begin = (int64_t)blockIdx.y * a.a_per_block;
  if (a_begin >= a.nA) return;
  const int64_t a_end = a_begin + a.a_per_block < a.nA ? a_begin + a.a_per_block : a.nA;
  const int W32 = a.W32;
  const int nchunks = W32 / WC;
  const uint32_t* brow = a.B + (size_t)bb * W32;

  double Tb = 0.0;
  float Tb32 = 0.0f;
  int32_t xb = 0;
  if (EST) xb = a.popB[bb];
  if (MODE == 1) Tb = a.t64[xb];
  if (MODE == 2) Tb32 = a.t32[xb];

  uint32_t bw[WC];
  if (nchunks == 1) {
#pragma unroll
    for (int w = 0; w < WC; ++w) bw[w] = brow[w];
  }
  for (int64_t a0 = a_begin; a0 < a_end; a0 += TA) {
    uint32_t acc[TA];
#pragma unroll
    for (int t = 0; t < TA; ++t) acc[t] = 0;
    for (int c = 0; c < nchunks; ++c) {
      if (nchunks != 1) {
#pragma unroll
        for (int w = 0; w < WC; ++w) bw[w] = brow[c * WC + w];
      }
#pragma unroll
      for (int t = 0; t < TA; ++t) {
        const int64_t ar = (a0 + t < a_end) ? a0 + t : a_end - 1;
        const cptr<uint32_t> arow = as_const(a.A + (size_t)ar * W32 + c * WC);
#pragma unroll
        for (int w = 0; w < WC; ++w) acc[t] = bcnt_add(arow[w] & bw[w], acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < TA; ++t) {
      const int64_t ar = a0 + t;
      if (ar >= a_end || !b_ok) continue;
      const size_t o = (size_t)ar * a.nB + b;
      if (MODE == 0) {
        __builtin_nontemporal_store((int32_t)acc[t], a.xab_out + o);
      } else if (MODE == 2) {
        const int32_t xa = as_const(a.popA)[ar];
        const float sc = score_f32<M>(a.t32[xa], Tb32, a.t32[xa + xb - (int32_t)acc[t]]);
        __builtin_nontemporal_store(sc, a.f32 + o);
      } else {
        const int32_t xa = as_const(a.popA)[ar];
        const double Ta = a.t64[xa];
        const double Tu = a.t64[xa + xb - (int32_t)acc[t]];
        const double s = Ta + Tb;
        const double ip = s - Tu;
        const double ham = s - 2.0 * ip;
        if (a.ip) __builtin_nontemporal_store(ip, a.ip + o);
        if (a.ham) __builtin_nontemporal_store(ham, a.ham + o);
        if (a.js) {
          const double den = ip + ham;
          __builtin_nontemporal_store(den == 0.0 ? 0.0 : ip / den, a.js + o);
        }
        if (a.cs) {
          const double pr = Ta * Tb;
          __builtin_nontemporal_store(pr == 0.0 ? 0.0 : ip / sqrt(pr), a.cs + o);
        }
      }
    }
  }
}

template <int MODE, int M = 0>
bs_status launch_dense(DenseArgs a, hipStream_t s, bool timed = true) {
  const int W32 = a.W32;
  // Largest power of two <= 64 that divides W32 (W32 is even).
  int WC = 64;
  while (W32 % WC) WC >>= 1;
  const int64_t bblocks = (a.nB + kPairThreads - 1) / kPairThreads;
  // Enough blocks to fill 256 CUs several times over; A tile rows multiple of 4.
  int64_t per = (a.nA * bblocks + 4095) / 4096;
  per = per < 4 ? 4 : (per > 256 ? 256 : per);
  per = (per + 3) / 4 * 4;
  a.a_per_block = (int32_t)per;
  const int64_t ablocks = (a.nA + per - 1) / per;
  if (bblocks > INT32_MAX || ablocks > 65535) return BS_ERR_ARG;
  dim3 grid((unsigned)bblocks, (unsigned)ablocks);
  dim3 block(kPairThreads);
  ScopedTiming timing(timed ? (MODE != 0 ? "pair_estimate" : "pair_and_popcount") : nullptr, s);
#define BS_DENSE_CASE(wc, ta)                                                          \
  case wc:                                                                             \
    hipLaunchKernelGGL((pair_dense_kernel<wc, ta, MODE, M>), grid, block, 0, s, a); \
    break;
  switch (WC) {
    BS_DENSE_CASE(2, 4)
    BS_DENSE_CASE(4, 4)
    BS_DENSE_CASE(8, 4)
    BS_DENSE_CASE(16, 4)
    BS_DENSE_CASE(32, 4)
    BS_DENSE_CASE(64, 4)
    default:
      return BS_ERR_ARG;
  }
#undef BS_DENSE_CASE
  return launch_status();
}

}  // namespace
}  // namespace bs

extern "C" bs_status bs_and_popcount(const uint64_t* A, int64_t nA, const uint64_t* B, int64_t nB,
                                     int32_t N, int32_t* out, void* stream) {
  using namespace bs;
  if (nA < 0 || nB < 0 || !valid_width(N)) return BS_ERR_ARG;
  if ((!A && nA > 0) || (!B && nB > 0) || (!out && nA > 0 && nB > 0)) return BS_ERR_NULL;
  if (nA > 0 && nB > (INT64_C(1) << 62) / nA) return BS_ERR_ARG;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  if (nA == 0 || nB == 0) return BS_OK;
  DenseArgs a = {};
  a.A = reinterpret_cast<const uint32_t*>(A);
  a.B = reinterpret_cast<const uint32_t*>(B);
  a.xab_out = out;
  a.nA = nA;
  a.nB = nB;
  a.W32 = N / 32;
  return launch_dense<0>(a, as_stream(stream));
}

// Fixed scratch of bs_estimate_noalloc: the T table and, when the caller
// passes none, the row popcounts. One copy per GPU, held until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[BS_NOALLOC_SCRATCH_BYTES];

namespace bs {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};  // device address of `scratch`, per device

// Address of the current device's copy of `scratch`, looked up on the first
// call on that device (with it current) and kept.
bs_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BS_ERR_HIP;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return BS_OK;
}

// Bytes of scratch bs_estimate needs: the FP64 T table, then the row
// popcounts that the caller did not pass.
// Saturates at SIZE_MAX (row counts are only bounded by nA * nB < 2^62).
size_t estimate_scratch_bytes(int64_t nA, int64_t nB, int32_t N, bool needA, bool needB) {
  const int64_t cap = INT64_C(1) << 40;
  if ((needA && nA > cap) || (needB && nB > cap)) return SIZE_MAX;
  return align256((size_t)(N + 1) * sizeof(double)) + (needA ? align256((size_t)nA * 4) : 0) +
         (needB ? align256((size_t)nB * 4) : 0);
}

bs_status estimate_check(const uint64_t* A, int64_t nA, const uint64_t* B, int64_t nB, int32_t N, const double* ip,
                         const double* ham, const double* js, const double* cos) {
  if (nA < 0 || nB < 0 || !valid_width(N)) return BS_ERR_ARG;
  if ((!A && nA > 0) || (!B && nB > 0)) return BS_ERR_NULL;
  if (!ip && !ham && !js && !cos) return BS_ERR_NULL;
  if (nA > 0 && nB > (INT64_C(1) << 62) / nA) return BS_ERR_ARG;
  return BS_OK;
}

// The estimate's launches: the FP64 T table into t64, the row popcounts the
// caller did not pass into wpopA / wpopB, then the dense estimate kernel.
bs_status estimate_run(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B, const int32_t* popB,
                       int64_t nB, int32_t N, double* ip, double* ham, double* js, double* cos, double* t64,
                       int32_t* wpopA, int32_t* wpopB, hipStream_t s, bool timed) {
  launch_lut(N, t64, nullptr, s);
  if (!popA) launch_row_popcount(A, nA, N, wpopA, s);
  if (!popB) launch_row_popcount(B, nB, N, wpopB, s);
  bs_status st = launch_status();
  if (st != BS_OK) return st;
  DenseArgs a = {};
  a.A = reinterpret_cast<const uint32_t*>(A);
  a.B = reinterpret_cast<const uint32_t*>(B);
  a.popA = popA ? popA : wpopA;
  a.popB = popB ? popB : wpopB;
  a.t64 = t64;
  a.ip = ip;
  a.ham = ham;
  a.js = js;
  a.cs = cos;
  a.nA = nA;
  a.nB = nB;
  a.W32 = N / 32;
  return launch_dense<1>(a, s, timed);
}

}  // namespace
}  // namespace bs

extern "C" size_t bs_estimate_workspace_size(int64_t nA, int64_t nB, int32_t N) {
  using namespace bs;
  if (!valid_width(N) || nA < 0 || nB < 0) return 0;
  return align256((size_t)(N + 1) * sizeof(double)) + align256((size_t)nA * 4) +
         align256((size_t)nB * 4);
}

extern "C" bs_status bs_estimate(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                                 const int32_t* popB, int64_t nB, int32_t N, double* ip, double* ham,
                                 double* js, double* cos, void* workspace, size_t workspace_bytes,
                                 void* stream) {
  using namespace bs;
  bs_status st = estimate_check(A, nA, B, nB, N, ip, ham, js, cos);
  if (st != BS_OK) return st;
  const size_t need = bs_estimate_workspace_size(nA, nB, N);
  if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return BS_ERR_WORKSPACE;
  st = check_device();
  if (st != BS_OK) return st;
  if (nA == 0 || nB == 0) return BS_OK;
  char* ws = static_cast<char*>(workspace);
  double* t64 = reinterpret_cast<double*>(ws);
  int32_t* wpopA = reinterpret_cast<int32_t*>(ws + align256((size_t)(N + 1) * sizeof(double)));
  int32_t* wpopB = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(wpopA) + align256((size_t)nA * 4));
  return estimate_run(A, popA, nA, B, popB, nB, N, ip, ham, js, cos, t64, wpopA, wpopB, as_stream(stream), true);
}

extern "C" bs_status bs_estimate_noalloc(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                                         const int32_t* popB, int64_t nB, int32_t N, double* ip, double* ham,
                                         double* js, double* cos, void* stream) {
  using namespace bs;
  bs_status st = estimate_check(A, nA, B, nB, N, ip, ham, js, cos);
  if (st != BS_OK) return st;
  if (estimate_scratch_bytes(nA, nB, N, !popA, !popB) > (size_t)BS_NOALLOC_SCRATCH_BYTES) return BS_ERR_SCRATCH;
  st = check_device();
  if (st != BS_OK) return st;
  if (nA == 0 || nB == 0) return BS_OK;
  void* base = nullptr;
  st = noalloc_scratch(&base);
  if (st != BS_OK) return st;
  // scratch layout as estimate_scratch_bytes: T, then the missing popcounts;
  // every word is written before it is read, so nothing is cleared
  char* ws = static_cast<char*>(base);
  double* t64 = reinterpret_cast<double*>(ws);
  ws += align256((size_t)(N + 1) * sizeof(double));
  int32_t* wpopA = popA ? nullptr : reinterpret_cast<int32_t*>(ws);
  if (!popA) ws += align256((size_t)nA * 4);
  int32_t* wpopB = popB ? nullptr : reinterpret_cast<int32_t*>(ws);
  return estimate_run(A, popA, nA, B, popB, nB, N, ip, ham, js, cos, t64, wpopA, wpopB, as_stream(stream), false);
}

extern "C" bs_status bs_estimate_scores(const uint64_t* A, const int32_t* popA, int64_t nA, const uint64_t* B,
                                        const int32_t* popB, int64_t nB, int32_t N, int32_t measure, void* scores,
                                        int32_t score_dtype, void* workspace, size_t workspace_bytes, void* stream) {
  using namespace bs;
  if (measure < BS_IP || measure > BS_COSINE || (score_dtype != BS_F64 && score_dtype != BS_F32)) return BS_ERR_ARG;
  if (score_dtype == BS_F64) {
    double* out = static_cast<double*>(scores);
    return bs_estimate(A, popA, nA, B, popB, nB, N, measure == BS_IP ? out : nullptr,
                       measure == BS_HAMMING ? out : nullptr, measure == BS_JACCARD ? out : nullptr,
                       measure == BS_COSINE ? out : nullptr, workspace, workspace_bytes, stream);
  }
  float* out = static_cast<float*>(scores);
  if (nA < 0 || nB < 0 || !valid_width(N)) return BS_ERR_ARG;
  if ((!A && nA > 0) || (!B && nB > 0) || !out) return BS_ERR_NULL;
  if (nA > 0 && nB > (INT64_C(1) << 62) / nA) return BS_ERR_ARG;
  bs_status st = BS_OK;
  const size_t need = bs_estimate_workspace_size(nA, nB, N);
  if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return BS_ERR_WORKSPACE;
  st = check_device();
  if (st != BS_OK) return st;
  if (nA == 0 || nB == 0) return BS_OK;
  // the workspace layout of bs_estimate, with the FP32 table in the FP64 table's place
  char* ws = static_cast<char*>(workspace);
  float* t32 = reinterpret_cast<float*>(ws);
  int32_t* wpopA = reinterpret_cast<int32_t*>(ws + align256((size_t)(N + 1) * sizeof(double)));
  int32_t* wpopB = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(wpopA) + align256((size_t)nA * 4));
  hipStream_t s = as_stream(stream);
  launch_lut(N, nullptr, t32, s);
  if (!popA) launch_row_popcount(A, nA, N, wpopA, s);
  if (!popB) launch_row_popcount(B, nB, N, wpopB, s);
  st = launch_status();
  if (st != BS_OK) return st;
  DenseArgs a = {};
  a.A = reinterpret_cast<const uint32_t*>(A);
  a.B = reinterpret_cast<const uint32_t*>(B);
  a.popA = popA ? popA : wpopA;
  a.popB = popB ? popB : wpopB;
  a.t32 = t32;
  a.f32 = out;
  a.nA = nA;
  a.nB = nB;
  a.W32 = N / 32;
  switch (measure) {
    case BS_IP: return launch_dense<2, BS_IP>(a, s);
    case BS_HAMMING: return launch_dense<2, BS_HAMMING>(a, s);
    case BS_JACCARD: return launch_dense<2, BS_JACCARD>(a, s);
    default: return launch_dense<2, BS_COSINE>(a, s);
  }
}

extern "C" bs_status bs_pair_popcount(const uint64_t* A, int64_t nA, const int32_t* ia, const uint64_t* B,
                                      int64_t nB, const int32_t* ib, int64_t n_pairs, int32_t N, int32_t* out,
                                      int32_t* err_flag, void* stream) {
  using namespace bs;
  if (nA < 0 || nB < 0 || n_pairs < 0 || !valid_width(N)) return BS_ERR_ARG;
  if (n_pairs > 0 && (!A || !B || !ia || !ib || !out)) return BS_ERR_NULL;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  if (n_pairs == 0) return BS_OK;
  const int64_t blocks = (n_pairs + 255) / 256;
  if (blocks > INT32_MAX) return BS_ERR_ARG;
  hipLaunchKernelGGL(pair_list_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), A, nA, ia, B, nB,
                     ib, n_pairs, N / 64, out, err_flag);
  return launch_status();
}
