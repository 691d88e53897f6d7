// Learned Jaccard estimator on gfx950: a 4 -> 64 -> 64 -> 1 ReLU network
// with BF16 weights and FP32 accumulation that corrects the closed-form
// Jaccard estimate (Algorithms 1-3, canonical FP32 form) where sketches
// saturate. Inputs per pair: the sketch counts |a_s|, |b_s|, |a_s AND b_s|
// (Algorithm 1, steps 1-2) and the width N.
//
//   f  = (x_a/N, x_b/N, x_ab/N, log2(N)/16)
//   z1 = W1 f + b1, h1 = relu(z1)                      (VALU, FP32)
//   z2 = W2 bf16(h1) + b2, h2 = relu(z2)               (MFMA bf16 -> FP32)
//   y  = w3 . h2 + b3;  p = JS_closed + y              (VALU, FP32)
// Training minimises mean (p - label)^2; the backward pass forms
// dW2 = dz2^T bf16(h1) and dh1 = dz2 W2 on the MFMA units (dz2 rounded to
// BF16), everything else in FP32.
//
// Layout of v_mfma_f32_16x16x16_bf16 used throughout (one wave, lane l,
// j = 0..3): A[i = l%16][k = 4(l/16)+j], B[k = 4(l/16)+j][n = l%16],
// D[m = 4(l/16)+j][n = l%16].
//
// A wave works on tiles of 16 pairs. Weight gradients of a wave accumulate
// in registers across its tiles and are written once to the wave's slot of
// a partial-gradient buffer, which a second kernel sums in a fixed order, so
// gradients are deterministic.
#include "bs_common.h"

namespace bs {

void launch_lut(int32_t N, double* t64, float* t32, hipStream_t s);

namespace {

constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 320, OFF_B2 = 4416, OFF_W3 = 4480, OFF_B3 = 4544;
constexpr int NP = 4545;       // parameters
constexpr int NPL = NP + 1;    // partial slot: gradients then the loss sum
constexpr int kMlpWaves = 4;   // waves per block
constexpr int kMaxWaves = 1024;

typedef short bf16x4 __attribute__((__vector_size__(4 * sizeof(short))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ __forceinline__ uint16_t to_bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MlpArgs {
  const uint16_t* __restrict__ w;  // BF16 parameters [NP]
  const float* __restrict__ t32;   // T(0..N)
  const int32_t* __restrict__ xa;
  const int32_t* __restrict__ xb;
  const int32_t* __restrict__ xab;
  const float* __restrict__ label;  // training only
  float* __restrict__ out;          // inference: [n]
  float* __restrict__ partial;      // training: [waves][NPL]
  int64_t n;
  int32_t N;
  float inv_n;  // 1/n (training)
};

struct WaveLds {
  float F[16][4];
  float base[16];
  float label[16];
  float z1[16][H];
  uint16_t h1b[16][H];
  uint16_t g2b[16][H];
};

template <bool TRAIN>
__global__ __launch_bounds__(kMlpWaves * kWave) void mlp_tile_kernel(MlpArgs a) {
  __shared__ WaveLds lds_all[kMlpWaves];
  __shared__ float w1s[H * 4 + H];  // W1 then b1, FP32
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  WaveLds& L = lds_all[wid];
  const int lr = lane % 16, lg = lane / 16;  // lane's position in the MFMA layouts
  for (int i = threadIdx.x; i < H * 4 + H; i += blockDim.x) w1s[i] = from_bf16(a.w[OFF_W1 + i]);

  // constant weight fragments
  bf16x4 bf[4][4];  // forward B = W2^T: [s = input block][t = output block]
  bf16x4 bb[4][4];  // backward B = W2:  [kk = output block][s = input block]
  float b2v[4], w3v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bf[s][t][j] = (short)a.w[OFF_W2 + (16 * t + lr) * H + 16 * s + 4 * lg + j];
        bb[t][s][j] = (short)a.w[OFF_W2 + (16 * t + 4 * lg + j) * H + 16 * s + lr];
      }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    b2v[t] = from_bf16(a.w[OFF_B2 + 16 * t + lr]);
    w3v[t] = from_bf16(a.w[OFF_W3 + 16 * t + lr]);
  }
  const float b3 = from_bf16(a.w[OFF_B3]);
  const float fN = (float)a.N;
  const float f3 = log2f(fN) * 0.0625f;
  __syncthreads();

  // gradient accumulators (training)
  f32x4 gW2[4][4];
  float gW1[4][4], gb1[4], gb2[4], gw3[4], gb3 = 0.0f, lsum = 0.0f;
  if (TRAIN) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      gb1[p] = gb2[p] = gw3[p] = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gW2[p][q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        gW1[p][q] = 0.0f;
      }
    }
  }

  const int64_t n_tiles = (a.n + 15) / 16;
  const int64_t wave_id = (int64_t)blockIdx.x * kMlpWaves + wid;
  const int64_t n_waves = (int64_t)gridDim.x * kMlpWaves;
  for (int64_t tile = wave_id; tile < n_tiles; tile += n_waves) {
    // 1. features, closed-form baseline, labels (lanes 0..15, one pair each)
    if (lane < 16) {
      const int64_t i = tile * 16 + lane;
      float f[4] = {0.0f, 0.0f, 0.0f, f3}, base = 0.0f, lab = 0.0f;
      if (i < a.n) {
        const int32_t N = a.N;
        int32_t xa = a.xa[i], xb = a.xb[i], xab = a.xab[i];
        xa = xa < 0 ? 0 : (xa > N ? N : xa);
        xb = xb < 0 ? 0 : (xb > N ? N : xb);
        xab = xab < 0 ? 0 : (xab > (xa < xb ? xa : xb) ? (xa < xb ? xa : xb) : xab);
        int32_t xu = xa + xb - xab;
        xu = xu > N ? N : xu;
        f[0] = (float)xa / fN;
        f[1] = (float)xb / fN;
        f[2] = (float)xab / fN;
        base = score_f32<BS_JACCARD>(a.t32[xa], a.t32[xb], a.t32[xu]);
        if (TRAIN) lab = a.label[i];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) L.F[lane][c] = f[c];
      L.base[lane] = base;
      L.label[lane] = lab;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // 2. layer 1 for row lr, units 16s + 4lg + j: straight into A fragments
    bf16x4 a1[4];
    {
      const float f0 = L.F[lr][0], f1 = L.F[lr][1], f2 = L.F[lr][2], f3v = L.F[lr][3];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 16 * s + 4 * lg + j;
          float z = w1s[H * 4 + u];
          z = fmaf(w1s[u * 4 + 0], f0, z);
          z = fmaf(w1s[u * 4 + 1], f1, z);
          z = fmaf(w1s[u * 4 + 2], f2, z);
          z = fmaf(w1s[u * 4 + 3], f3v, z);
          const uint16_t hb = to_bf16(z > 0.0f ? z : 0.0f);
          a1[s][j] = (short)hb;
          if (TRAIN) {
            L.z1[lr][u] = z;
            L.h1b[lr][u] = hb;
          }
        }
    }
    // 3. layer 2 on the matrix cores: z2[m][n] for rows 4lg+j, columns 16t+lr
    f32x4 z2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma16(a1[s], bf[s][t], acc);
      z2[t] = acc;
    }
    // 4. layer 3: y[row] summed over the 16 lanes that share the rows
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float z = z2[t][j] + b2v[t];
        z2[t][j] = z;
        part[j] = fmaf(w3v[t], z > 0.0f ? z : 0.0f, part[j]);
      }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) part[j] += __shfl_xor(part[j], off);
    float p[4], gy[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * lg + j;
      p[j] = L.base[row] + (part[j] + b3);
    }
    if (!TRAIN) {
      if (lr == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t i = tile * 16 + 4 * lg + j;
          if (i < a.n) a.out[i] = fminf(fmaxf(p[j], 0.0f), 1.0f);
        }
      }
      continue;
    }

    // 5. loss and dL/dy
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * lg + j;
      const bool ok = tile * 16 + row < a.n;
      const float r = ok ? p[j] - L.label[row] : 0.0f;
      gy[j] = 2.0f * r * a.inv_n;
      if (lr == 0) {
        lsum = fmaf(r, r, lsum);
        gb3 += gy[j];
      }
    }
    // 6. output layer and dz2 (D layout: rows 4lg+j, columns 16t+lr)
    f32x4 g2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float z = z2[t][j];
        const float h2 = z > 0.0f ? z : 0.0f;
        gw3[t] = fmaf(gy[j], h2, gw3[t]);
        const float g = z > 0.0f ? gy[j] * w3v[t] : 0.0f;
        g2[t][j] = g;
        gb2[t] += g;
        L.g2b[4 * lg + j][16 * t + lr] = to_bf16(g);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 7. dW2 += dz2^T bf16(h1): A = dz2^T (its D layout is the A layout), B = h1 rows
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bf16x4 ag;
#pragma unroll
      for (int j = 0; j < 4; ++j) ag[j] = (short)to_bf16(g2[t][j]);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bf16x4 bh;
#pragma unroll
        for (int j = 0; j < 4; ++j) bh[j] = (short)L.h1b[4 * lg + j][16 * s + lr];
        gW2[t][s] = mfma16(ag, bh, gW2[t][s]);
      }
    }
    // 8. dh1 = dz2 W2 (A = bf16(dz2) rows from LDS), then dz1 = dh1 * (z1 > 0)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        bf16x4 ag;
#pragma unroll
        for (int j = 0; j < 4; ++j) ag[j] = (short)L.g2b[lr][16 * kk + 4 * lg + j];
        acc = mfma16(ag, bb[kk][s], acc);
      }
      // acc: dh1 for rows 4lg+j, unit u = 16s+lr
      const int u = 16 * s + lr;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 4 * lg + j;
        const float g1 = L.z1[row][u] > 0.0f ? acc[j] : 0.0f;
        gb1[s] += g1;
#pragma unroll
        for (int c = 0; c < 4; ++c) gW1[s][c] = fmaf(g1, L.F[row][c], gW1[s][c]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (!TRAIN) return;

  // 9. this wave's partial gradients (every slot is written, zeros included)
  float* P = a.partial + (size_t)wave_id * NPL;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) P[OFF_W2 + (16 * t + 4 * lg + j) * H + 16 * s + lr] = gW2[t][s][j];
  // per-column sums are spread over the four lane groups: reduce across lg
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      gb1[q] += __shfl_xor(gb1[q], off);
      gb2[q] += __shfl_xor(gb2[q], off);
      gw3[q] += __shfl_xor(gw3[q], off);
#pragma unroll
      for (int c = 0; c < 4; ++c) gW1[q][c] += __shfl_xor(gW1[q][c], off);
    }
  }
  if (lg == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = 16 * q + lr;
      P[OFF_B1 + u] = gb1[q];
      P[OFF_B2 + u] = gb2[q];
      P[OFF_W3 + u] = gw3[q];
#pragma unroll
      for (int c = 0; c < 4; ++c) P[OFF_W1 + u * 4 + c] = gW1[q][c];
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    gb3 += __shfl_xor(gb3, off);
    lsum += __shfl_xor(lsum, off);
  }
  if (lane == 0) {
    P[OFF_B3] = gb3;
    P[NP] = lsum;
  }
}

// grad[p] = sum over waves of partial[w][p], in wave order (deterministic).
__global__ void mlp_reduce_kernel(const float* __restrict__ partial, int32_t n_waves, float* __restrict__ grad,
                                  float* __restrict__ loss, float inv_n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPL) return;
  float s = 0.0f;
  for (int w = 0; w < n_waves; ++w) s += partial[(size_t)w * NPL + p];
  if (p < NP) grad[p] = s;
  else if (loss) *loss = s * inv_n;
}

// Adam on the FP32 master weights, then the BF16 copy.
__global__ void mlp_adam_kernel(float* __restrict__ theta, uint16_t* __restrict__ wb, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ grad, float lr, float beta1,
                                float omb1, float beta2, float omb2, float eps, float c1, float c2) {
  // omb1 = 1 - beta1 and omb2 = 1 - beta2 come rounded from double: formed in
  // FP32 from the rounded betas, 1 - beta2 would be off by 1.3e-5 relative
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = grad[p];
  const float mm = beta1 * m[p] + omb1 * g;
  const float vv = beta2 * v[p] + omb2 * g * g;
  m[p] = mm;
  v[p] = vv;
  const float th = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  theta[p] = th;
  wb[p] = to_bf16(th);
}

__global__ void mlp_to_bf16_kernel(const float* __restrict__ theta, uint16_t* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) wb[p] = to_bf16(theta[p]);
}

int64_t grid_waves(int64_t n) {
  int64_t tiles = (n + 15) / 16;
  int64_t w = tiles < kMaxWaves ? tiles : kMaxWaves;
  return w < 1 ? 1 : w;
}

size_t mlp_ws(int64_t n, int32_t N) {
  return align256((size_t)(N + 1) * 4) + align256((size_t)kMaxWaves * NPL * 4) + align256((size_t)NP * 4);
}

bs_status mlp_check(const uint16_t* w, const int32_t* xa, const int32_t* xb, const int32_t* xab, int64_t n,
                    int32_t N, void* ws, size_t ws_bytes) {
  if (n < 0 || !valid_width(N)) return BS_ERR_ARG;
  if (!w || ((!xa || !xb || !xab) && n > 0)) return BS_ERR_NULL;
  if (!ws || ws_bytes < mlp_ws(n, N) || (reinterpret_cast<uintptr_t>(ws) & 255)) return BS_ERR_WORKSPACE;
  return BS_OK;
}

// Launches the training tile kernel and the reduction into grad/loss.
bs_status mlp_grad_launch(const uint16_t* w, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                          const float* label, int64_t n, int32_t N, float* grad, float* loss, void* ws,
                          hipStream_t s) {
  char* p = static_cast<char*>(ws);
  float* t32 = reinterpret_cast<float*>(p);
  float* partial = reinterpret_cast<float*>(p + align256((size_t)(N + 1) * 4));
  launch_lut(N, nullptr, t32, s);
  MlpArgs a;
  a.w = w;
  a.t32 = t32;
  a.xa = xa;
  a.xb = xb;
  a.xab = xab;
  a.label = label;
  a.out = nullptr;
  a.partial = partial;
  a.n = n;
  a.N = N;
  a.inv_n = n > 0 ? 1.0f / (float)n : 0.0f;
  const int64_t waves = grid_waves(n);
  const int64_t blocks = (waves + kMlpWaves - 1) / kMlpWaves;
  {
    ScopedTiming timing("mlp_train_tiles", s);
    hipLaunchKernelGGL((mlp_tile_kernel<true>), dim3((unsigned)blocks), dim3(kMlpWaves * kWave), 0, s, a);
  }
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPL + 255) / 256), dim3(256), 0, s, partial,
                     (int32_t)(blocks * kMlpWaves), grad, loss, a.inv_n);
  return launch_status();
}

}  // namespace
}  // namespace bs

extern "C" int32_t bs_mlp_param_count(void) { return bs::NP; }

extern "C" size_t bs_mlp_workspace_size(int64_t n, int32_t N) {
  using namespace bs;
  if (n < 0 || !valid_width(N)) return 0;
  return mlp_ws(n, N);
}

extern "C" bs_status bs_mlp_forward(const uint16_t* w, const int32_t* xa, const int32_t* xb,
                                    const int32_t* xab, int64_t n, int32_t N, float* out, void* workspace,
                                    size_t workspace_bytes, void* stream) {
  using namespace bs;
  bs_status st = mlp_check(w, xa, xb, xab, n, N, workspace, workspace_bytes);
  if (st != BS_OK) return st;
  if (!out && n > 0) return BS_ERR_NULL;
  st = check_device();
  if (st != BS_OK) return st;
  if (n == 0) return BS_OK;
  hipStream_t s = as_stream(stream);
  float* t32 = static_cast<float*>(workspace);
  launch_lut(N, nullptr, t32, s);
  MlpArgs a = {};
  a.w = w;
  a.t32 = t32;
  a.xa = xa;
  a.xb = xb;
  a.xab = xab;
  a.out = out;
  a.n = n;
  a.N = N;
  const int64_t tiles = (n + 15) / 16;
  int64_t blocks = (tiles + kMlpWaves - 1) / kMlpWaves;
  if (blocks > 4096) blocks = 4096;
  ScopedTiming timing("mlp_forward", s);
  hipLaunchKernelGGL((mlp_tile_kernel<false>), dim3((unsigned)blocks), dim3(kMlpWaves * kWave), 0, s, a);
  return launch_status();
}

extern "C" bs_status bs_mlp_grad(const uint16_t* w, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                                 const float* label, int64_t n, int32_t N, float* grad, float* loss,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  using namespace bs;
  bs_status st = mlp_check(w, xa, xb, xab, n, N, workspace, workspace_bytes);
  if (st != BS_OK) return st;
  if (!grad || (!label && n > 0)) return BS_ERR_NULL;
  if (n < 1) return BS_ERR_ARG;
  st = check_device();
  if (st != BS_OK) return st;
  return mlp_grad_launch(w, xa, xb, xab, label, n, N, grad, loss, workspace, as_stream(stream));
}

extern "C" bs_status bs_mlp_train_step(float* master, uint16_t* w, float* adam_m, float* adam_v, int64_t step,
                                       float lr, const int32_t* xa, const int32_t* xb, const int32_t* xab,
                                       const float* label, int64_t n, int32_t N, float* loss, void* workspace,
                                       size_t workspace_bytes, void* stream) {
  using namespace bs;
  bs_status st = mlp_check(w, xa, xb, xab, n, N, workspace, workspace_bytes);
  if (st != BS_OK) return st;
  if (!master || !adam_m || !adam_v || (!label && n > 0)) return BS_ERR_NULL;
  if (n < 1 || step < 1 || !(lr > 0.0f)) return BS_ERR_ARG;
  st = check_device();
  if (st != BS_OK) return st;
  hipStream_t s = as_stream(stream);
  char* p = static_cast<char*>(workspace);
  float* grad = reinterpret_cast<float*>(p + align256((size_t)(N + 1) * 4) + align256((size_t)kMaxWaves * NPL * 4));
  st = mlp_grad_launch(w, xa, xb, xab, label, n, N, grad, loss, workspace, s);
  if (st != BS_OK) return st;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)step)));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, master, w, adam_m, adam_v, grad,
                     lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), 1e-8f, c1, c2);
  return launch_status();
}

extern "C" bs_status bs_mlp_to_bf16(const float* master, uint16_t* w, void* stream) {
  using namespace bs;
  if (!master || !w) return BS_ERR_NULL;
  bs_status st = check_device();
  if (st != BS_OK) return st;
  hipLaunchKernelGGL(mlp_to_bf16_kernel, dim3((NP + 255) / 256), dim3(256), 0, as_stream(stream), master, w);
  return launch_status();
}
