// Learned cardinality estimator: a two-hidden-layer (64, 64) network that maps
// a host's per-array column popcounts to ln(1 + cardinality), as a learned
// correction of the Thm. 2 linear count. Weights are bfloat16, accumulation
// fp32; training is mean-squared error with Adam on an fp32 master copy.
//
// Block-level structure: a block takes tiles of 64 samples; each of its four
// waves computes a quarter of every hidden layer for the tile (lane = sample),
// activations live in LDS, and the weight gradients are tile GEMMs
// (dz^T h) accumulated in registers of the thread that owns each weight, then
// added to the global gradient once per block.
//
// The second layer takes its input activations in bfloat16, like its
// weights: the 64 x 64 x 64 product of a tile is a dense bf16 contraction,
// which the inference kernel runs on the matrix cores (one 32 x 32 quadrant
// of the tile per wave, v_mfma_f32_32x32x8_bf16, fp32 accumulation); the
// training kernels compute the same layer on the vector units from the same
// bf16 activations.
#include <math.h>

#include "../../include/cbaa_mlp.h"
#include "cbaa_internal.hpp"

namespace cbaa {

namespace {

constexpr int kH = 64;        // hidden width
constexpr int kMaxF = 8;      // features
constexpr int kTile = 64;     // samples per tile
constexpr int kThreads = 256; // 4 waves
constexpr int kW2PerThread = kH * kH / kThreads;  // 16

struct Offsets {
  uint32_t W1, b1, W2, b2, w3, b3, P;
};

__host__ __device__ inline Offsets offsets(uint32_t F) {
  Offsets o;
  o.W1 = 0;
  o.b1 = kH * F;
  o.W2 = o.b1 + kH;
  o.b2 = o.W2 + kH * kH;
  o.w3 = o.b2 + kH;
  o.b3 = o.w3 + kH;
  o.P = o.b3 + 1;
  return o;
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest, ties to even (NaN kept quiet).
__device__ inline uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

struct Net {
  float W1[kH * kMaxF];
  float b1[kH];
  float W2[kH * kH];
  float b2[kH];
  float w3[kH];
  float b3;
};

// Weights from the bf16 copy, biases from the fp32 master.
__device__ inline void load_net(Net& n, uint32_t F, const float* master, const uint16_t* wbf) {
  const Offsets o = offsets(F);
  for (uint32_t i = threadIdx.x; i < kH * F; i += kThreads) n.W1[i] = bf16_to_f32(wbf[o.W1 + i]);
  for (uint32_t i = threadIdx.x; i < kH * kH; i += kThreads) n.W2[i] = bf16_to_f32(wbf[o.W2 + i]);
  for (uint32_t i = threadIdx.x; i < kH; i += kThreads) {
    n.b1[i] = master[o.b1 + i];
    n.b2[i] = master[o.b2 + i];
    n.w3[i] = bf16_to_f32(wbf[o.w3 + i]);
  }
  if (threadIdx.x == 0) n.b3 = master[o.b3];
}

struct Tile {
  float x[kTile][kMaxF];
  float a[kTile][kH + 1];   // h1, later dz1 (padded row against bank conflicts)
  float b[kTile][kH + 1];   // h2, later dz2
  float ypart[4][kTile];
  float dy[kTile];
};

// Forward for one tile: fills t.a = h1, t.b = h2 and returns y of the lane's
// sample to wave 0 lanes (all lanes of all waves get y in ypart sums).
__device__ inline void tile_forward(const Net& n, Tile& t, uint32_t F, const float* x, uint64_t s0,
                                    uint64_t ns) {
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t q = threadIdx.x / kWave;  // wave: a quarter of the hidden units
  for (uint32_t i = threadIdx.x; i < kTile * F; i += kThreads) {
    const uint32_t s = i / F, f = i % F;
    t.x[s][f] = s0 + s < ns ? x[(s0 + s) * F + f] : 0.0f;
  }
  __syncthreads();
  float xs[kMaxF];
#pragma unroll
  for (int f = 0; f < kMaxF; ++f) xs[f] = f < (int)F ? t.x[lane][f] : 0.0f;
#pragma unroll 4
  for (int jj = 0; jj < kH / 4; ++jj) {
    const int j = q * (kH / 4) + jj;
    float z = n.b1[j];
#pragma unroll
    for (int f = 0; f < kMaxF; ++f)
      if (f < (int)F) z += n.W1[j * F + f] * xs[f];
    // layer 2 reads h1 in bf16
    t.a[lane][j] = bf16_to_f32(f32_to_bf16(z > 0.0f ? z : 0.0f));
  }
  __syncthreads();
  float part = 0.0f;
  for (int kk = 0; kk < kH / 4; ++kk) {
    const int k = q * (kH / 4) + kk;
    float z = n.b2[k];
#pragma unroll 16
    for (int j = 0; j < kH; ++j) z += n.W2[k * kH + j] * t.a[lane][j];
    const float h = z > 0.0f ? z : 0.0f;
    t.b[lane][k] = h;
    part += n.w3[k] * h;
  }
  t.ypart[q][lane] = part;
  __syncthreads();
}

__device__ inline float tile_y(const Net& n, const Tile& t, uint32_t s) {
  return ((t.ypart[0][s] + t.ypart[1][s]) + (t.ypart[2][s] + t.ypart[3][s])) + n.b3;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Inference with the second layer on the matrix cores. Per tile of 64
// samples: layer 1 on the vector units (lane = sample, a quarter of the units
// per wave), h1 stored in bf16; wave w computes the quadrant of z2 with
// samples 32 (w / 2) .. and units 32 (w % 2) .. as eight 32 x 32 x 8 MFMAs
// over the 64 inputs (A: h1 rows, B: W2 rows, both 4 consecutive bf16 per
// lane); z2 + b2, relu, and the output layer's partial sums per quarter.
__global__ __launch_bounds__(kThreads) void k_mlp_forward_mfma(uint32_t F, const float* master,
                                                               const uint16_t* wbf,
                                                               const float* x, uint64_t ns,
                                                               float* y) {
  __shared__ float W1[kH * kMaxF];
  __shared__ float b1[kH], b2[kH], w3[kH];
  __shared__ float b3;
  __shared__ __align__(8) uint16_t W2[kH][kH + 4];   // bf16 rows (unit, input), padded
  __shared__ __align__(8) uint16_t h1[kTile][kH + 4]; // bf16 (sample, unit), padded
  __shared__ float xs[kTile][kMaxF];
  __shared__ float h2[kTile][kH + 1];
  __shared__ float ypart[4][kTile];
  const Offsets o = offsets(F);
  for (uint32_t i = threadIdx.x; i < kH * F; i += kThreads) W1[i] = bf16_to_f32(wbf[o.W1 + i]);
  for (uint32_t i = threadIdx.x; i < kH * kH; i += kThreads) W2[i / kH][i % kH] = wbf[o.W2 + i];
  for (uint32_t i = threadIdx.x; i < kH; i += kThreads) {
    b1[i] = master[o.b1 + i];
    b2[i] = master[o.b2 + i];
    w3[i] = bf16_to_f32(wbf[o.w3 + i]);
  }
  if (threadIdx.x == 0) b3 = master[o.b3];
  __syncthreads();
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t q = threadIdx.x / kWave;
  const uint32_t mi = q >> 1, ni = q & 1;          // this wave's quadrant
  const uint32_t r = lane % 32, kq = (lane / 32) * 4;
  for (uint64_t s0 = (uint64_t)blockIdx.x * kTile; s0 < ns; s0 += (uint64_t)gridDim.x * kTile) {
    for (uint32_t i = threadIdx.x; i < kTile * F; i += kThreads) {
      const uint32_t s = i / F, f = i % F;
      xs[s][f] = s0 + s < ns ? x[(s0 + s) * F + f] : 0.0f;
    }
    __syncthreads();
    // layer 1, in the same operation order as the training kernels
    for (int jj = 0; jj < kH / 4; ++jj) {
      const int j = q * (kH / 4) + jj;
      float z = b1[j];
      for (int f = 0; f < (int)F; ++f) z += W1[j * F + f] * xs[lane][f];
      h1[lane][j] = f32_to_bf16(z > 0.0f ? z : 0.0f);
    }
    __syncthreads();
    // layer 2 on the matrix cores
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < kH / 8; ++kb) {
      const uint32_t k = kb * 8 + kq;
      const bf16x4 a = *(const bf16x4*)&h1[mi * 32 + r][k];
      const bf16x4 bv = *(const bf16x4*)&W2[ni * 32 + r][k];
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, bv, acc, 0, 0, 0);
    }
    // lane holds z2[sample][unit] for unit ni*32 + r and samples
    // mi*32 + (v % 4) + 4 (lane / 32) + 8 (v / 4), v < 16
    const uint32_t unit = ni * 32 + r;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t s = mi * 32 + (v % 4) + kq + 8 * (v / 4);
      const float z = acc[v] + b2[unit];
      h2[s][unit] = z > 0.0f ? z : 0.0f;
    }
    __syncthreads();
    float part = 0.0f;
    for (int kk = 0; kk < kH / 4; ++kk) {
      const int k = q * (kH / 4) + kk;
      part += w3[k] * h2[lane][k];
    }
    ypart[q][lane] = part;
    __syncthreads();
    if (threadIdx.x < kTile && s0 + threadIdx.x < ns)
      y[s0 + threadIdx.x] = ((ypart[0][threadIdx.x] + ypart[1][threadIdx.x]) +
                             (ypart[2][threadIdx.x] + ypart[3][threadIdx.x])) + b3;
    __syncthreads();
  }
}

// Gradient of mean (y - t)^2 / 2 over ns samples (the batch), added into grad
// (zeroed by the caller), and the loss added into *loss.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(uint32_t F, const float* master,
                                                       const uint16_t* wbf, const float* x,
                                                       const float* target, uint64_t ns,
                                                       float* grad, float* loss) {
  __shared__ Net n;
  __shared__ Tile t;
  __shared__ float lsum[kThreads / kWave];
  load_net(n, F, master, wbf);
  __syncthreads();
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t q = threadIdx.x / kWave;
  const float inv_n = 1.0f / (float)ns;
  // owned accumulators: dW2 entries (k, j) = (threadIdx.x / 4, (threadIdx.x % 4) * 16 + u)
  float gW2[kW2PerThread];
#pragma unroll
  for (int u = 0; u < kW2PerThread; ++u) gW2[u] = 0.0f;
  const uint32_t k_own = threadIdx.x / 4, j_base = (threadIdx.x % 4) * 16;
  // dW1 entries: e = threadIdx.x and threadIdx.x + 256 over kH * F
  float gW1[2] = {0.0f, 0.0f};
  // vectors: thread < 64 owns b1[j], thread in [64,128) b2, [128,192) w3; 192 owns b3
  float gvec = 0.0f;
  float lacc = 0.0f;
  for (uint64_t s0 = (uint64_t)blockIdx.x * kTile; s0 < ns; s0 += (uint64_t)gridDim.x * kTile) {
    tile_forward(n, t, F, x, s0, ns);
    if (threadIdx.x < kTile) {
      const uint32_t s = threadIdx.x;
      float dy = 0.0f;
      if (s0 + s < ns) {
        const float r = tile_y(n, t, s) - target[s0 + s];
        lacc += 0.5f * r * r;
        dy = r * inv_n;
      }
      t.dy[s] = dy;
    }
    __syncthreads();
    // dw3[k] = sum_s dy_s h2[s][k]; db3 = sum_s dy_s
    if (threadIdx.x >= 128 && threadIdx.x < 192) {
      const uint32_t k = threadIdx.x - 128;
      float acc = 0.0f;
      for (int s = 0; s < kTile; ++s) acc += t.dy[s] * t.b[s][k];
      gvec += acc;
    } else if (threadIdx.x == 192) {
      float acc = 0.0f;
      for (int s = 0; s < kTile; ++s) acc += t.dy[s];
      gvec += acc;
    }
    __syncthreads();
    // dz2 = dy * w3 * [h2 > 0], in place of h2
    for (int kk = 0; kk < kH / 4; ++kk) {
      const int k = q * (kH / 4) + kk;
      t.b[lane][k] = t.b[lane][k] > 0.0f ? t.dy[lane] * n.w3[k] : 0.0f;
    }
    __syncthreads();
    // dW2[k][j] += sum_s dz2[s][k] h1[s][j]; db2[k] += sum_s dz2[s][k]
    for (int s = 0; s < kTile; ++s) {
      const float dz = t.b[s][k_own];
#pragma unroll
      for (int u = 0; u < kW2PerThread; ++u) gW2[u] += dz * t.a[s][j_base + u];
    }
    if (threadIdx.x >= 64 && threadIdx.x < 128) {
      const uint32_t k = threadIdx.x - 64;
      float acc = 0.0f;
      for (int s = 0; s < kTile; ++s) acc += t.b[s][k];
      gvec += acc;
    }
    __syncthreads();
    // dz1[s][j] = (sum_k W2[k][j] dz2[s][k]) * [h1 > 0], in place of h1
    float dz1[kH / 4];
#pragma unroll
    for (int jj = 0; jj < kH / 4; ++jj) {
      const int j = q * (kH / 4) + jj;
      float acc = 0.0f;
#pragma unroll 16
      for (int k = 0; k < kH; ++k) acc += n.W2[k * kH + j] * t.b[lane][k];
      dz1[jj] = t.a[lane][j] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kH / 4; ++jj) t.a[lane][q * (kH / 4) + jj] = dz1[jj];
    __syncthreads();
    // dW1[j][f] += sum_s dz1[s][j] x[s][f]; db1[j] += sum_s dz1[s][j]
#pragma unroll
    for (int e2 = 0; e2 < 2; ++e2) {
      const uint32_t e = threadIdx.x + e2 * kThreads;
      if (e < kH * F) {
        const uint32_t j = e / F, f = e % F;
        float acc = 0.0f;
        for (int s = 0; s < kTile; ++s) acc += t.a[s][j] * t.x[s][f];
        gW1[e2] += acc;
      }
    }
    if (threadIdx.x < 64) {
      float acc = 0.0f;
      for (int s = 0; s < kTile; ++s) acc += t.a[s][threadIdx.x];
      gvec += acc;
    }
    __syncthreads();
  }
  const Offsets o = offsets(F);
#pragma unroll
  for (int u = 0; u < kW2PerThread; ++u) atomicAdd(&grad[o.W2 + k_own * kH + j_base + u], gW2[u]);
#pragma unroll
  for (int e2 = 0; e2 < 2; ++e2) {
    const uint32_t e = threadIdx.x + e2 * kThreads;
    if (e < kH * F) atomicAdd(&grad[o.W1 + e], gW1[e2]);
  }
  if (threadIdx.x < 64) atomicAdd(&grad[o.b1 + threadIdx.x], gvec);
  else if (threadIdx.x < 128) atomicAdd(&grad[o.b2 + threadIdx.x - 64], gvec);
  else if (threadIdx.x < 192) atomicAdd(&grad[o.w3 + threadIdx.x - 128], gvec);
  else if (threadIdx.x == 192) atomicAdd(&grad[o.b3], gvec);
  // loss
  float l = lacc;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, kWave);
  if (lane == 0) lsum[q] = l;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, ((lsum[0] + lsum[1]) + (lsum[2] + lsum[3])) * inv_n);
}

__global__ void k_zero_f32(float* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// Adam on the fp32 master copy, then refresh the bf16 weights.
__global__ void k_mlp_adam(uint32_t P, float* master, uint16_t* wbf, const float* grad, float* m,
                           float* v, float lr, float beta1, float beta2, float eps, float c1,
                           float c2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * g;
  const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1;
  const float vh = vi / c2;
  const float w = master[i] - lr * mh / (sqrtf(vh) + eps);
  master[i] = w;
  wbf[i] = f32_to_bf16(w);
}

// He-uniform weights from a counter-based hash of (seed, index); zero biases;
// optionally a zero output layer (the network then outputs exactly 0).
__global__ void k_mlp_init(uint32_t F, uint32_t seed, int zero_output, float* master,
                           uint16_t* wbf) {
  const Offsets o = offsets(F);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= o.P) return;
  float w = 0.0f;
  float fan_in = 0.0f;
  if (i < o.b1) fan_in = (float)F;
  else if (i >= o.W2 && i < o.b2) fan_in = (float)kH;
  else if (i >= o.w3 && i < o.b3 && !zero_output) fan_in = (float)kH;
  if (fan_in > 0.0f) {
    const uint32_t h = lowbias32(fmix32(seed) ^ (i * 0x9E3779B9u));
    const float u = (float)(h >> 8) * (1.0f / 16777216.0f);  // [0, 1)
    w = (2.0f * u - 1.0f) * sqrtf(6.0f / fan_in);
  }
  master[i] = w;
  wbf[i] = f32_to_bf16(w);
}

int check(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, what);
}

uint32_t grid_tiles(uint64_t ns) {
  uint64_t t = (ns + kTile - 1) / kTile;
  if (t > 1024) t = 1024;
  return t == 0 ? 1u : (uint32_t)t;
}

}  // namespace

}  // namespace cbaa

using namespace cbaa;

extern "C" {

uint32_t cbaa_mlp_param_count(uint32_t n_features) {
  if (n_features < 1 || n_features > kMaxF) return 0;
  return offsets(n_features).P;
}

int cbaa_mlp_init(uint32_t F, uint32_t seed, int zero_output, float* d_master, uint16_t* d_wbf,
                  void* stream) {
  if (F < 1 || F > kMaxF || !d_master || !d_wbf) {
    set_error("bad feature count or null buffer");
    return CBAA_EINVAL;
  }
  const uint32_t P = offsets(F).P;
  hipLaunchKernelGGL(k_mlp_init, dim3((P + 255) / 256), dim3(256), 0, (hipStream_t)stream, F, seed,
                     zero_output, d_master, d_wbf);
  return check("mlp init launch");
}

int cbaa_mlp_forward(uint32_t F, const float* d_master, const uint16_t* d_wbf, const float* d_x,
                     uint64_t n, float* d_y, void* stream) {
  if (F < 1 || F > kMaxF || !d_master || !d_wbf) {
    set_error("bad feature count or null buffer");
    return CBAA_EINVAL;
  }
  if (n == 0) return CBAA_OK;
  if (!d_x || !d_y) {
    set_error("null input or output");
    return CBAA_EINVAL;
  }
  hipLaunchKernelGGL(k_mlp_forward_mfma, dim3(grid_tiles(n)), dim3(kThreads), 0,
                     (hipStream_t)stream, F, d_master, d_wbf, d_x, n, d_y);
  return check("mlp forward launch");
}

int cbaa_mlp_loss_grad(uint32_t F, const float* d_master, const uint16_t* d_wbf, const float* d_x,
                       const float* d_t, uint64_t n, float* d_grad, float* d_loss, void* stream) {
  if (F < 1 || F > kMaxF || !d_master || !d_wbf || !d_grad || !d_loss || n == 0 || !d_x || !d_t) {
    set_error("bad feature count, empty batch or null buffer");
    return CBAA_EINVAL;
  }
  const uint32_t P = offsets(F).P;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f32, dim3((P + 255) / 256), dim3(256), 0, s, d_grad, P);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, d_loss, 1u);
  int rc = check("mlp zero launch");
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid_tiles(n)), dim3(kThreads), 0, s, F, d_master, d_wbf, d_x,
                     d_t, n, d_grad, d_loss);
  return check("mlp grad launch");
}

int cbaa_mlp_adam(uint32_t F, float* d_master, uint16_t* d_wbf, const float* d_grad, float* d_m,
                  float* d_v, uint32_t step, float lr, float beta1, float beta2, float eps,
                  void* stream) {
  if (F < 1 || F > kMaxF || !d_master || !d_wbf || !d_grad || !d_m || !d_v || step == 0) {
    set_error("bad feature count, step or null buffer");
    return CBAA_EINVAL;
  }
  const uint32_t P = offsets(F).P;
  const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((P + 255) / 256), dim3(256), 0, (hipStream_t)stream, P,
                     d_master, d_wbf, d_grad, d_m, d_v, lr, beta1, beta2, eps, c1, c2);
  return check("mlp adam launch");
}

}  // extern "C"
