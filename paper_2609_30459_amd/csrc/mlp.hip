// Learned-initialisation MLP on gfx950 BF16 MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): forward, loss, backward and Adam, plus the C ABI of
// vio_mlp.h.
//
// MFMA operand layout (16x16x32): lane l holds A[l%16][8(l/16) .. +7] (a row
// segment of 8 bf16), B[8(l/16) .. +7][l%16] (a column segment) and returns
// D[4(l/16) + q][l%16], q = 0..3.
//
// Forward: one wave per 16 rows. Layer 1 is one MFMA per 16 hidden units
// (K = 32 is one step); the ReLU'd bf16 activations go through the wave's LDS
// to become the next layer's A operand. Backward: a data pass (dH2 = dY W3,
// dH1 = dH2 W2, masked by the ReLUs) writes the bf16 operands transposed, and
// the weight gradients are MFMA tiles reduced over the batch
// (dW = dH^T H_prev); bias gradients are the same product against a ones
// operand. Every sum has a fixed order: no atomics, deterministic results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fe_common.h"
#include "mfma_ops.h"
#include "vio_mlp.h"

namespace vio {

constexpr int kMlpWaves = 4;

__device__ __forceinline__ bool relu_active(uint16_t h) { return h != 0 && !(h & 0x8000u); }

// Training scratch, transposed bf16 operands with leading dimension ldt.
struct MlpScratch {
  int ldt;
  uint16_t *Xt, *H1t, *H2t, *dYt, *dH2t, *dH1t;  // [32|128|128|3|128|128][ldt]
  float* dY;                                     // [ldt][3]
  float* loss;                                   // [1]
};

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
template <bool kTrain>
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_fwd(MlpDev M, const float* __restrict__ X, int K, int Kpad,
                                                            float* __restrict__ Y, MlpScratch S) {
  __shared__ __align__(16) uint16_t sH[kMlpWaves][2][16][MH];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = ((int)blockIdx.x * kMlpWaves + wv) * 16;
  if (i0 >= Kpad) return;
  const int r = lane & 15, g = lane >> 4;
  uint16_t (*h1)[MH] = sH[wv][0];
  uint16_t (*h2)[MH] = sH[wv][1];
  // A operand of layer 1: row i0 + r, features 8g .. 8g+7
  uint16_t xv[8];
  {
    const int i = i0 + r;
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[e] = i < K ? bf16_bits(X[(size_t)i * MI + 8 * g + e]) : (uint16_t)0;
    if (kTrain) {
#pragma unroll
      for (int e = 0; e < 8; ++e) S.Xt[(size_t)(8 * g + e) * S.ldt + i] = xv[e];
    }
  }
  const bf16x8 a = pack8(xv);
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // layer 1: 8 tiles of 16 hidden units
#pragma unroll
  for (int jt = 0; jt < MH / 16; ++jt) {
    const int j = 16 * jt + r;
    const f32x4 acc = mfma(a, load8(M.W1b + (size_t)j * MI + 8 * g), zero);
    const float b = M.P[OFF_B1 + j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      h1[row][j] = (i0 + row) < K ? bf16_bits(fmaxf(acc[q] + b, 0.f)) : (uint16_t)0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // layer 2: K = 128 in four MFMA steps
#pragma unroll
  for (int jt = 0; jt < MH / 16; ++jt) {
    const int j = 16 * jt + r;
    f32x4 acc = zero;
#pragma unroll
    for (int kc = 0; kc < MH / 32; ++kc)
      acc = mfma(load8(&h1[r][32 * kc + 8 * g]), load8(M.W2b + (size_t)j * MH + 32 * kc + 8 * g), acc);
    const float b = M.P[OFF_B2 + j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      h2[row][j] = (i0 + row) < K ? bf16_bits(fmaxf(acc[q] + b, 0.f)) : (uint16_t)0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // layer 3: 3 outputs padded to a 16-column tile
  f32x4 acc = zero;
  const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int kc = 0; kc < MH / 32; ++kc) {
    const bf16x8 b = r < MO ? load8(M.W3b + (size_t)r * MH + 32 * kc + 8 * g) : pack8(z8);
    acc = mfma(load8(&h2[r][32 * kc + 8 * g]), b, acc);
  }
  if (r < MO) {
    const float b = M.P[OFF_B3 + r];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 4 * g + q;
      if (i < K) Y[(size_t)i * MO + r] = acc[q] + b;
    }
  }
  if (kTrain) {
    for (int idx = lane; idx < 16 * MH; idx += 64) {
      const int row = idx & 15, j = idx >> 4;
      S.H1t[(size_t)j * S.ldt + i0 + row] = h1[row][j];
      S.H2t[(size_t)j * S.ldt + i0 + row] = h2[row][j];
    }
  }
}

// ---------------------------------------------------------------------------
// inference forward: the same MFMA sequence as k_mlp_fwd (so the same
// results). The bf16 weights and the biases (42 KB, L2-resident) are read
// straight from global memory as MFMA operands, so a workgroup holds only its
// waves' 4 KB activation tiles in LDS and fits beside the pyramid kernel's
// workgroups when both run at once; layer 2's eight output tiles stay in
// registers so its output reuses the wave's layer-1 tile.
// ---------------------------------------------------------------------------
constexpr int kInferWaves = 4;
__global__ __launch_bounds__(64 * kInferWaves) void k_mlp_infer(MlpDev M, const float* __restrict__ X, int K,
                                                               int Kpad, float* __restrict__ Y) {
  __shared__ __align__(16) uint16_t sH[kInferWaves][16][MH];
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int i0 = ((int)blockIdx.x * kInferWaves + wv) * 16;
  if (i0 >= Kpad) return;  // no barrier follows
  const int r = lane & 15, g = lane >> 4;
  uint16_t (*h)[MH] = sH[wv];
  uint16_t xv[8];
  {
    const int i = i0 + r;
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[e] = i < K ? bf16_bits(X[(size_t)i * MI + 8 * g + e]) : (uint16_t)0;
  }
  const bf16x8 a = pack8(xv);
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // layer 1
#pragma unroll
  for (int jt = 0; jt < MH / 16; ++jt) {
    const int j = 16 * jt + r;
    const f32x4 acc = mfma(a, load8(&M.W1b[j * MI + 8 * g]), zero);
    const float b = M.P[OFF_B1 + j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      h[row][j] = (i0 + row) < K ? bf16_bits(fmaxf(acc[q] + b, 0.f)) : (uint16_t)0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // layer 2: all eight output tiles in registers, then written over h1
  f32x4 acc2[MH / 16];
#pragma unroll
  for (int jt = 0; jt < MH / 16; ++jt) {
    const int j = 16 * jt + r;
    f32x4 acc = zero;
#pragma unroll
    for (int kc = 0; kc < MH / 32; ++kc)
      acc = mfma(load8(&h[r][32 * kc + 8 * g]), load8(&M.W2b[j * MH + 32 * kc + 8 * g]), acc);
    acc2[jt] = acc;
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int jt = 0; jt < MH / 16; ++jt) {
    const int j = 16 * jt + r;
    const float b = M.P[OFF_B2 + j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      h[row][j] = (i0 + row) < K ? bf16_bits(fmaxf(acc2[jt][q] + b, 0.f)) : (uint16_t)0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // layer 3: 3 outputs padded to a 16-column tile (zero weight rows)
  f32x4 acc = zero;
#pragma unroll
  for (int kc = 0; kc < MH / 32; ++kc) {
    // output columns 3..15 are zero weight rows
    const bf16x8 w = r < MO ? load8(&M.W3b[r * MH + 32 * kc + 8 * g]) : __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
    acc = mfma(load8(&h[r][32 * kc + 8 * g]), w, acc);
  }
  if (r < MO) {
    const float b = M.P[OFF_B3 + r];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + 4 * g + q;
      if (i < K) Y[(size_t)i * MO + r] = acc[q] + b;
    }
  }
}

// ---------------------------------------------------------------------------
// loss: Huber (1 px) on (16 y0, 16 y1) - target plus BCE of y2 against
// [|guess - target| <= 2 px]; mean over the batch. One workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ T, int K,
                                                   int Kpad, MlpScratch S) {
  __shared__ float red[1024];
  float part = 0.f;
  const float inv = 1.f / (float)K;
  for (int i = threadIdx.x; i < Kpad; i += 1024) {
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
    if (i < K) {
      const float gx = 16.f * Y[i * MO], gy = 16.f * Y[i * MO + 1], z = Y[i * MO + 2];
      const float ex = gx - T[2 * i], ey = gy - T[2 * i + 1];
      const float hx = fabsf(ex) <= 1.f ? 0.5f * ex * ex : fabsf(ex) - 0.5f;
      const float hy = fabsf(ey) <= 1.f ? 0.5f * ey * ey : fabsf(ey) - 0.5f;
      const float c = sqrtf(ex * ex + ey * ey) <= 2.f ? 1.f : 0.f;
      const float bce = (z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z))) - c * z;
      part += hx + hy + bce;
      d0 = 16.f * fmaxf(-1.f, fminf(1.f, ex)) * inv;
      d1 = 16.f * fmaxf(-1.f, fminf(1.f, ey)) * inv;
      d2 = (1.f / (1.f + expf(-z)) - c) * inv;
    }
    S.dY[i * MO] = d0;
    S.dY[i * MO + 1] = d1;
    S.dY[i * MO + 2] = d2;
    S.dYt[(size_t)0 * S.ldt + i] = bf16_bits(d0);
    S.dYt[(size_t)1 * S.ldt + i] = bf16_bits(d1);
    S.dYt[(size_t)2 * S.ldt + i] = bf16_bits(d2);
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *S.loss = red[0] * inv;
}

// ---------------------------------------------------------------------------
// backward, data pass: dH2 = (dY W3) * [h2 > 0], dH1 = (dH2 W2) * [h1 > 0]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_bwd_data(MlpDev M, int Kpad, MlpScratch S) {
  __shared__ __align__(16) uint16_t sD[kMlpWaves][16][MH];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = ((int)blockIdx.x * kMlpWaves + wv) * 16;
  if (i0 >= Kpad) return;
  const int r = lane & 15, g = lane >> 4;
  uint16_t (*d2)[MH] = sD[wv];
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  uint16_t av[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = 8 * g + e;
    av[e] = c < MO ? bf16_bits(S.dY[(size_t)(i0 + r) * MO + c]) : (uint16_t)0;
  }
  const bf16x8 a = pack8(av);
#pragma unroll
  for (int kt = 0; kt < MH / 16; ++kt) {
    const int k = 16 * kt + r;
    uint16_t bv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = 8 * g + e;
      bv[e] = c < MO ? M.W3b[(size_t)c * MH + k] : (uint16_t)0;
    }
    const f32x4 acc = mfma(a, pack8(bv), zero);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      const uint16_t d = relu_active(S.H2t[(size_t)k * S.ldt + i0 + row]) ? bf16_bits(acc[q]) : (uint16_t)0;
      d2[row][k] = d;
      S.dH2t[(size_t)k * S.ldt + i0 + row] = d;
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int kt = 0; kt < MH / 16; ++kt) {
    const int k = 16 * kt + r;
    f32x4 acc = zero;
#pragma unroll
    for (int jc = 0; jc < MH / 32; ++jc)
      acc = mfma(load8(&d2[r][32 * jc + 8 * g]), load8(M.W2tb + (size_t)k * MH + 32 * jc + 8 * g), acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 4 * g + q;
      S.dH1t[(size_t)k * S.ldt + i0 + row] =
          relu_active(S.H1t[(size_t)k * S.ldt + i0 + row]) ? bf16_bits(acc[q]) : (uint16_t)0;
    }
  }
}

// ---------------------------------------------------------------------------
// backward, weight gradients: one wave per 16x16 tile of dW (or of a bias,
// against a ones operand), reduced over the padded batch in steps of 32.
// ---------------------------------------------------------------------------
struct GradTile {
  int a_src, b_src;  // 0 Xt, 1 H1t, 2 H2t, 3 dYt, 4 dH2t, 5 dH1t, 6 ones
  int m0, n0;        // tile origin in the gradient matrix
  int rows, cols;    // valid extent of the matrix
  int off;           // parameter offset; bias tiles write column 0 only
  int bias;
};

__constant__ GradTile c_tiles[105];

__device__ __forceinline__ const uint16_t* src_of(const MlpScratch& S, int s) {
  switch (s) {
    case 0: return S.Xt;
    case 1: return S.H1t;
    case 2: return S.H2t;
    case 3: return S.dYt;
    case 4: return S.dH2t;
    default: return S.dH1t;
  }
}

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_wgrad(int n_tiles, int Kpad, MlpScratch S,
                                                              float* __restrict__ G) {
  const int lane = threadIdx.x & 63;
  const int t = (int)blockIdx.x * kMlpWaves + (int)(threadIdx.x >> 6);
  if (t >= n_tiles) return;
  const GradTile T = c_tiles[t];
  const int r = lane & 15, g = lane >> 4;
  const uint16_t* A = src_of(S, T.a_src);
  const uint16_t* B = T.b_src == 6 ? nullptr : src_of(S, T.b_src);
  const bool arow = T.m0 + r < T.rows;
  const bool bcol = T.b_src == 6 || T.n0 + r < T.cols;
  const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint16_t one8[8] = {0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80};
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < Kpad; i0 += 32) {
    const bf16x8 a = arow ? load8(A + (size_t)(T.m0 + r) * S.ldt + i0 + 8 * g) : pack8(z8);
    const bf16x8 b = T.b_src == 6 ? pack8(one8) : (bcol ? load8(B + (size_t)(T.n0 + r) * S.ldt + i0 + 8 * g) : pack8(z8));
    acc = mfma(a, b, acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = T.m0 + 4 * g + q, n = T.n0 + r;
    if (m >= T.rows) continue;
    if (T.bias) {
      if (r == 0) G[T.off + m] = acc[q];
    } else if (n < T.cols) {
      G[T.off + (size_t)m * T.cols + n] = acc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Adam on the master weights; refreshes the bf16 copies. t >= 1; step == 0
// only refreshes the copies.
// ---------------------------------------------------------------------------
__global__ void k_mlp_adam(MlpDev M, const float* __restrict__ G, int step, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= NP) return;
  float p = M.P[i];
  if (step > 0) {
    const float g = G[i];
    const float m = b1 * M.m[i] + (1.f - b1) * g;
    const float v = b2 * M.v[i] + (1.f - b2) * g * g;
    M.m[i] = m;
    M.v[i] = v;
    p -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    M.P[i] = p;
  }
  const uint16_t b = bf16_bits(p);
  if (i < OFF_B1) {
    M.W1b[i] = b;
  } else if (i >= OFF_W2 && i < OFF_B2) {
    const int j = (i - OFF_W2) / MH, k = (i - OFF_W2) % MH;
    M.W2b[j * MH + k] = b;
    M.W2tb[k * MH + j] = b;
  } else if (i >= OFF_W3 && i < OFF_B3) {
    M.W3b[i - OFF_W3] = b;
  }
}

std::vector<GradTile> grad_tiles() {
  std::vector<GradTile> t;
  // dW3 [3][128] = dY^T H2 and db3
  for (int n0 = 0; n0 < MH; n0 += 16) t.push_back({3, 2, 0, n0, MO, MH, OFF_W3, 0});
  t.push_back({3, 6, 0, 0, MO, 1, OFF_B3, 1});
  // dW2 [128][128] = dH2^T H1 and db2
  for (int m0 = 0; m0 < MH; m0 += 16) {
    for (int n0 = 0; n0 < MH; n0 += 16) t.push_back({4, 1, m0, n0, MH, MH, OFF_W2, 0});
    t.push_back({4, 6, m0, 0, MH, 1, OFF_B2, 1});
  }
  // dW1 [128][32] = dH1^T X and db1
  for (int m0 = 0; m0 < MH; m0 += 16) {
    for (int n0 = 0; n0 < MI; n0 += 16) t.push_back({5, 0, m0, n0, MH, MI, OFF_W1, 0});
    t.push_back({5, 6, m0, 0, MH, 1, OFF_B1, 1});
  }
  return t;
}

hipError_t mlp_pack_launch(const MlpDev& M, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, s, M, (const float*)nullptr, 0, 0.f, 0.f, 0.f,
                     0.f, 1.f, 1.f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Library-held training scratch of vio_mlp_gradient_noalloc: one array per
// GPU, held until the process ends, for batches of up to
// VIO_MLP_NOALLOC_MAX_ROWS rows. Host code reaches it only through the
// device address hipGetSymbolAddress returns (per device, at the first call on
// that device); the array's name itself is not a device address on the host.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t up256c(size_t v) { return (v + 255) / 256 * 256; }
// bytes of the scratch for a padded batch of kp rows (kp a multiple of 32)
constexpr size_t noalloc_bytes(size_t kp) {
  return up256c(2 * (size_t)MI * kp) + 4 * up256c(2 * (size_t)MH * kp) + up256c(2 * (size_t)MO * kp) +
         2 * up256c(4 * (size_t)MO * kp) + up256c(4);
}
constexpr size_t kNoallocBytes = noalloc_bytes(VIO_MLP_NOALLOC_MAX_ROWS);
static_assert(VIO_MLP_NOALLOC_MAX_ROWS % 32 == 0, "row maximum is a whole number of MFMA batch steps");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};  // per device ordinal

// the current device's scratch address (looked up once per device, with that
// device current); nullptr on a HIP error
void* noalloc_scratch(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  *dev_out = dev;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// The training scratch laid out in `base` for a padded batch of kp rows: the
// same sub-buffers as a handle's arena, with the batch as leading dimension.
struct NoallocLayout {
  MlpScratch S;
  float* y;
};
NoallocLayout noalloc_layout(unsigned char* base, int kp) {
  size_t off = 0;
  auto take = [&](size_t b) {
    unsigned char* p = base + off;
    off = up256c(off + b);
    return p;
  };
  NoallocLayout L{};
  L.S.ldt = kp;
  L.S.Xt = reinterpret_cast<uint16_t*>(take(2 * (size_t)MI * kp));
  L.S.H1t = reinterpret_cast<uint16_t*>(take(2 * (size_t)MH * kp));
  L.S.H2t = reinterpret_cast<uint16_t*>(take(2 * (size_t)MH * kp));
  L.S.dYt = reinterpret_cast<uint16_t*>(take(2 * (size_t)MO * kp));
  L.S.dH2t = reinterpret_cast<uint16_t*>(take(2 * (size_t)MH * kp));
  L.S.dH1t = reinterpret_cast<uint16_t*>(take(2 * (size_t)MH * kp));
  L.S.dY = reinterpret_cast<float*>(take(4 * (size_t)MO * kp));
  L.y = reinterpret_cast<float*>(take(4 * (size_t)MO * kp));
  L.S.loss = reinterpret_cast<float*>(take(4));
  return L;
}
}  // namespace

hipError_t mlp_forward_launch(const MlpDev& M, const float* X, int K, float* Y, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const int Kpad = (K + 15) / 16 * 16;
  const int blocks = (Kpad / 16 + kInferWaves - 1) / kInferWaves;
  launch_kernel(k_mlp_infer, dim3(blocks), dim3(64 * kInferWaves), 0, s, M, X, K, Kpad, Y);
  return hipGetLastError();
}

}  // namespace vio

// ===========================================================================
// C ABI
// ===========================================================================
using namespace vio;

struct vio_mlp {
  int max_batch = 0;
  void* arena = nullptr;
  MlpDev M{};
  MlpScratch S{};
  float* d_y = nullptr;   // [ldt][3]
  float* d_g = nullptr;   // [NP]
  float* h_loss = nullptr;
  int step = 0;
  int n_tiles = 0;
};

namespace {
size_t up256(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

extern "C" {

int vio_mlp_create(int32_t max_batch, vio_mlp** out) {
  if (!out || max_batch < 1 || max_batch > 65536) return VIO_EINVAL;
  *out = nullptr;
  auto* m = new (std::nothrow) vio_mlp();
  if (!m) return VIO_ENOMEM;
  m->max_batch = max_batch;
  const int ldt = (max_batch + 31) / 32 * 32;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = up256(off + b);
    return o;
  };
  const size_t oP = take(4 * NP), om = take(4 * NP), ov = take(4 * NP), oW1 = take(2 * MH * MI), oW2 = take(2 * MH * MH),
               oW2t = take(2 * MH * MH), oW3 = take(2 * MO * MH), oXt = take(2 * (size_t)MI * ldt),
               oH1 = take(2 * (size_t)MH * ldt), oH2 = take(2 * (size_t)MH * ldt), odYt = take(2 * (size_t)MO * ldt),
               odH2 = take(2 * (size_t)MH * ldt), odH1 = take(2 * (size_t)MH * ldt), odY = take(4 * (size_t)MO * ldt),
               oL = take(4), oy = take(4 * (size_t)MO * ldt), og = take(4 * NP);
  if (hipMalloc(&m->arena, off) != hipSuccess) {
    delete m;
    return VIO_ENOMEM;
  }
  if (hipMemset(m->arena, 0, off) != hipSuccess ||
      hipHostMalloc((void**)&m->h_loss, sizeof(float)) != hipSuccess) {
    vio_mlp_destroy(m);
    return VIO_EDEVICE;
  }
  char* b = static_cast<char*>(m->arena);
  m->M = {reinterpret_cast<float*>(b + oP), reinterpret_cast<float*>(b + om), reinterpret_cast<float*>(b + ov),
          reinterpret_cast<uint16_t*>(b + oW1), reinterpret_cast<uint16_t*>(b + oW2),
          reinterpret_cast<uint16_t*>(b + oW2t), reinterpret_cast<uint16_t*>(b + oW3)};
  m->S = {ldt,
          reinterpret_cast<uint16_t*>(b + oXt),
          reinterpret_cast<uint16_t*>(b + oH1),
          reinterpret_cast<uint16_t*>(b + oH2),
          reinterpret_cast<uint16_t*>(b + odYt),
          reinterpret_cast<uint16_t*>(b + odH2),
          reinterpret_cast<uint16_t*>(b + odH1),
          reinterpret_cast<float*>(b + odY),
          reinterpret_cast<float*>(b + oL)};
  m->d_y = reinterpret_cast<float*>(b + oy);
  m->d_g = reinterpret_cast<float*>(b + og);
  const std::vector<GradTile> tiles = grad_tiles();
  m->n_tiles = (int)tiles.size();
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_tiles), tiles.data(), sizeof(GradTile) * tiles.size()) != hipSuccess) {
    vio_mlp_destroy(m);
    return VIO_EDEVICE;
  }
  *out = m;
  return VIO_OK;
}

void vio_mlp_destroy(vio_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  if (m->arena) (void)hipFree(m->arena);
  if (m->h_loss) (void)hipHostFree(m->h_loss);
  delete m;
}

int vio_mlp_set_params(vio_mlp* m, const float* params, int32_t n) {
  if (!m || !params || n != NP) return VIO_EINVAL;
  if (hipMemcpy(m->M.P, params, 4 * NP, hipMemcpyHostToDevice) != hipSuccess) return VIO_EDEVICE;
  if (hipMemset(m->M.m, 0, 4 * NP) != hipSuccess || hipMemset(m->M.v, 0, 4 * NP) != hipSuccess) return VIO_EDEVICE;
  m->step = 0;
  if (mlp_pack_launch(m->M, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return VIO_EDEVICE;
  return VIO_OK;
}

int vio_mlp_get_params(vio_mlp* m, float* params, int32_t n) {
  if (!m || !params || n < NP) return VIO_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return VIO_EDEVICE;
  return hipMemcpy(params, m->M.P, 4 * NP, hipMemcpyDeviceToHost) == hipSuccess ? VIO_OK : VIO_EDEVICE;
}

int vio_mlp_forward(vio_mlp* m, const float* d_x, int32_t k, float* d_y, void* hip_stream) {
  if (!m || !d_x || !d_y || k < 0) return VIO_EINVAL;
  return mlp_forward_launch(m->M, d_x, k, d_y, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? VIO_OK
                                                                                                  : VIO_EDEVICE;
}

// Forward, loss, backward and weight gradients of a batch through the
// training scratch S (every scratch row the kernels read, padding rows
// included, is written earlier in the same sequence) and forward output y.
static int gradient_impl(vio_mlp* m, const float* d_x, const float* d_t, int k, float* d_grad, const MlpScratch& S,
                         float* y, hipStream_t s) {
  const int Kpad = (k + 31) / 32 * 32;
  const int blocks = (Kpad / 16 + kMlpWaves - 1) / kMlpWaves;
  hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(blocks), dim3(64 * kMlpWaves), 0, s, m->M, d_x, k, Kpad, y, S);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(1024), 0, s, (const float*)y, d_t, k, Kpad, S);
  hipLaunchKernelGGL(k_mlp_bwd_data, dim3(blocks), dim3(64 * kMlpWaves), 0, s, m->M, Kpad, S);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((m->n_tiles + kMlpWaves - 1) / kMlpWaves), dim3(64 * kMlpWaves), 0, s,
                     m->n_tiles, Kpad, S, d_grad);
  return hipGetLastError() == hipSuccess ? VIO_OK : VIO_EDEVICE;
}

int vio_mlp_gradient(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float* d_grad, float* loss,
                     void* hip_stream) {
  if (!m || !d_x || !d_targets || !d_grad || k < 1 || k > m->max_batch) return VIO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = gradient_impl(m, d_x, d_targets, k, d_grad, m->S, m->d_y, s);
  if (rc != VIO_OK) return rc;
  if (hipMemcpyAsync(m->h_loss, m->S.loss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return VIO_EDEVICE;
  if (loss) *loss = *m->h_loss;
  return VIO_OK;
}

int vio_mlp_gradient_noalloc(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float* d_grad,
                             float* loss, void* hip_stream) {
  if (!m || !d_x || !d_targets || !d_grad || k < 1 || k > VIO_MLP_NOALLOC_MAX_ROWS) return VIO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  void* base = noalloc_scratch(&dev);
  if (!base) return VIO_EDEVICE;
  const NoallocLayout L = noalloc_layout(static_cast<unsigned char*>(base), (k + 31) / 32 * 32);
  int rc = gradient_impl(m, d_x, d_targets, k, d_grad, L.S, L.y, s);
  if (rc != VIO_OK) return rc;
  if (hipMemcpyAsync(m->h_loss, L.S.loss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return VIO_EDEVICE;
  if (loss) *loss = *m->h_loss;
  return VIO_OK;
}

int vio_mlp_train_step(vio_mlp* m, const float* d_x, const float* d_targets, int32_t k, float lr, float* loss,
                       void* hip_stream) {
  if (!m || !d_x || !d_targets || k < 1 || k > m->max_batch || !(lr > 0.f)) return VIO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = gradient_impl(m, d_x, d_targets, k, m->d_g, m->S, m->d_y, s);
  if (rc != VIO_OK) return rc;
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, s, m->M, (const float*)m->d_g, m->step, lr, b1,
                     b2, 1e-8f, c1, c2);
  if (hipGetLastError() != hipSuccess) return VIO_EDEVICE;
  if (loss) {
    if (hipMemcpyAsync(m->h_loss, m->S.loss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return VIO_EDEVICE;
    *loss = *m->h_loss;
  }
  return VIO_OK;
}

}  // extern "C"
