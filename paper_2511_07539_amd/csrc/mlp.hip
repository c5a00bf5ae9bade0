// Learned warm start for the NLTE solve: an MLP 6 -> 256 -> 256 -> 256 -> 100
// (SiLU hidden layers) from cell features to log10 level populations, trained
// and evaluated by the kernels below.
//
// GEMMs run on the matrix cores: v_mfma_f32_16x16x16bf16 with BF16 operands
// (FP32 values rounded when staged into LDS) and FP32 accumulation. Master
// weights, activations, gradients and the Adam moments stay FP32. A 64x64
// output tile per 256-thread workgroup, each wavefront owning a 32x32 quarter
// as 2x2 MFMA tiles; K advances 64 at a time through LDS. Weight gradients
// reduce over the batch, so their K range is split across workgroups that add
// into a zeroed FP32 result. The first layer (K = 6) is too thin for a
// matrix instruction and runs as plain FP32 FMAs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "atom.hpp"
#include "common.hpp"

namespace extrass {
namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 6, kHid = 256, kOut = 100;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid,
                  kOffB3 = kOffW3 + kHid * kHid, kOffW4 = kOffB3 + kHid,
                  kOffB4 = kOffW4 + kOut * kHid, kParams = kOffB4 + kOut;

constexpr int BM = 64, BN = 64, BK = 64, KPAD = 4;

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_ATOMIC = 3 };

struct Gemm {
  int M, N, K;
  const float* A;  // element (m, k) at A[m*sam + k*sak]
  int64_t sam, sak;
  const float* B;  // element (k, n) at B[k*sbk + n*sbn]
  int64_t sbk, sbn;
  float* C;        // element (m, n) at C[m*ldc + n]
  int64_t ldc;
  const float* bias;  // [N]
  float* act;         // silu(C), same layout
  int mode;
  int ksplit;         // K range per blockIdx.z
};

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ __bf16 As[BM][BK + KPAD];
  __shared__ __bf16 Bs[BN][BK + KPAD];  // transposed: [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int kbeg = blockIdx.z * g.ksplit;
  const int kend = min(g.K, kbeg + g.ksplit);
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK, kk = e % BK, m = m0 + r, k = k0 + kk;
      const float v = (m < g.M && k < kend) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.f;
      As[r][kk] = static_cast<__bf16>(v);
    }
    for (int e = tid; e < BN * BK; e += 256) {
      const int r = e / BK, kk = e % BK, n = n0 + r, k = k0 + kk;
      const float v = (n < g.N && k < kend) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.f;
      Bs[r][kk] = static_cast<__bf16>(v);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int kq = ks + 4 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        bf16x4 a;
        const int ar = wm + i * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = As[ar][kq + q];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          bf16x4 b;
          const int br = wn + j * 16 + (lane & 15);
#pragma unroll
          for (int q = 0; q < 4; ++q) b[q] = Bs[br][kq + q];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // D layout of the 16x16 tile: lane holds column lane%16, rows 4*(lane/16) + q
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + q;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][q];
        const int64_t o = (int64_t)m * g.ldc + n;
        if (g.mode == EPI_ATOMIC) {
          atomicAdd(g.C + o, v);
        } else {
          if (g.mode != EPI_STORE) v += g.bias[n];
          g.C[o] = v;
          if (g.mode == EPI_BIAS_SILU) g.act[o] = silu(v);
        }
      }
}

// First layer, K = 6: z1 = x W1^T + b1, a1 = silu(z1).
__global__ void k_layer1(const float* __restrict__ x, const float* __restrict__ P, int64_t B,
                         float* __restrict__ z, float* __restrict__ a) {
  const int64_t total = B * kHid;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / kHid;
    const int o = (int)(e - b * kHid);
    float s = P[kOffB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) s += x[b * kIn + i] * P[kOffW1 + o * kIn + i];
    z[e] = s;
    a[e] = silu(s);
  }
}

// dy = 2 (y - t) / (B*O), loss += sum (y - t)^2 / (B*O)
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                      float inv, float* __restrict__ dy, float* __restrict__ loss) {
  float acc = 0.f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[e] - t[e];
    dy[e] = 2.f * r * inv;
    acc += r * r * inv;
  }
  // one atomic per block: wavefront sums, then the block's sum in LDS
  __shared__ float part[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (part[0] + part[1]) + (part[2] + part[3]));
}

__global__ void k_dsilu(const float* __restrict__ da, const float* __restrict__ z, int64_t n,
                        float* __restrict__ dz) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dz[e] = da[e] * dsilu(z[e]);
}

// column sums of a [B, N] matrix into g[N] (bias gradients), atomics per block
__global__ void k_colsum(const float* __restrict__ d, int64_t B, int N, float* __restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t rows = (B + gridDim.y - 1) / gridDim.y;
  const int64_t r0 = blockIdx.y * rows, r1 = min(B, r0 + rows);
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) s += d[r * N + n];
  atomicAdd(g + n, s);
}

// dW1[o][i] = sum_b dz1[b][o] x[b][i]  (K = batch, 256 x 6 outputs)
__global__ void k_dw1(const float* __restrict__ dz, const float* __restrict__ x, int64_t B,
                      float* __restrict__ g) {
  const int o = threadIdx.x;  // 256 threads
  const int64_t rows = (B + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * rows, r1 = min(B, r0 + rows);
  float s[kIn] = {0, 0, 0, 0, 0, 0};
  for (int64_t r = r0; r < r1; ++r) {
    const float d = dz[r * kHid + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) s[i] += d * x[r * kIn + i];
  }
#pragma unroll
  for (int i = 0; i < kIn; ++i) atomicAdd(g + kOffW1 + o * kIn + i, s[i]);
}

__global__ void k_fill(float* p, int64_t n, float v) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = 0.9f * m[e] + 0.1f * gi;
    const float vi = 0.999f * v[e] + 0.001f * gi * gi;
    m[e] = mi;
    v[e] = vi;
    P[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  }
}

struct Acts {
  float *z1, *a1, *z2, *a2, *z3, *a3, *y, *dy, *da, *dz, *grad;
};

size_t acts_bytes(int64_t B) {
  return carve_bytes<float>(B * kHid) * 8 + carve_bytes<float>(B * kOut) * 2 +
         carve_bytes<float>(kParams) + 512;
}

Acts carve_acts(void* ws, int64_t B) {
  Carver cv(ws, ~size_t(0));
  Acts a;
  a.z1 = cv.take<float>(B * kHid);
  a.a1 = cv.take<float>(B * kHid);
  a.z2 = cv.take<float>(B * kHid);
  a.a2 = cv.take<float>(B * kHid);
  a.z3 = cv.take<float>(B * kHid);
  a.a3 = cv.take<float>(B * kHid);
  a.da = cv.take<float>(B * kHid);
  a.dz = cv.take<float>(B * kHid);
  a.y = cv.take<float>(B * kOut);
  a.dy = cv.take<float>(B * kOut);
  a.grad = cv.take<float>(kParams);
  return a;
}

inline unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

void gemm(hipStream_t st, Gemm g) {
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, 1);
  if (g.mode == EPI_ATOMIC) {
    // split K so that the grid has a few hundred workgroups
    int tiles = grid.x * grid.y;
    int splits = std::max(1, std::min(256 / std::max(tiles, 1) * 2, (g.K + 255) / 256));
    g.ksplit = ((g.K + splits - 1) / splits + BK - 1) / BK * BK;
    grid.z = (g.K + g.ksplit - 1) / g.ksplit;
  } else {
    g.ksplit = ((g.K + BK - 1) / BK) * BK;
  }
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
}

void forward(hipStream_t st, const float* P, const float* x, int64_t B, const Acts& a) {
  hipLaunchKernelGGL(k_layer1, dim3(blocks_for(B * kHid)), dim3(256), 0, st, x, P, B, a.z1, a.a1);
  // z = a_prev W^T + b: A = a_prev [B, 256] row-major, B(k, n) = W[n][k]
  gemm(st, Gemm{(int)B, kHid, kHid, a.a1, kHid, 1, P + kOffW2, 1, kHid, a.z2, kHid, P + kOffB2,
                a.a2, EPI_BIAS_SILU, 0});
  gemm(st, Gemm{(int)B, kHid, kHid, a.a2, kHid, 1, P + kOffW3, 1, kHid, a.z3, kHid, P + kOffB3,
                a.a3, EPI_BIAS_SILU, 0});
  gemm(st, Gemm{(int)B, kOut, kHid, a.a3, kHid, 1, P + kOffW4, 1, kHid, a.y, kOut, P + kOffB4,
                nullptr, EPI_BIAS, 0});
}

// gradient of the MSE w.r.t. all parameters into g (zeroed here)
void backward(hipStream_t st, const float* P, const float* x, const float* t, int64_t B,
              const Acts& a, float* g, float* loss) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(kParams)), dim3(256), 0, st, g, kParams, 0.f);
  hipLaunchKernelGGL(k_mse, dim3((unsigned)std::min<int64_t>(blocks_for(B * kOut), 512)), dim3(256),
                     0, st, a.y, t, B * kOut, 1.0f / (float)(B * kOut), a.dy, loss);
  // row splits of the column sums and of dW1: enough work-groups to fill the
  // GPU, 16 rows each (atomics then land on N addresses from B/16 groups)
  const unsigned ysplit = (unsigned)std::max<int64_t>(1, std::min<int64_t>(B / 16, 1024));
  // output layer: dW4 = dy^T a3, db4 = colsum(dy), da3 = dy W4
  gemm(st, Gemm{kOut, kHid, (int)B, a.dy, 1, kOut, a.a3, kHid, 1, g + kOffW4, kHid, nullptr,
                nullptr, EPI_ATOMIC, 0});
  hipLaunchKernelGGL(k_colsum, dim3((kOut + 255) / 256, ysplit), dim3(256), 0, st, a.dy, B, kOut,
                     g + kOffB4);
  gemm(st, Gemm{(int)B, kHid, kOut, a.dy, kOut, 1, P + kOffW4, kHid, 1, a.da, kHid, nullptr,
                nullptr, EPI_STORE, 0});
  // hidden layers 3 and 2
  const float* zs[2] = {a.z3, a.z2};
  const float* ins[2] = {a.a2, a.a1};
  const int64_t offW[2] = {kOffW3, kOffW2}, offB[2] = {kOffB3, kOffB2};
  for (int l = 0; l < 2; ++l) {
    hipLaunchKernelGGL(k_dsilu, dim3(blocks_for(B * kHid)), dim3(256), 0, st, a.da, zs[l],
                       B * kHid, a.dz);
    gemm(st, Gemm{kHid, kHid, (int)B, a.dz, 1, kHid, ins[l], kHid, 1, g + offW[l], kHid, nullptr,
                  nullptr, EPI_ATOMIC, 0});
    hipLaunchKernelGGL(k_colsum, dim3(1, ysplit), dim3(256), 0, st, a.dz, B, kHid, g + offB[l]);
    gemm(st, Gemm{(int)B, kHid, kHid, a.dz, kHid, 1, P + offW[l], kHid, 1, a.da, kHid, nullptr,
                  nullptr, EPI_STORE, 0});
  }
  // first layer
  hipLaunchKernelGGL(k_dsilu, dim3(blocks_for(B * kHid)), dim3(256), 0, st, a.da, a.z1, B * kHid,
                     a.dz);
  hipLaunchKernelGGL(k_dw1, dim3(ysplit), dim3(256), 0, st, a.dz, x, B, g);
  hipLaunchKernelGGL(k_colsum, dim3(1, ysplit), dim3(256), 0, st, a.dz, B, kHid, g + kOffB1);
}

// ---- warm start: features -> MLP -> populations ----------------------------

// Features of a cell: log10 n_tot, log10 T_e, log10 n_e, log10 deposition and
// the number fractions of the two species, each normalised by (mean, std).
// Inference of the whole network, 64 rows per work-group of 4 wavefronts
// (16 rows each). Layer 1 is computed in FP32 as k_layer1 computes it; the
// hidden and output layers run on BF16 MFMA 16x16x16 with K taken in chunks
// of 64 and steps of 16, the order k_gemm takes it, so every output equals
// forward()'s. The activations stay in LDS as BF16, the value k_gemm rounds
// them to when it stages its next A tile. The weights, converted to BF16
// once per call (k_weights_bf16, the same rounding k_gemm applies when it
// stages them), are staged in 64 x 64 tiles with 16-byte loads. One launch
// replaces layer 1 and three GEMMs, and no pre-activation is written.
constexpr int kIR = 64;           // rows per work-group
constexpr int kHS = kHid + 8;     // LDS row stride of the activations (bf16)
constexpr int kWS = BK + 8;       // LDS row stride of a weight tile (bf16; rows 16-byte aligned)
constexpr int64_t kWb2 = 0, kWb3 = kWb2 + kHid * kHid, kWb4 = kWb3 + kHid * kHid,
                  kWbN = kWb4 + kOut * kHid;  // BF16 copies of W2, W3, W4

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ void k_weights_bf16(const float* __restrict__ P, __bf16* __restrict__ Wb) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < kWbN;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = i < kWb3 ? kOffW2 + i : (i < kWb4 ? kOffW3 + (i - kWb3) : kOffW4 + (i - kWb4));
    Wb[i] = static_cast<__bf16>(P[src]);
  }
}

// One weight tile: rows n in [nc, nc + 64), columns k in [kc, kc + 64) of
// W[n][k] (row-major BF16), 8 values per load; two loads per thread.
__device__ __forceinline__ void load_wtile(const __bf16* W, int N, int nc, int kc, bf16x8 (&v)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int e = threadIdx.x + 256 * i;
    const int r = e / (BK / 8), kk = 8 * (e % (BK / 8)), n = nc + r;
    if (n < N) {
      v[i] = *reinterpret_cast<const bf16x8*>(W + n * kHid + kc + kk);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[i][q] = static_cast<__bf16>(0.f);
    }
  }
}
__device__ __forceinline__ void store_wtile(__bf16 (*Ws)[kWS], const bf16x8 (&v)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int e = threadIdx.x + 256 * i;
    *reinterpret_cast<bf16x8*>(&Ws[e / (BK / 8)][8 * (e % (BK / 8))]) = v[i];
  }
}

__device__ __forceinline__ void infer_layer(__bf16 (*H)[kHS], __bf16 (*Ws)[64][kWS], const __bf16* W,
                                            const float* bias, int N, bool silu_out, float* y,
                                            int64_t row0, int64_t B) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ntile = (N + 15) / 16;  // 16 for the hidden layers, 7 for the output layer
  const int ncs = (ntile + 3) / 4;  // 64-column tiles
  const int stages = (kHid / BK) * ncs;  // (kc, nc) with nc fastest: K stays in order per column
  f32x4 acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ar = wave * 16 + (lane & 15);
  (void)tid;
  bf16x8 v[2];
  load_wtile(W, N, 0, 0, v);
  store_wtile(Ws[0], v);
  __syncthreads();
  for (int sg = 0; sg < stages; ++sg) {
    const int kc = (sg / ncs) * BK, nc = (sg % ncs) * 64;
    // the next tile's loads are in flight during this tile's products
    if (sg + 1 < stages) load_wtile(W, N, ((sg + 1) % ncs) * 64, ((sg + 1) / ncs) * BK, v);
    __bf16 (*Wt)[kWS] = Ws[sg & 1];
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int kq = ks + 4 * (lane >> 4);
      bf16x4 a;
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = H[ar][kc + kq + q];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int tt = nc / 16 + t;
        if (tt < ntile) {
          bf16x4 b;
#pragma unroll
          for (int q = 0; q < 4; ++q) b[q] = Wt[t * 16 + (lane & 15)][kq + q];
          acc[tt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[tt], 0, 0, 0);
        }
      }
    }
    if (sg + 1 < stages) store_wtile(Ws[(sg + 1) & 1], v);
    __syncthreads();
  }
  // every wave has read its rows of H: write the layer's output in place
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t >= ntile) break;
    const int n = t * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = wave * 16 + 4 * (lane >> 4) + q;
      if (n >= N) continue;
      const float v = acc[t][q] + bias[n];
      if (silu_out) {
        H[r][n] = static_cast<__bf16>(silu(v));
      } else if (row0 + r < B) {
        y[(row0 + r) * kOut + n] = v;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ x,
                                                   const float* __restrict__ P,
                                                   const __bf16* __restrict__ Wb, int64_t B,
                                                   float* __restrict__ y) {
  __shared__ __bf16 H[kIR][kHS];
  __shared__ __align__(16) __bf16 Ws[2][64][kWS];
  const int64_t row0 = (int64_t)blockIdx.x * kIR;
  // layer 1 (K = 6), as k_layer1
  for (int e = threadIdx.x; e < kIR * kHid; e += 256) {
    const int r = e / kHid, o = e % kHid;
    const int64_t b = row0 + r;
    float s = P[kOffB1 + o];
    if (b < B) {
#pragma unroll
      for (int i = 0; i < kIn; ++i) s += x[b * kIn + i] * P[kOffW1 + o * kIn + i];
    }
    H[r][o] = static_cast<__bf16>(silu(s));
  }
  __syncthreads();
  infer_layer(H, Ws, Wb + kWb2, P + kOffB2, kHid, true, nullptr, row0, B);
  infer_layer(H, Ws, Wb + kWb3, P + kOffB3, kHid, true, nullptr, row0, B);
  infer_layer(H, Ws, Wb + kWb4, P + kOffB4, kOut, false, y, row0, B);
}

// The six warm-start features of each cell, normalised by norm (means, then
// standard deviations) or raw when norm is NULL.
__global__ void k_features(int64_t c0, int64_t n, int S, const double* __restrict__ T,
                           const double* __restrict__ ne, const double* __restrict__ ns,
                           const double* __restrict__ dep, const float* __restrict__ norm,
                           float* __restrict__ x) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = c0 + e;
    double tot = 0.0;
    for (int s = 0; s < S; ++s) tot += ns[c * S + s];
    const double safe = tot > 0.0 ? tot : 1.0;
    double f[kIn];
    f[0] = log10(safe);
    f[1] = log10(T[c]);
    f[2] = log10(ne[c] > 0.0 ? ne[c] : 1.0);
    f[3] = log10(dep[c] > 0.0 ? dep[c] : 1e-30);
    f[4] = ns[c * S + 0] / safe;
    f[5] = ns[c * S + 1] / safe;
    for (int i = 0; i < kIn; ++i)
      x[e * kIn + i] = norm ? (float)((f[i] - norm[i]) / norm[kIn + i]) : (float)f[i];
  }
}

// y (normalised log10 n_i / n_species) -> populations, renormalised per species
// One wavefront per (cell, species), lane i holding the species' level i (a
// species has at most 64 levels): log10 populations from the network's
// normalised outputs, scaled to the species' total.
__global__ __launch_bounds__(256) void k_warm_out(int64_t c0, int64_t n, int S,
                                                 const int32_t* __restrict__ off,
                                                 const double* __restrict__ ns,
                                                 const float* __restrict__ norm,
                                                 const float* __restrict__ y,
                                                 double* __restrict__ pops) {
  const float* ym = norm + 2 * kIn;
  const float* ys = ym + kOut;
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= n * S) return;  // whole wavefronts
  const int64_t cl = item / S;
  const int s = (int)(item - cl * S);
  const int64_t c = c0 + cl;
  const int i = off[s] + lane;
  const bool live = i < off[s + 1];
  const double v = live ? (double)(y[cl * kOut + i] * ys[i] + ym[i]) : -1e300;
  const double mx = wave_max(v);
  const double e = live ? exp10(v - mx) : 0.0;
  const double sum = wave_sum(e);
  const double ntot = ns[c * S + s];
  if (live) pops[c * kOut + i] = ntot > 0.0 ? ntot * e / sum : 0.0;
}

}  // namespace
}  // namespace extrass

using namespace extrass;

extern "C" size_t extrass_mlp_param_count(void) { return (size_t)kParams; }

extern "C" size_t extrass_mlp_workspace(int64_t batch) {
  if (batch <= 0) return 0;
  return acts_bytes(batch);
}

extern "C" int extrass_mlp_forward(extrass_handle h, const float* params, const float* x, float* y,
                                   int64_t batch, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !params || !x || !y || !ws || batch <= 0 || batch > (1 << 24))
    return fail(h, EXTRASS_EINVAL, "extrass_mlp_forward: bad argument");
  if (ws_bytes < acts_bytes(batch))
    return fail(h, EXTRASS_ENOSPACE, "extrass_mlp_forward: workspace too small");
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Acts a = carve_acts(ws, batch);
  a.y = y;
  forward(st, params, x, batch, a);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

extern "C" int extrass_mlp_train_step(extrass_handle h, float* params, float* adam_m,
                                      float* adam_v, int32_t step, float lr, const float* x,
                                      const float* t, int64_t batch, float* loss, float* grad,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!h || !params || !x || !t || !ws || batch <= 0 || batch > (1 << 24))
    return fail(h, EXTRASS_EINVAL, "extrass_mlp_train_step: bad argument");
  if ((adam_m == nullptr) != (adam_v == nullptr) || (adam_m && step < 1))
    return fail(h, EXTRASS_EINVAL, "extrass_mlp_train_step: Adam state or step missing");
  if (ws_bytes < acts_bytes(batch))
    return fail(h, EXTRASS_ENOSPACE, "extrass_mlp_train_step: workspace too small");
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Acts a = carve_acts(ws, batch);
  float* g = grad ? grad : a.grad;
  forward(st, params, x, batch, a);
  backward(st, params, x, t, batch, a, g, loss);
  if (adam_m) {
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)step));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams)), dim3(256), 0, st, params, adam_m, adam_v,
                       g, kParams, lr, c1, c2);
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

extern "C" int extrass_mlp_features(extrass_handle h, extrass_atom_handle atom,
                                    const extrass_cells* cells, const double* deposition,
                                    float* x, void* stream) {
  if (!h || !atom || !cells || !deposition || !x || !cells->T_e || !cells->n_e ||
      !cells->n_species || cells->n_cells < 0)
    return fail(h, EXTRASS_EINVAL, "extrass_mlp_features: bad argument");
  if (atom->S != 2)
    return fail(h, EXTRASS_EINVAL, "extrass_mlp_features: the features need 2 species");
  if (cells->n_cells == 0) return EXTRASS_OK;
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipLaunchKernelGGL(k_features, dim3(blocks_for(cells->n_cells)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), (int64_t)0, cells->n_cells, atom->S,
                     cells->T_e, cells->n_e, cells->n_species, deposition,
                     static_cast<const float*>(nullptr), x);
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}

extern "C" size_t extrass_nlte_warm_start_workspace(int64_t n_cells) {
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(n_cells, 1), 65536);
  return acts_bytes(chunk) + carve_bytes<float>(chunk * kIn) + kWbN * sizeof(__bf16) + 512;
}

extern "C" int extrass_nlte_warm_start(extrass_handle h, extrass_atom_handle atom,
                                       const extrass_cells* cells, const double* deposition,
                                       const float* params, const float* norm, double* pops,
                                       void* ws, size_t ws_bytes, void* stream) {
  if (!h || !atom || !cells || !deposition || !params || !norm || !pops || !ws)
    return fail(h, EXTRASS_EINVAL, "extrass_nlte_warm_start: null argument");
  if (atom->N != kOut || atom->S != 2)
    return fail(h, EXTRASS_EUNSUPPORTED,
                "extrass_nlte_warm_start: the network predicts 100 levels of 2 species");
  const int64_t C = cells->n_cells;
  if (C <= 0) return EXTRASS_OK;
  if (ws_bytes < extrass_nlte_warm_start_workspace(C))
    return fail(h, EXTRASS_ENOSPACE, "extrass_nlte_warm_start: workspace too small");
  EXTRASS_HIP_TRY(h, hipSetDevice(h->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t chunk = std::min<int64_t>(C, 65536);
  Acts a = carve_acts(ws, chunk);
  float* x = reinterpret_cast<float*>(static_cast<char*>(ws) + acts_bytes(chunk));
  // 256-byte aligned, after the features
  const uintptr_t wb_at = (reinterpret_cast<uintptr_t>(x + chunk * kIn) + 255) & ~uintptr_t(255);
  __bf16* wb = reinterpret_cast<__bf16*>(wb_at);
  hipLaunchKernelGGL(k_weights_bf16, dim3(blocks_for(kWbN)), dim3(256), 0, st, params, wb);
  for (int64_t c0 = 0; c0 < C; c0 += chunk) {
    const int64_t n = std::min(chunk, C - c0);
    hipLaunchKernelGGL(k_features, dim3(blocks_for(n)), dim3(256), 0, st, c0, n, atom->S,
                       cells->T_e, cells->n_e, cells->n_species, deposition, norm, x);
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((n + kIR - 1) / kIR)), dim3(256), 0, st, x,
                       params, wb, n, a.y);
    hipLaunchKernelGGL(k_warm_out, dim3((unsigned)((n * atom->S + 3) / 4)), dim3(256), 0, st, c0,
                       n, atom->S, atom->d.off, cells->n_species, norm, a.y, pops);
  }
  EXTRASS_HIP_TRY(h, hipGetLastError());
  return EXTRASS_OK;
}
