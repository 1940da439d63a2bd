// Learned FFCP initializer (the initialization step of Algorithm 1).
//
// A 3-layer MLP maps a normalized Tucker core x = vec(G)/||G|| to
// compressed CP factors V_n (R_n x R) of that core:
//     h1 = gelu(x W1 + b1),  h2 = gelu(h1 W2 + b2),  y = h2 W3 + b3,
//     y = [vec V_1, ..., vec V_N]  (row-major V_n),
// trained on the CP reconstruction loss of the core,
//     L = ||G/||G|| - [[V_1, ..., V_N]]||^2,
// whose gradient with respect to V_n is eq. (5) applied to the core
// (FFCP on an orthonormal Tucker format is CP of the core, eq. (17)):
//     dL/dV_n = 2 (V_n hadamard_{p != n} V_p^T V_p - Ghat_(n) KR_{p != n} V_p).
// FFCP starts from V_n ||G||^(1/N) (A_n = U_n V_n).
//
// Every matrix product runs on v_mfma_f32_32x32x16_bf16: BF16 operands
// (weights, activations, and in the backward pass the output and
// pre-activation gradients), FP32 accumulation; master weights, biases and
// Adam moments are FP32.  The core loss and its gradient are computed in
// FP32, one workgroup per core.
#include <cmath>

#include "../../include/rtucker.h"
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kTM = 64, kTK = 32, kLdsK = 40;   // GEMM tile (M = N = 64, K = 32)

enum { kEpiStore = 0, kEpiBiasGelu = 1, kEpiBias = 2, kEpiDGelu = 3 };

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  int lda;
  const uint16_t* B;
  int ldb;
  float* C;          // FP32 result (ldc)
  int ldc;
  uint16_t* Cb;      // BF16 result (same layout), or null
  const float* bias;  // per column n
  const float* Zin;   // pre-activation (ldc layout) for the GELU derivative
  // split-K: workgroup z of the grid takes k in [z kper, (z + 1) kper) and
  // writes its FP32 partial product to part[z][M][N] (the epilogue follows
  // in gemm_finish_kernel); part == null: one range, epilogue in place
  int kper;
  float* part;
};

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = expf(-0.5f * z * z) * 0.39894228040143268f;
  return cdf + z * pdf;
}

// 8 consecutive BF16 values at p (elements e0.. of a row of length `len`);
// entries past `len` or past the matrix are zero.
__device__ __forceinline__ uint4 load8(const uint16_t* row, int e0, int len, bool rowok) {
  if (rowok && e0 + 8 <= len) return *reinterpret_cast<const uint4*>(row + e0);
  uint16_t h[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = (rowok && e0 + j < len) ? row[e0 + j] : 0;
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                    h[6] | (h[7] << 16));
}

__device__ __forceinline__ uint16_t half_of(const uint4& u, int j) {
  const uint32_t w = j < 2 ? u.x : (j < 4 ? u.y : (j < 6 ? u.z : u.w));
  return static_cast<uint16_t>(w >> (16 * (j & 1)));
}

// Writes element (m, n) of the product x through the epilogue EPI.
template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int m, int n, float x) {
  const int64_t o = static_cast<int64_t>(m) * g.ldc + n;
  if (EPI == kEpiBias || EPI == kEpiBiasGelu) x += g.bias[n];
  if (EPI == kEpiBiasGelu) {
    g.C[o] = x;                               // pre-activation
    g.Cb[o] = f32_to_bf16_rne(gelu_f(x));     // activation (BF16)
  } else if (EPI == kEpiDGelu) {
    const float d = x * gelu_grad_f(g.Zin[o]);
    g.C[o] = d;
    g.Cb[o] = f32_to_bf16_rne(d);
  } else {
    g.C[o] = x;
    if (g.Cb) g.Cb[o] = f32_to_bf16_rne(x);
  }
}

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
constexpr int kKp = 72;   // halfwords per k-row of a tile staged with k along rows

// MFMA operand (lane l: index c0 + l % 32, k = k0 + 8 (l / 32) + 0..7) from
// a tile staged with k along rows (kKp halfwords per row), by two
// ds_read_b64_tr_b16: lane j of a 16-lane group receives element j % 4 of
// the four halfwords lanes 4 q + j / 4 address (q = 0..3), so lane i of the
// group points at row i / 4 of a 4-row half and columns 4 (i % 4) .. + 3.
__device__ __forceinline__ v8bf kmajor_operand(const uint16_t* tile, int k0, int c0, int lane) {
  const int G = lane >> 4, i = lane & 15;
  const int row = k0 + 8 * (G >> 1) + (i >> 2);
  const int col = c0 + 16 * (G & 1) + 4 * (i & 3);
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(tile + row * kKp + col));
  const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(tile + (row + 4) * kKp + col));
  const v8s v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(v8bf, v);
}

// C (M x N) = op(A) op(B); op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k],
// op(B)[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n].  64 x 64 tiles staged in
// LDS as they are read (K contiguous, or k along rows: then the MFMA operand
// comes through the LDS transpose read); four wavefronts, one 32 x 32 MFMA
// block each.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  constexpr int kTile = kTM * kLdsK > kTK * kKp ? kTM * kLdsK : kTK * kKp;
  __shared__ __align__(16) uint16_t As[kTile];
  __shared__ __align__(16) uint16_t Bs[kTile];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1, lr = lane & 31, gq = lane >> 5;
  const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTM;
  const int kb = g.part ? blockIdx.z * g.kper : 0;
  const int ke = g.part && kb + g.kper < g.K ? kb + g.kper : g.K;   // this range's end
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += kTK) {
    __syncthreads();
    if (!TA) {  // A rows are m: 64 rows x 32 k, 16 bytes per thread
      const int m = t >> 2, k8 = (t & 3) * 8;
      const uint4 u = load8(g.A + static_cast<int64_t>(m0 + m) * g.lda, k0 + k8, ke,
                            m0 + m < g.M);
      *reinterpret_cast<uint4*>(As + m * kLdsK + k8) = u;
    } else {    // A rows are k: 32 rows x 64 m, kept with k along rows
      const int k = t >> 3, m8 = (t & 7) * 8;
      const uint4 u = load8(g.A + static_cast<int64_t>(k0 + k) * g.lda, m0 + m8, g.M,
                            k0 + k < ke);
      *reinterpret_cast<uint4*>(As + k * kKp + m8) = u;
    }
    if (TB) {   // B rows are n
      const int n = t >> 2, k8 = (t & 3) * 8;
      const uint4 u = load8(g.B + static_cast<int64_t>(n0 + n) * g.ldb, k0 + k8, ke,
                            n0 + n < g.N);
      *reinterpret_cast<uint4*>(Bs + n * kLdsK + k8) = u;
    } else {    // B rows are k, kept with k along rows
      const int k = t >> 3, n8 = (t & 7) * 8;
      const uint4 u = load8(g.B + static_cast<int64_t>(k0 + k) * g.ldb, n0 + n8, g.N,
                            k0 + k < ke);
      *reinterpret_cast<uint4*>(Bs + k * kKp + n8) = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 16) {
      const v8bf a = TA ? kmajor_operand(As, kk, wm * 32, lane)
                        : __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(
                                                       As + (wm * 32 + lr) * kLdsK + kk + 8 * gq));
      const v8bf b = !TB ? kmajor_operand(Bs, kk, wn * 32, lane)
                         : __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(
                                                        Bs + (wn * 32 + lr) * kLdsK + kk + 8 * gq));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  }
  const int n = n0 + wn * 32 + lr;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + 8 * (v / 4) + 4 * gq + (v % 4);
    if (m < g.M && n < g.N) {
      if (g.part)
        g.part[(static_cast<int64_t>(blockIdx.z) * g.M + m) * g.N + n] = acc[v];
      else
        epilogue<EPI>(g, m, n, acc[v]);
    }
  }
}

// The split-K ranges' partial products summed in range order, then the
// epilogue.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_finish_kernel(GemmArgs g, int splits) {
  const int64_t o = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t mn = static_cast<int64_t>(g.M) * g.N;
  if (o >= mn) return;
  float x = 0.0f;
  for (int z = 0; z < splits; ++z) x += g.part[z * mn + o];
  epilogue<EPI>(g, static_cast<int>(o / g.N), static_cast<int>(o % g.N), x);
}

// K ranges for a product whose 64 x 64 tiles alone would leave most of the
// 256 compute units idle (the products with M = batch rows): enough ranges
// for about 256 workgroups, each at least 512 deep, at most kSplitMax.
constexpr int kSplitMax = 8;
int gemm_splits(int M, int N, int K) {
  const int tiles = ((N + kTM - 1) / kTM) * ((M + kTM - 1) / kTM);
  if (tiles >= 192 || K < 1024) return 1;
  int sp = (256 + tiles - 1) / tiles;
  sp = sp < K / 512 ? sp : K / 512;
  return sp < kSplitMax ? sp : kSplitMax;
}

// kpart: FP32 scratch of kSplitMax M N floats for the split-K form, or null
// (one range per tile)
template <bool TA, bool TB, int EPI>
int gemm(GemmArgs g, hipStream_t s, float* kpart = nullptr) {
  const int splits = kpart ? gemm_splits(g.M, g.N, g.K) : 1;
  if (splits > 1) {
    g.kper = ((g.K + splits - 1) / splits + kTK - 1) / kTK * kTK;
    g.part = kpart;
  }
  const int used = splits > 1 ? (g.K + g.kper - 1) / g.kper : 1;
  const dim3 grid((g.N + kTM - 1) / kTM, (g.M + kTM - 1) / kTM, used);
  hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), grid, dim3(256), 0, s, g);
  RT_LAUNCH_CHECK("mlp gemm");
  if (splits > 1) {
    const int64_t mn = static_cast<int64_t>(g.M) * g.N;
    hipLaunchKernelGGL(gemm_finish_kernel<EPI>, dim3(static_cast<unsigned>((mn + 255) / 256)),
                       dim3(256), 0, s, g, used);
    RT_LAUNCH_CHECK("mlp gemm finish");
  }
  return kOk;
}

// Few rows (inference on a handful of cores): C = A B with A [M][K] (M <=
// kGvMaxM) and B [K][N] row-major, N % 8 == 0.  The weight matrix is
// streamed once, split over K across the grid: workgroup (x, s) owns 512
// columns and the K rows of chunk s, one wavefront per row residue mod 4,
// 8 columns per lane; the four waves' sums meet in LDS and each chunk's
// partial goes to part[s][m][n].  A second kernel sums the chunks in a
// fixed order and applies the epilogue.
constexpr int kGvMaxM = 8;
constexpr int kGvCols = 512;
constexpr int kGvMaxSplit = 128;

int gemv_splits(int K) {
  const int s = (K + 15) / 16;   // at least 16 rows per chunk
  return s < kGvMaxSplit ? s : kGvMaxSplit;
}

__global__ __launch_bounds__(256) void gemv_partial_kernel(GemmArgs g, int kchunk,
                                                           float* part) {
  __shared__ float red[4][kGvMaxM][kGvCols];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.x * kGvCols + 8 * lane;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = k0 + kchunk < g.K ? k0 + kchunk : g.K;
  const bool colok = n < g.N;                 // N % 8 == 0: all 8 or none
  float acc[kGvMaxM][8];
#pragma unroll
  for (int m = 0; m < kGvMaxM; ++m)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[m][j] = 0.0f;
  // k in order per wave; the unrolled rows' loads are in flight together
#pragma unroll 8
  for (int k = k0 + w; k < k1; k += 4) {
    const uint4 u = colok ? *reinterpret_cast<const uint4*>(
                                g.B + static_cast<int64_t>(k) * g.ldb + n)
                          : make_uint4(0, 0, 0, 0);
    float bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bv[j] = bf16_to_f32(half_of(u, j));
#pragma unroll
    for (int m = 0; m < kGvMaxM; ++m) {
      if (m < g.M) {
        const float av = bf16_to_f32(g.A[static_cast<int64_t>(m) * g.lda + k]);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[m][j] += av * bv[j];
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kGvMaxM; ++m)
    if (m < g.M)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[w][m][8 * lane + j] = acc[m][j];
  __syncthreads();
  for (int l = threadIdx.x; l < g.M * kGvCols; l += 256) {
    const int m = l / kGvCols, c = l % kGvCols;
    const int nn = blockIdx.x * kGvCols + c;
    if (nn < g.N)
      part[(static_cast<int64_t>(blockIdx.y) * g.M + m) * g.N + nn] =
          (red[0][m][c] + red[1][m][c]) + (red[2][m][c] + red[3][m][c]);
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemv_finish_kernel(GemmArgs g, int splits,
                                                          const float* part) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= g.M * g.N) return;
  const int m = l / g.N, n = l % g.N;
  float x = 0.0f;
#pragma unroll 8
  for (int sp = 0; sp < splits; ++sp) x += part[(static_cast<int64_t>(sp) * g.M + m) * g.N + n];
  epilogue<EPI>(g, m, n, x);
}

// C = A B (A rows m, B rows k): the split-K path for M <= kGvMaxM.
template <int EPI>
int gemv(const GemmArgs& g, float* part, hipStream_t s) {
  const int splits = gemv_splits(g.K);
  const int kchunk = (g.K + splits - 1) / splits;
  const dim3 grid((g.N + kGvCols - 1) / kGvCols, splits);
  hipLaunchKernelGGL(gemv_partial_kernel, grid, dim3(256), 0, s, g, kchunk, part);
  RT_LAUNCH_CHECK("mlp gemv");
  hipLaunchKernelGGL(gemv_finish_kernel<EPI>, dim3((g.M * g.N + 255) / 256), dim3(256), 0,
                     s, g, splits, part);
  RT_LAUNCH_CHECK("mlp gemv finish");
  return kOk;
}

// Per core: ||G|| and x = bf16(G / ||G||).
__global__ __launch_bounds__(256) void mlp_prep_kernel(const float* G, int d0,
                                                       uint16_t* X, float* norms) {
  __shared__ double red[4];
  const int b = blockIdx.x, t = threadIdx.x;
  const float* g = G + static_cast<int64_t>(b) * d0;
  double s = 0.0;
  for (int i = t; i < d0; i += 256) s += static_cast<double>(g[i]) * g[i];
  s = block_sum(s, red);
  const float nrm = static_cast<float>(sqrt(s));
  const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
  for (int i = t; i < d0; i += 256)
    X[static_cast<int64_t>(b) * d0 + i] = f32_to_bf16_rne(g[i] * inv);
  if (t == 0) norms[b] = nrm;
}

struct LossArgs {
  const float* G;      // batch x d0 (unnormalized cores)
  const float* norms;  // batch
  const float* Y;      // batch x d3 (network output)
  float* dY;           // batch x d3, dL/dy / batch
  uint16_t* dYb;       // BF16 copy
  float* loss;         // batch (per-core loss)
  int d0, d3, R, B;
  int n0, n1, n2;      // core dims (order 3)
};

// CP loss of one normalized core and its gradient (eq. (5) on the core),
// one workgroup per core; FP32.
__global__ __launch_bounds__(256) void mlp_loss_kernel(LossArgs a) {
  extern __shared__ __align__(16) float sm[];
  const int b = blockIdx.x, t = threadIdx.x;
  const int R = a.R, n0 = a.n0, n1 = a.n1, n2 = a.n2;
  float* gh = sm;                        // core, n0 x n1 x n2
  float* T = gh + a.d0;                  // n0 x max(n1, n2) x R
  float* V0 = T + n0 * (n1 > n2 ? n1 : n2) * R;
  float* V1 = V0 + n0 * R;
  float* V2 = V1 + n1 * R;
  float* Gm = V2 + n2 * R;               // 3 x R x R
  float* H = Gm + 3 * R * R;             // (n0 + n1 + n2) x R
  __shared__ double red[4];
  const float inv = a.norms[b] > 0.0f ? 1.0f / a.norms[b] : 0.0f;
  const float* gb = a.G + static_cast<int64_t>(b) * a.d0;
  const float* yb = a.Y + static_cast<int64_t>(b) * a.d3;
  double gsq = 0.0;
  for (int i = t; i < a.d0; i += 256) {
    const float x = gb[i] * inv;
    gh[i] = x;
    gsq += static_cast<double>(x) * x;
  }
  for (int i = t; i < (n0 + n1 + n2) * R; i += 256) V0[i] = yb[i];
  __syncthreads();
  const float* Vs[3] = {V0, V1, V2};
  const int ns[3] = {n0, n1, n2};
  for (int l = t; l < 3 * R * R; l += 256) {
    const int n = l / (R * R), i = (l / R) % R, j = l % R;
    float s = 0.0f;
    for (int q = 0; q < ns[n]; ++q) s += Vs[n][q * R + i] * Vs[n][q * R + j];
    Gm[l] = s;
  }
  // T[j0, j1, r] = sum_j2 G[j0, j1, j2] V2[j2, r]
  for (int l = t; l < n0 * n1 * R; l += 256) {
    const int r = l % R, j01 = l / R;
    float s = 0.0f;
    for (int j2 = 0; j2 < n2; ++j2) s += gh[j01 * n2 + j2] * V2[j2 * R + r];
    T[l] = s;
  }
  __syncthreads();
  float* H0 = H;
  float* H1 = H0 + n0 * R;
  float* H2 = H1 + n1 * R;
  for (int l = t; l < n0 * R; l += 256) {   // H0[j0, r] = sum_j1 T[j0, j1, r] V1[j1, r]
    const int j0 = l / R, r = l % R;
    float s = 0.0f;
    for (int j1 = 0; j1 < n1; ++j1) s += T[(j0 * n1 + j1) * R + r] * V1[j1 * R + r];
    H0[l] = s;
  }
  for (int l = t; l < n1 * R; l += 256) {   // H1[j1, r] = sum_j0 T[j0, j1, r] V0[j0, r]
    const int j1 = l / R, r = l % R;
    float s = 0.0f;
    for (int j0 = 0; j0 < n0; ++j0) s += T[(j0 * n1 + j1) * R + r] * V0[j0 * R + r];
    H1[l] = s;
  }
  __syncthreads();
  // T[j0, j2, r] = sum_j1 G[j0, j1, j2] V1[j1, r]
  for (int l = t; l < n0 * n2 * R; l += 256) {
    const int r = l % R, j02 = l / R, j0 = j02 / n2, j2 = j02 % n2;
    float s = 0.0f;
    for (int j1 = 0; j1 < n1; ++j1) s += gh[(j0 * n1 + j1) * n2 + j2] * V1[j1 * R + r];
    T[l] = s;
  }
  __syncthreads();
  for (int l = t; l < n2 * R; l += 256) {   // H2[j2, r] = sum_j0 T[j0, j2, r] V0[j0, r]
    const int j2 = l / R, r = l % R;
    float s = 0.0f;
    for (int j0 = 0; j0 < n0; ++j0) s += T[(j0 * n2 + j2) * R + r] * V0[j0 * R + r];
    H2[l] = s;
  }
  __syncthreads();
  // loss = ||Ghat||^2 - 2 <H0, V0> + 1^T (had Gram) 1
  double p = 0.0;
  for (int l = t; l < n0 * R; l += 256) p += static_cast<double>(H0[l]) * V0[l];
  for (int l = t; l < R * R; l += 256)
    p -= 0.5 * static_cast<double>(Gm[l]) * Gm[R * R + l] * Gm[2 * R * R + l];
  const double gs = block_sum(gsq, red);
  const double ps = block_sum(p, red);
  if (t == 0) a.loss[b] = static_cast<float>(gs - 2.0 * ps);
  // dV_n = 2 (V_n T_n - H_n) / B, T_n = hadamard of the other Grams
  const float scale = 2.0f / static_cast<float>(a.B);
  const float* Hs[3] = {H0, H1, H2};
  int off = 0;
  for (int n = 0; n < 3; ++n) {
    const float* Ga = Gm + (n == 0 ? 1 : 0) * R * R;
    const float* Gb2 = Gm + (n == 2 ? 1 : 2) * R * R;
    for (int l = t; l < ns[n] * R; l += 256) {
      const int j = l / R, r = l % R;
      float s = 0.0f;
      for (int q = 0; q < R; ++q) s += Vs[n][j * R + q] * (Ga[q * R + r] * Gb2[q * R + r]);
      const float d = scale * (s - Hs[n][l]);
      const int64_t o = static_cast<int64_t>(b) * a.d3 + off + l;
      a.dY[o] = d;
      a.dYb[o] = f32_to_bf16_rne(d);
    }
    off += ns[n] * R;
  }
}

// db[n] = sum_b dZ[b][n]
__global__ void colsum_kernel(const float* dZ, int B, int N, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += dZ[static_cast<int64_t>(b) * N + n];
  db[n] = s;
}

// Adam (Kingma & Ba, bias-corrected) on FP32 master values; optional BF16
// copy of the updated values.
__global__ void adam_kernel(float* w, float* m, float* v, const float* g, int64_t n,
                            float lr, float c1, float c2, uint16_t* wb) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float wi = w[i] - lr * mh / (sqrtf(vh) + 1e-8f);
  w[i] = wi;
  if (wb) wb[i] = f32_to_bf16_rne(wi);
}

__global__ void to_bf16_kernel(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f32_to_bf16_rne(x[i]);
}

// V_out[b][i] = y[b][i] * ||G_b||^(1/N)
__global__ void scale_out_kernel(const float* Y, const float* norms, int d3, int N,
                                 int B, float* V) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(B) * d3) return;
  const int b = static_cast<int>(i / d3);
  V[i] = Y[i] * powf(norms[b], 1.0f / static_cast<float>(N));
}

struct MlpDims {
  int B, N, R, d0, d1, d2, d3;
  int cd[RT_MAX_MODES];
};

int mlp_dims(const rt_mlp_desc* d, MlpDims* m) {
  if (!d) {
    set_error("desc is NULL");
    return kErrInvalid;
  }
  if (d->N != 3) {
    set_error("learned initializer: core order %d (order 3 only)", d->N);
    return kErrUnsupported;
  }
  if (d->batch < 1 || d->R < 1 || d->R > 32 || d->hidden1 < 8 || d->hidden2 < 8 ||
      d->hidden1 % 8 || d->hidden2 % 8) {
    set_error("learned initializer: batch %d, R %d, hidden %d/%d invalid", d->batch, d->R,
              d->hidden1, d->hidden2);
    return kErrInvalid;
  }
  m->B = d->batch;
  m->N = d->N;
  m->R = d->R;
  m->d0 = 1;
  int sum = 0;
  for (int n = 0; n < d->N; ++n) {
    if (d->core_dims[n] < 1 || d->core_dims[n] > 32) {
      set_error("learned initializer: core dim %d outside 1..32", d->core_dims[n]);
      return kErrInvalid;
    }
    m->cd[n] = d->core_dims[n];
    m->d0 *= d->core_dims[n];
    sum += d->core_dims[n];
  }
  m->d1 = d->hidden1;
  m->d2 = d->hidden2;
  m->d3 = d->R * sum;
  if (m->d0 % 8 || m->d3 % 8) {
    set_error("learned initializer: input %d and output %d widths must be multiples of 8",
              m->d0, m->d3);
    return kErrUnsupported;
  }
  return kOk;
}

size_t loss_lds_bytes(const MlpDims& m) {
  const int n0 = m.cd[0], n1 = m.cd[1], n2 = m.cd[2], R = m.R;
  const int64_t f = m.d0 + static_cast<int64_t>(n0) * (n1 > n2 ? n1 : n2) * R +
                    static_cast<int64_t>(n0 + n1 + n2) * R + 3 * R * R +
                    static_cast<int64_t>(n0 + n1 + n2) * R;
  return static_cast<size_t>(f) * 4;
}

struct MlpPlan {
  uint16_t* X;
  float* norms;
  float *Z1, *Z2, *Yo, *dY, *dZ1, *dZ2, *loss;
  uint16_t *H1, *H2, *dYb, *dZ1b, *dZ2b;
  float* part;    // split-K partial sums (few cores)
  float* kpart;   // split-K partial sums of the batch-row products
  float* gW[3];
  float* gb[3];
  size_t plan(const MlpDims& m, void* ws, bool grads) {
    Arena ar(ws);
    const int64_t B = m.B;
    X = ar.take<uint16_t>(B * m.d0);
    norms = ar.take<float>(B);
    Z1 = ar.take<float>(B * m.d1);
    Z2 = ar.take<float>(B * m.d2);
    H1 = ar.take<uint16_t>(B * m.d1);
    H2 = ar.take<uint16_t>(B * m.d2);
    Yo = ar.take<float>(B * m.d3);
    dY = ar.take<float>(B * m.d3);
    dYb = ar.take<uint16_t>(B * m.d3);
    dZ1 = ar.take<float>(B * m.d1);
    dZ2 = ar.take<float>(B * m.d2);
    dZ1b = ar.take<uint16_t>(B * m.d1);
    dZ2b = ar.take<uint16_t>(B * m.d2);
    loss = ar.take<float>(B);
    const int dims[4] = {m.d0, m.d1, m.d2, m.d3};
    part = nullptr;
    if (m.B <= kGvMaxM) {
      int64_t most = 0;
      for (int l = 0; l < 3; ++l) {
        const int64_t e = static_cast<int64_t>(gemv_splits(dims[l])) * m.B * dims[l + 1];
        most = e > most ? e : most;
      }
      part = ar.take<float>(most);
    }
    kpart = nullptr;
    if (part == nullptr) {
      int64_t wmax = m.d1 > m.d2 ? m.d1 : m.d2;
      wmax = wmax > m.d3 ? wmax : m.d3;
      kpart = ar.take<float>(static_cast<int64_t>(kSplitMax) * m.B * wmax);
    }
    for (int l = 0; l < 3; ++l) {
      gW[l] = grads ? ar.take<float>(static_cast<int64_t>(dims[l]) * dims[l + 1]) : nullptr;
      gb[l] = grads ? ar.take<float>(dims[l + 1]) : nullptr;
    }
    return ar.need;
  }
};

int check_params(const rt_mlp_params* p, bool train) {
  if (!p) {
    set_error("params is NULL");
    return kErrInvalid;
  }
  for (int l = 0; l < 3; ++l) {
    if (!p->Wb[l] || !p->b[l] || (train && (!p->W[l] || !p->mW[l] || !p->vW[l] ||
                                           !p->mb[l] || !p->vb[l]))) {
      set_error("params: layer %d pointers missing", l);
      return kErrInvalid;
    }
  }
  return kOk;
}

// Forward pass on the workspace buffers (X and norms filled first).
int forward(const MlpDims& m, const rt_mlp_params* p, const float* G, MlpPlan& P,
            hipStream_t s) {
  hipLaunchKernelGGL(mlp_prep_kernel, dim3(m.B), dim3(256), 0, s, G, m.d0, P.X, P.norms);
  RT_LAUNCH_CHECK("mlp prep");
  // a handful of cores: the weights are streamed once, split over K
  const bool few = P.part != nullptr;
  GemmArgs g{};
  g.M = m.B; g.N = m.d1; g.K = m.d0;
  g.A = P.X; g.lda = m.d0; g.B = p->Wb[0]; g.ldb = m.d1;
  g.C = P.Z1; g.ldc = m.d1; g.Cb = P.H1; g.bias = p->b[0];
  RT_TRY((few ? gemv<kEpiBiasGelu>(g, P.part, s)
              : gemm<false, false, kEpiBiasGelu>(g, s, P.kpart)));
  g.N = m.d2; g.K = m.d1; g.A = P.H1; g.lda = m.d1; g.B = p->Wb[1]; g.ldb = m.d2;
  g.C = P.Z2; g.ldc = m.d2; g.Cb = P.H2; g.bias = p->b[1];
  RT_TRY((few ? gemv<kEpiBiasGelu>(g, P.part, s)
              : gemm<false, false, kEpiBiasGelu>(g, s, P.kpart)));
  g.N = m.d3; g.K = m.d2; g.A = P.H2; g.lda = m.d2; g.B = p->Wb[2]; g.ldb = m.d3;
  g.C = P.Yo; g.ldc = m.d3; g.Cb = nullptr; g.bias = p->b[2];
  RT_TRY((few ? gemv<kEpiBias>(g, P.part, s) : gemm<false, false, kEpiBias>(g, s, P.kpart)));
  return kOk;
}

// Loss and gradients into P.gW / P.gb (FP32).
int backward(const MlpDims& m, const rt_mlp_params* p, const float* G, MlpPlan& P,
             float* const* gW, float* const* gb, hipStream_t s) {
  LossArgs la{};
  la.G = G; la.norms = P.norms; la.Y = P.Yo; la.dY = P.dY; la.dYb = P.dYb;
  la.loss = P.loss; la.d0 = m.d0; la.d3 = m.d3; la.R = m.R; la.B = m.B;
  la.n0 = m.cd[0]; la.n1 = m.cd[1]; la.n2 = m.cd[2];
  const size_t lds = loss_lds_bytes(m);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mlp_loss_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return hip_fail(e, "mlp loss LDS attribute");
  }
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(m.B), dim3(256), lds, s, la);
  RT_LAUNCH_CHECK("mlp loss");
  GemmArgs g{};
  // layer 3: gW3 = H2^T dY, gb3 = colsum(dY), dZ2 = (dY W3^T) * gelu'(Z2)
  g.M = m.d2; g.N = m.d3; g.K = m.B;
  g.A = P.H2; g.lda = m.d2; g.B = P.dYb; g.ldb = m.d3; g.C = gW[2]; g.ldc = m.d3;
  RT_TRY((gemm<true, false, kEpiStore>(g, s)));
  hipLaunchKernelGGL(colsum_kernel, dim3((m.d3 + 255) / 256), dim3(256), 0, s, P.dY, m.B,
                     m.d3, gb[2]);
  RT_LAUNCH_CHECK("mlp colsum");
  g = GemmArgs{};
  g.M = m.B; g.N = m.d2; g.K = m.d3;
  g.A = P.dYb; g.lda = m.d3; g.B = p->Wb[2]; g.ldb = m.d3; g.C = P.dZ2; g.ldc = m.d2;
  g.Cb = P.dZ2b; g.Zin = P.Z2;
  RT_TRY((gemm<false, true, kEpiDGelu>(g, s, P.kpart)));
  // layer 2
  g = GemmArgs{};
  g.M = m.d1; g.N = m.d2; g.K = m.B;
  g.A = P.H1; g.lda = m.d1; g.B = P.dZ2b; g.ldb = m.d2; g.C = gW[1]; g.ldc = m.d2;
  RT_TRY((gemm<true, false, kEpiStore>(g, s)));
  hipLaunchKernelGGL(colsum_kernel, dim3((m.d2 + 255) / 256), dim3(256), 0, s, P.dZ2, m.B,
                     m.d2, gb[1]);
  RT_LAUNCH_CHECK("mlp colsum");
  g = GemmArgs{};
  g.M = m.B; g.N = m.d1; g.K = m.d2;
  g.A = P.dZ2b; g.lda = m.d2; g.B = p->Wb[1]; g.ldb = m.d2; g.C = P.dZ1; g.ldc = m.d1;
  g.Cb = P.dZ1b; g.Zin = P.Z1;
  RT_TRY((gemm<false, true, kEpiDGelu>(g, s, P.kpart)));
  // layer 1
  g = GemmArgs{};
  g.M = m.d0; g.N = m.d1; g.K = m.B;
  g.A = P.X; g.lda = m.d0; g.B = P.dZ1b; g.ldb = m.d1; g.C = gW[0]; g.ldc = m.d1;
  RT_TRY((gemm<true, false, kEpiStore>(g, s)));
  hipLaunchKernelGGL(colsum_kernel, dim3((m.d1 + 255) / 256), dim3(256), 0, s, P.dZ1, m.B,
                     m.d1, gb[0]);
  RT_LAUNCH_CHECK("mlp colsum");
  return kOk;
}

int mlp_setup(const rt_mlp_desc* desc, const rt_mlp_params* p, const void* G, void* ws,
              size_t ws_bytes, bool train, MlpDims* m, MlpPlan* P) {
  RT_TRY(mlp_dims(desc, m));
  RT_TRY(check_params(p, train));
  if (!G || !ws) {
    set_error("G and ws must not be NULL");
    return kErrInvalid;
  }
  const size_t need = P->plan(*m, ws, train);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  if (loss_lds_bytes(*m) > 160 * 1024 - 64) {
    set_error("learned initializer: core too large for one workgroup");
    return kErrUnsupported;
  }
  return kOk;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_mlp_workspace(const rt_mlp_desc* desc, size_t* bytes) {
  MlpDims m;
  RT_TRY(mlp_dims(desc, &m));
  if (!bytes) {
    set_error("bytes is NULL");
    return kErrInvalid;
  }
  MlpPlan P;
  *bytes = P.plan(m, nullptr, true);
  return kOk;
}

int rt_mlp_sync_bf16(const rt_mlp_desc* desc, const rt_mlp_params* p, void* stream) {
  MlpDims m;
  RT_TRY(mlp_dims(desc, &m));
  RT_TRY(check_params(p, false));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dims[4] = {m.d0, m.d1, m.d2, m.d3};
  for (int l = 0; l < 3; ++l) {
    if (!p->W[l]) {
      set_error("params: W[%d] missing", l);
      return kErrInvalid;
    }
    const int64_t n = static_cast<int64_t>(dims[l]) * dims[l + 1];
    hipLaunchKernelGGL(to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p->W[l],
                       p->Wb[l], n);
    RT_LAUNCH_CHECK("mlp bf16 copy");
  }
  return kOk;
}

int rt_mlp_forward(const rt_mlp_desc* desc, const rt_mlp_params* p, const float* G,
                   float* V, void* ws, size_t ws_bytes, void* stream) {
  MlpDims m;
  MlpPlan P;
  RT_TRY(mlp_setup(desc, p, G, ws, ws_bytes, false, &m, &P));
  if (!V) {
    set_error("V is NULL");
    return kErrInvalid;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RT_TRY(forward(m, p, G, P, s));
  const int64_t n = static_cast<int64_t>(m.B) * m.d3;
  hipLaunchKernelGGL(scale_out_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P.Yo,
                     P.norms, m.d3, m.N, m.B, V);
  RT_LAUNCH_CHECK("mlp scale");
  return kOk;
}

int rt_mlp_grad(const rt_mlp_desc* desc, const rt_mlp_params* p, const float* G,
                float* const* gW, float* const* gb, float* loss, void* ws,
                size_t ws_bytes, void* stream) {
  MlpDims m;
  MlpPlan P;
  RT_TRY(mlp_setup(desc, p, G, ws, ws_bytes, false, &m, &P));
  if (!gW || !gb || !loss) {
    set_error("gW, gb and loss must not be NULL");
    return kErrInvalid;
  }
  for (int l = 0; l < 3; ++l)
    if (!gW[l] || !gb[l]) {
      set_error("gW[%d] / gb[%d] is NULL", l, l);
      return kErrInvalid;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RT_TRY(forward(m, p, G, P, s));
  RT_TRY(backward(m, p, G, P, gW, gb, s));
  if (hipMemcpyAsync(loss, P.loss, m.B * sizeof(float), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return hip_fail(hipGetLastError(), "loss copy");
  return kOk;
}

int rt_mlp_train_step(const rt_mlp_desc* desc, const rt_mlp_params* p, const float* G,
                      float lr, int32_t step, float* loss, void* ws, size_t ws_bytes,
                      void* stream) {
  MlpDims m;
  MlpPlan P;
  RT_TRY(mlp_setup(desc, p, G, ws, ws_bytes, true, &m, &P));
  if (step < 1 || !(lr > 0.0f)) {
    set_error("train step: step %d must be >= 1 and lr > 0", step);
    return kErrInvalid;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RT_TRY(forward(m, p, G, P, s));
  RT_TRY(backward(m, p, G, P, P.gW, P.gb, s));
  const float c1 = 1.0f - powf(0.9f, static_cast<float>(step));
  const float c2 = 1.0f - powf(0.999f, static_cast<float>(step));
  const int dims[4] = {m.d0, m.d1, m.d2, m.d3};
  for (int l = 0; l < 3; ++l) {
    const int64_t nw = static_cast<int64_t>(dims[l]) * dims[l + 1];
    hipLaunchKernelGGL(adam_kernel, dim3((nw + 255) / 256), dim3(256), 0, s, p->W[l],
                       p->mW[l], p->vW[l], P.gW[l], nw, lr, c1, c2, p->Wb[l]);
    RT_LAUNCH_CHECK("mlp adam");
    hipLaunchKernelGGL(adam_kernel, dim3((dims[l + 1] + 255) / 256), dim3(256), 0, s,
                       p->b[l], p->mb[l], p->vb[l], P.gb[l],
                       static_cast<int64_t>(dims[l + 1]), lr, c1, c2,
                       static_cast<uint16_t*>(nullptr));
    RT_LAUNCH_CHECK("mlp adam");
  }
  if (loss && hipMemcpyAsync(loss, P.loss, m.B * sizeof(float), hipMemcpyDeviceToDevice,
                             s) != hipSuccess)
    return hip_fail(hipGetLastError(), "loss copy");
  return kOk;
}

}  // extern "C"
