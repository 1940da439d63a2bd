// Sketch products Z_n = X_(n) Omega~_n of Algorithm 3 computed from the streamed
// intermediates without forming X_n.
//
// With T = Y x_{p in S} B_p^T the streamed intermediate (S = the modes one
// pass contracted: {N} for TA, {N-1} for TB), the sketch of mode n is
//     Z_n = X_(n) Omega~_n,   X_n = T x_{p not in S, p != n} B_p^T,
// i.e. Z_n[i, r] = sum_{a, c} T[a, i, c] W_n[a, c, r]  with T viewed as
// [A, I_n, C] and W_n = Omega~_n (reshaped over (j_p)_{p != n}) expanded in
// every mode p not in S, p != n, by B_p (K_p -> I_p).  W_n is small (the
// random test matrix of Section IV-A step 1 in Kronecker-structured form),
// so each sketch is one split-K product instead of a chain of mode products.
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kThreads = 256;

// out[a, i, c] = sum_j B[i, j] X[a, j, c]; one thread per output (J <= 64).
// out[a, i, c] = sum_j B[i, j] X[a, j, c] (the expansion of a test matrix by
// a factor).  Each thread produces kExpRows rows i of one column c, so every
// X value it loads serves kExpRows products (X is read once per block of
// rows, not once per row); the block's B rows sit in LDS.  The sum runs over
// j in order, as a plain loop would.
constexpr int kExpRows = 8;
constexpr int kExpMaxJ = 64;

template <typename T>
__global__ __launch_bounds__(kThreads) void expand_kernel(
    const T* __restrict__ X, const T* __restrict__ B, T* __restrict__ out,
    int64_t A, int64_t I, int J, int64_t C) {
  __shared__ T bs[kExpRows][kExpMaxJ];
  const int64_t c = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const int64_t nib = (I + kExpRows - 1) / kExpRows;
  // row blocks and a strided over the grid (block-uniform trip counts, so
  // every thread reaches the barriers)
  for (int64_t ib = blockIdx.y; ib < nib; ib += gridDim.y) {
    const int64_t i0 = ib * kExpRows;
    __syncthreads();   // the previous block's rows are no longer read
    for (int l = threadIdx.x; l < kExpRows * J; l += kThreads) {
      const int u = l / J, j = l - u * J;
      bs[u][j] = (i0 + u < I) ? B[(i0 + u) * J + j] : T(0);
    }
    __syncthreads();
    if (c >= C) continue;
    for (int64_t a = blockIdx.z; a < A; a += gridDim.z) {
      const T* xp = X + a * J * C + c;
      T acc[kExpRows];
#pragma unroll
      for (int u = 0; u < kExpRows; ++u) acc[u] = T(0);
      // eight X loads in flight at a time, then their products (j in order)
      int j = 0;
      for (; j + 8 <= J; j += 8) {
        T x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = xp[static_cast<int64_t>(j + q) * C];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
          for (int u = 0; u < kExpRows; ++u) acc[u] += bs[u][j + q] * x[q];
      }
      for (; j < J; ++j) {
        const T x = xp[static_cast<int64_t>(j) * C];
#pragma unroll
        for (int u = 0; u < kExpRows; ++u) acc[u] += bs[u][j] * x;
      }
#pragma unroll
      for (int u = 0; u < kExpRows; ++u)
        if (i0 + u < I) out[(a * I + i0 + u) * C + c] = acc[u];
    }
  }
}

// Split-K product part[s][i][r] = sum over the s-th range of k = a*C + c of
// T[a, i, c] W[k, r].  Tile: 64 rows i x RT (<= 32 or 64) columns r, k in
// chunks of 32 staged through LDS.  Loads are coalesced along c (C > 1) or
// along i (C == 1).
template <typename T, int RT>
__global__ __launch_bounds__(kThreads) void sketch_gemm_kernel(
    const T* __restrict__ Tm, const T* __restrict__ W, T* __restrict__ part,
    int64_t A, int64_t I, int64_t C, int R, int64_t kper) {
  constexpr int BI = 64, BK = 32;
  __shared__ T ts[BK][BI + 1];
  __shared__ T ws[BK][RT];
  const int t = threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * BI;
  const int64_t K = A * C;
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kper;
  const int64_t k1 = (k0 + kper < K) ? k0 + kper : K;
  // thread -> (row group, column group): 64 rows x RT cols over 256 threads
  constexpr int CPT = RT / 4;  // columns per thread
  const int ti = t & 63;       // row within tile
  const int tc = t >> 6;       // column group 0..3
  T acc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = T(0);
  for (int64_t kb = k0; kb < k1; kb += BK) {
    __syncthreads();
    // stage T tile [BK x BI]
    for (int l = t; l < BK * BI; l += kThreads) {
      int kk, ii;
      if (C == 1) {       // i contiguous
        kk = l / BI;
        ii = l % BI;
      } else {            // c contiguous
        kk = l % BK;
        ii = l / BK;
      }
      const int64_t k = kb + kk, i = i0 + ii;
      T v = T(0);
      if (k < k1 && i < I) {
        const int64_t a = k / C, c = k % C;
        v = Tm[(a * I + i) * C + c];
      }
      ts[kk][ii] = v;
    }
    for (int l = t; l < BK * RT; l += kThreads) {
      const int kk = l / RT, r = l % RT;
      const int64_t k = kb + kk;
      ws[kk][r] = (k < k1 && r < R) ? W[k * R + r] : T(0);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < BK; ++kk) {
      const T x = ts[kk][ti];
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[q] += x * ws[kk][tc * CPT + q];
    }
  }
  const int64_t i = i0 + ti;
  if (i < I) {
    T* op = part + (static_cast<int64_t>(blockIdx.y) * I + i) * R;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int r = tc * CPT + q;
      if (r < R) op[r] = acc[q];
    }
  }
}

// FP32 form of the split-K sketch product on the matrix cores
// (v_mfma_f32_32x32x2_f32): a workgroup owns 128 rows i (32 per wavefront)
// and all R <= 32 columns r over its range of k; k goes in chunks of 32 staged
// through LDS with the same coalesced loads as above.  Exact FP32 products,
// FP32 accumulation.
typedef float v16f __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(kThreads) void sketch_mfma_kernel(
    const float* __restrict__ Tm, const float* __restrict__ W, float* __restrict__ part,
    int64_t A, int64_t I, int64_t C, int R, int64_t kper) {
  constexpr int BI = 128, BK = 32;
  static_assert(kThreads == 256, "staging maps");
  __shared__ float ts[BK][BI + 1];
  __shared__ float ws[BK][32];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 31, g = lane >> 5;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * BI;
  const int64_t K = A * C;
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kper;
  const int64_t k1 = (k0 + kper < K) ? k0 + kper : K;
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  // stage kb is loaded into registers one stage ahead of its products
  constexpr int kTv = BK * BI / kThreads, kWv = BK * 32 / kThreads;
  float tv[kTv], wv[kWv];
  auto load_stage = [&](int64_t kb) __attribute__((always_inline)) {
    if (C == 1) {
      // rows i contiguous: thread t takes row i0 + t % 128, k = kb + t / 128 + 2m
      const int64_t i = i0 + (t & (BI - 1));
#pragma unroll
      for (int m = 0; m < kTv; ++m) {
        const int64_t k = kb + (t >> 7) + 2 * m;
        tv[m] = (k < k1 && i < I) ? Tm[k * I + i] : 0.0f;
      }
    } else {
      // c contiguous: thread t takes k = kb + t % 32, rows t / 32 + 8m; one
      // division per stage
      const int64_t k = kb + (t & (BK - 1));
      const bool kok = k < k1;
      const int64_t a = kok ? k / C : 0;
      const float* base = Tm + (a * I) * C + (kok ? k - a * C : 0);
#pragma unroll
      for (int m = 0; m < kTv; ++m) {
        const int64_t i = i0 + (t >> 5) + 8 * m;
        tv[m] = (kok && i < I) ? base[i * C] : 0.0f;
      }
    }
#pragma unroll
    for (int m = 0; m < kWv; ++m) {
      const int l = t + kThreads * m;
      const int64_t k = kb + (l >> 5);
      const int r = l & 31;
      wv[m] = (k < k1 && r < R) ? W[k * R + r] : 0.0f;
    }
  };
  if (k0 < k1) load_stage(k0);
  for (int64_t kb = k0; kb < k1; kb += BK) {
    __syncthreads();   // the previous stage's products have read the tiles
    if (C == 1) {
#pragma unroll
      for (int m = 0; m < kTv; ++m) ts[(t >> 7) + 2 * m][t & (BI - 1)] = tv[m];
    } else {
#pragma unroll
      for (int m = 0; m < kTv; ++m) ts[t & (BK - 1)][(t >> 5) + 8 * m] = tv[m];
    }
#pragma unroll
    for (int m = 0; m < kWv; ++m) {
      const int l = t + kThreads * m;
      ws[l >> 5][l & 31] = wv[m];
    }
    __syncthreads();
    if (kb + BK < k1) load_stage(kb + BK);   // in flight during the products
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ts[kk + g][32 * w + lr], ws[kk + g][lr],
                                                 acc, 0, 0, 0);
  }
  // acc[v]: row 8 (v / 4) + 4 g + v % 4 of this wave's 32, column lr
  if (lr < R) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t i = i0 + 32 * w + 8 * (v / 4) + 4 * g + (v % 4);
      if (i < I) part[(static_cast<int64_t>(blockIdx.y) * I + i) * R + lr] = acc[v];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void sum_splits_kernel(
    const T* __restrict__ part, T* __restrict__ out, int64_t n, int S) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= n) return;
  T acc = T(0);
#pragma unroll 8
  for (int s = 0; s < S; ++s) acc += part[s * n + idx];  // fixed order
  out[idx] = acc;
}

// out[a, k, c] = sum_i X[a, i, c] M[i, k] for small C (<= 64) and K (<= 64):
// one workgroup per a; X[a] and M staged through LDS in 64-row chunks; each
// thread owns a 4 (k) x 4 (c) register block of the output.
template <typename T>
__global__ __launch_bounds__(kThreads) void ttm_small_c_kernel(
    const T* __restrict__ X, const T* __restrict__ M, T* __restrict__ out,
    int64_t A, int64_t I, int C, int K) {
  constexpr int BI = 64;
  __shared__ T xs[BI][64];
  __shared__ T ms[BI][64];
  const int t = threadIdx.x;
  const int64_t a = blockIdx.x;
  const int kb = (t >> 4) * 4, cb = (t & 15) * 4;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  const T* xa = X + a * I * C;
  for (int64_t i0 = 0; i0 < I; i0 += BI) {
    __syncthreads();
    const int rows = static_cast<int>((I - i0) < BI ? (I - i0) : BI);
    for (int l = t; l < BI * 64; l += kThreads) {
      const int ii = l >> 6, c = l & 63;
      xs[ii][c] = (ii < rows && c < C) ? xa[(i0 + ii) * C + c] : T(0);
      ms[ii][c] = (ii < rows && c < K) ? M[(i0 + ii) * K + c] : T(0);
    }
    __syncthreads();
    for (int ii = 0; ii < rows; ++ii) {
      T xv[4], mv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        xv[j] = xs[ii][cb + j];
        mv[j] = ms[ii][kb + j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += mv[i] * xv[j];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (kb + i < K && cb + j < C) out[(a * K + kb + i) * C + cb + j] = acc[i][j];
}

// FP32 form of ttm_small_c for C, K <= 32 on the matrix cores: one
// workgroup per a computes the 32 x 32 block out[a] = M^T X[a] with
// v_mfma_f32_32x32x2_f32 (A operand M^T: lane l holds M[i][l % 32]; B
// operand X[a]: lane l holds X[a][i][l % 32]; i = the pair of rows of the
// step, by l / 32).  The four wavefronts take interleaved row pairs and
// their sums meet in LDS in a fixed order.
__global__ __launch_bounds__(kThreads) void ttm_small_mfma_kernel(
    const float* __restrict__ X, const float* __restrict__ M, float* __restrict__ out,
    int64_t A, int64_t I, int C, int K) {
  __shared__ float red[4][32][33];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 31, g = lane >> 5;
  const int64_t a = blockIdx.x;
  const float* xa = X + a * I * C;
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll 8
  for (int64_t i0 = 2 * w; i0 < I; i0 += 8) {
    const int64_t i = i0 + g;
    const float mv = (i < I && lr < K) ? M[i * K + lr] : 0.0f;
    const float xv = (i < I && lr < C) ? xa[i * C + lr] : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(mv, xv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) red[w][8 * (v / 4) + 4 * g + (v % 4)][lr] = acc[v];
  __syncthreads();
  for (int l = t; l < K * C; l += kThreads) {
    const int k = l / C, c = l % C;
    out[(a * K + k) * C + c] = (red[0][k][c] + red[1][k][c]) + (red[2][k][c] + red[3][k][c]);
  }
}

// out[c][r] = in[r][c] for an R x C matrix (tiled through LDS).
template <typename T>
__global__ void transpose_kernel(const T* __restrict__ in, T* __restrict__ out,
                                 int64_t R, int64_t C) {
  __shared__ T tl[32][33];
  const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 32, c0 = static_cast<int64_t>(blockIdx.x) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    tl[j][tx] = (r < R && c < C) ? in[r * C + c] : T(0);
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + j, r = r0 + tx;
    if (r < R && c < C) out[c * R + r] = tl[tx][j];
  }
}

// S = X_(n) X_(n)^T in FP64 for X viewed [A, I, C]; one wavefront per
// entry of the upper triangle (lanes stride the (a, c) pairs).
template <typename T>
__device__ __forceinline__ void gram_wave_entry(const T* __restrict__ X,
                                                double* __restrict__ S, int64_t A,
                                                int I, int64_t C, int pair, int lane) {
  int o = pair, r = 0;
  while (o >= I - r) {
    o -= I - r;
    ++r;
  }
  const int c2 = r + o;
  double acc = 0.0;
  const int64_t n = A * C;
  if (n <= 0x7fffffff && C <= 0x7fffffff) {
    // 32-bit index arithmetic (the usual core-sized case); l in order
    const int n32 = static_cast<int>(n), C32 = static_cast<int>(C);
#pragma unroll 4
    for (int l = lane; l < n32; l += 64) {
      const int a = l / C32, c = l - a * C32;
      acc += static_cast<double>(X[(static_cast<int64_t>(a) * I + r) * C32 + c]) *
             static_cast<double>(X[(static_cast<int64_t>(a) * I + c2) * C32 + c]);
    }
  } else {
    for (int64_t l = lane; l < n; l += 64) {
      const int64_t a = l / C, c = l % C;
      acc += static_cast<double>(X[(a * I + r) * C + c]) *
             static_cast<double>(X[(a * I + c2) * C + c]);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    S[r * I + c2] = acc;
    S[c2 * I + r] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gram_waves_kernel(
    const T* __restrict__ X, double* __restrict__ S, int64_t A, int I, int64_t C) {
  const int pair = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (pair >= I * (I + 1) / 2) return;
  gram_wave_entry(X, S, A, I, C, pair, threadIdx.x & 63);
}

// the batch: the wave's entry picks its mode (uniform per wave)
template <typename T>
__global__ __launch_bounds__(kThreads) void gram_waves_batch_kernel(const T* __restrict__ X,
                                                                    GramWavesBatch b) {
  const int q = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (q >= b.first[b.nb]) return;
  int m = 0;
  while (m + 1 < b.nb && q >= b.first[m + 1]) ++m;
  gram_wave_entry(X, b.S[m], b.A[m], b.I[m], b.C[m], q - b.first[m], threadIdx.x & 63);
}

}  // namespace

template <typename T>
int launch_expand(const T* X, const T* B, T* out, int64_t A, int64_t I, int J,
                  int64_t C, hipStream_t s) {
  if (A <= 0 || I <= 0 || C <= 0) return kOk;
  const int64_t gx = ceil_div(C, kThreads), nib = ceil_div(I, kExpRows);
  if (J > kExpMaxJ || gx > 0x7fffffff) {
    set_error("expand: J %d or C %lld out of range", J, (long long)C);
    return kErrUnsupported;
  }
  hipLaunchKernelGGL(expand_kernel<T>,
                     dim3(static_cast<unsigned>(gx),
                          static_cast<unsigned>(nib < 65535 ? nib : 65535),
                          static_cast<unsigned>(A < 65535 ? A : 65535)),
                     dim3(kThreads), 0, s, X, B, out, A, I, J, C);
  RT_LAUNCH_CHECK("expand");
  return kOk;
}

int64_t sketch_gemm_splits(int64_t I, int64_t K) {
  const int64_t iblocks = ceil_div(I, 64);
  int64_t S = ceil_div(kSketchTargetBlocks, iblocks);
  const int64_t maxS = ceil_div(K, 32);
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  return S;
}

// The split-K partials take Sused * I * R elements of part.
static int check_part(int64_t Sused, int64_t I, int R, int64_t part_cap) {
  if (Sused * I * R > part_cap) {
    set_error("sketch partials need %lld elements, scratch holds %lld",
              static_cast<long long>(Sused * I * R), static_cast<long long>(part_cap));
    return kErrWorkspace;
  }
  return kOk;
}

template <typename T>
int launch_sketch_gemm(const T* Tm, const T* W, T* Z, T* part, int64_t part_cap,
                       int64_t A, int64_t I, int64_t C, int R, hipStream_t s) {
  const int64_t K = A * C;
  const int64_t S = sketch_gemm_splits(I, K);
  int64_t kper = ceil_div(K, S);
  kper = ceil_div(kper, 32) * 32;
  const int64_t Sused = ceil_div(K, kper);
  RT_TRY(check_part(Sused, I, R, part_cap));
  dim3 grid(static_cast<unsigned>(ceil_div(I, 64)), static_cast<unsigned>(Sused));
  if (R <= 32) {
    hipLaunchKernelGGL((sketch_gemm_kernel<T, 32>), grid, dim3(kThreads), 0, s, Tm,
                       W, part, A, I, C, R, kper);
  } else if (R <= 64) {
    hipLaunchKernelGGL((sketch_gemm_kernel<T, 64>), grid, dim3(kThreads), 0, s, Tm,
                       W, part, A, I, C, R, kper);
  } else {
    set_error("sketch width %d exceeds 64", R);
    return kErrUnsupported;
  }
  RT_LAUNCH_CHECK("sketch_gemm");
  const int64_t n = I * R;
  hipLaunchKernelGGL(sum_splits_kernel<T>, dim3(static_cast<unsigned>(ceil_div(n, kThreads))),
                     dim3(kThreads), 0, s, part, Z, n, static_cast<int>(Sused));
  RT_LAUNCH_CHECK("sketch_gemm sum");
  return kOk;
}

// FP32, R <= 32: the matrix-core form (same split-K partials and sum).
template <>
int launch_sketch_gemm<float>(const float* Tm, const float* W, float* Z, float* part,
                              int64_t part_cap, int64_t A, int64_t I, int64_t C, int R,
                              hipStream_t s) {
  if (R > 32) {
    const int64_t K = A * C;
    const int64_t S = sketch_gemm_splits(I, K);
    int64_t kper = ceil_div(ceil_div(K, S), 32) * 32;
    const int64_t Sused = ceil_div(K, kper);
    RT_TRY(check_part(Sused, I, R, part_cap));
    dim3 grid(static_cast<unsigned>(ceil_div(I, 64)), static_cast<unsigned>(Sused));
    if (R > 64) {
      set_error("sketch width %d exceeds 64", R);
      return kErrUnsupported;
    }
    hipLaunchKernelGGL((sketch_gemm_kernel<float, 64>), grid, dim3(kThreads), 0, s, Tm, W,
                       part, A, I, C, R, kper);
    RT_LAUNCH_CHECK("sketch_gemm");
    const int64_t n = I * R;
    hipLaunchKernelGGL(sum_splits_kernel<float>,
                       dim3(static_cast<unsigned>(ceil_div(n, kThreads))), dim3(kThreads),
                       0, s, part, Z, n, static_cast<int>(Sused));
    RT_LAUNCH_CHECK("sketch_gemm sum");
    return kOk;
  }
  const int64_t K = A * C;
  const int64_t S = sketch_gemm_splits(I, K);   // the partial buffer holds S splits
  int64_t kper = ceil_div(ceil_div(K, S), 32) * 32;
  const int64_t Sused = ceil_div(K, kper);
  RT_TRY(check_part(Sused, I, R, part_cap));
  dim3 grid(static_cast<unsigned>(ceil_div(I, 128)), static_cast<unsigned>(Sused));
  hipLaunchKernelGGL(sketch_mfma_kernel, grid, dim3(kThreads), 0, s, Tm, W, part, A, I, C,
                     R, kper);
  RT_LAUNCH_CHECK("sketch_mfma");
  const int64_t n = I * R;
  hipLaunchKernelGGL(sum_splits_kernel<float>,
                     dim3(static_cast<unsigned>(ceil_div(n, kThreads))), dim3(kThreads), 0,
                     s, part, Z, n, static_cast<int>(Sused));
  RT_LAUNCH_CHECK("sketch_mfma sum");
  return kOk;
}

template <typename T>
int launch_transpose(const T* in, T* out, int64_t R, int64_t C, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(C, 32)), static_cast<unsigned>(ceil_div(R, 32)));
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, in, out, R, C);
  RT_LAUNCH_CHECK("transpose");
  return kOk;
}

template <typename T>
int launch_gram_waves(const T* X, double* S, int64_t A, int I, int64_t C,
                      hipStream_t s) {
  const int npairs = I * (I + 1) / 2;
  hipLaunchKernelGGL(gram_waves_kernel<T>, dim3((npairs + 3) / 4), dim3(kThreads), 0,
                     s, X, S, A, I, C);
  RT_LAUNCH_CHECK("gram_waves");
  return kOk;
}

template <typename T>
int launch_gram_waves_batch(const T* X, const GramWavesBatch& b, hipStream_t s) {
  if (b.nb < 1 || b.nb > kBatchModes) {
    set_error("gram batch of %d views", b.nb);
    return kErrUnsupported;
  }
  const int total = b.first[b.nb];
  if (total <= 0) return kOk;
  hipLaunchKernelGGL(gram_waves_batch_kernel<T>, dim3((total + 3) / 4), dim3(kThreads),
                     0, s, X, b);
  RT_LAUNCH_CHECK("gram_waves_batch");
  return kOk;
}

template <typename T>
int launch_ttm_small_c(const T* X, const T* M, T* out, int64_t A, int64_t I,
                       int C, int K, hipStream_t s) {
  if (C > 64 || K > 64) {
    set_error("ttm_small_c: C=%d K=%d unsupported", C, K);
    return kErrUnsupported;
  }
  if constexpr (sizeof(T) == sizeof(float)) {
    if (C <= 32 && K <= 32) {
      hipLaunchKernelGGL(ttm_small_mfma_kernel, dim3(static_cast<unsigned>(A)),
                         dim3(kThreads), 0, s, X, M, out, A, I, C, K);
      RT_LAUNCH_CHECK("ttm_small_mfma");
      return kOk;
    }
  }
  hipLaunchKernelGGL(ttm_small_c_kernel<T>, dim3(static_cast<unsigned>(A)),
                     dim3(kThreads), 0, s, X, M, out, A, I, C, K);
  RT_LAUNCH_CHECK("ttm_small_c");
  return kOk;
}

#define RT_INST(T)                                                              \
  template int launch_expand<T>(const T*, const T*, T*, int64_t, int64_t, int,  \
                                int64_t, hipStream_t);                          \
  template int launch_ttm_small_c<T>(const T*, const T*, T*, int64_t, int64_t,  \
                                     int, int, hipStream_t);                    \
  template int launch_transpose<T>(const T*, T*, int64_t, int64_t, hipStream_t); \
  template int launch_gram_waves<T>(const T*, double*, int64_t, int, int64_t,   \
                                    hipStream_t);                               \
  template int launch_gram_waves_batch<T>(const T*, const GramWavesBatch&,      \
                                          hipStream_t);
RT_INST(float)
RT_INST(double)
#undef RT_INST
template int launch_sketch_gemm<double>(const double*, const double*, double*, double*,
                                        int64_t, int64_t, int64_t, int64_t, int,
                                        hipStream_t);

}  // namespace rt
