// Generic (any mode, any size) contractions on the vector ALUs: the mode-n
// product Y x_n M^T of eq. (1) / Algorithms 2-3, the sketch product
// Z_n = X_(n) Omega~_n of Algorithm 3, the mode-n Gram matrix of a small
// core, and FP64 norms.  These serve the R~-shrunk intermediates; the
// Y-streaming passes use the MFMA kernels in stream.hip.
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kThreads = 256;

// Rows case (C == 1): out[a, k] = sum_i X[a, i] M[i, k].  A 256-row tile of
// X is staged through LDS in ICH-column chunks (coalesced global reads,
// conflict-free LDS reads with a padded stride); each thread owns one row
// and keeps its KMAX accumulators in registers.
template <typename T, int KMAX, int ICH>
__global__ __launch_bounds__(kThreads) void ttm_rows_kernel(
    const T* __restrict__ X, const T* __restrict__ M, T* __restrict__ out,
    int64_t A, int64_t I, int K) {
  __shared__ T xs[kThreads][ICH + 1];
  __shared__ T ms[ICH][KMAX];
  const int t = threadIdx.x;
  const int64_t a0 = static_cast<int64_t>(blockIdx.x) * kThreads;
  T acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = T(0);
  for (int64_t i0 = 0; i0 < I; i0 += ICH) {
    __syncthreads();
#pragma unroll 16
    for (int e = 0; e < ICH; ++e) {
      int l = e * kThreads + t;
      int row = l / ICH, col = l % ICH;
      int64_t a = a0 + row, i = i0 + col;
      xs[row][col] = (a < A && i < I) ? X[a * I + i] : T(0);
    }
    for (int l = t; l < ICH * KMAX; l += kThreads) {
      int ii = l / KMAX, k = l % KMAX;
      int64_t i = i0 + ii;
      ms[ii][k] = (i < I && k < K) ? M[i * K + k] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < ICH; ++ii) {
      T x = xs[t][ii];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) acc[k] += x * ms[ii][k];
    }
  }
  int64_t a = a0 + t;
  if (a < A) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < K) out[a * K + k] = acc[k];
  }
}

// General case (C >= 2): one thread per (a, c); M staged through LDS.
template <typename T, int KMAX>
__global__ __launch_bounds__(kThreads) void ttm_cols_kernel(
    const T* __restrict__ X, const T* __restrict__ M, T* __restrict__ out,
    int64_t A, int64_t I, int64_t C, int K) {
  constexpr int ICH = 64;
  __shared__ T ms[ICH][KMAX];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const bool live = idx < A * C;
  const int64_t a = live ? idx / C : 0;
  const int64_t c = live ? idx % C : 0;
  const T* xp = X + a * I * C + c;
  T acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = T(0);
  for (int64_t i0 = 0; i0 < I; i0 += ICH) {
    __syncthreads();
    for (int l = threadIdx.x; l < ICH * KMAX; l += kThreads) {
      int ii = l / KMAX, k = l % KMAX;
      int64_t i = i0 + ii;
      ms[ii][k] = (i < I && k < K) ? M[i * K + k] : T(0);
    }
    __syncthreads();
    if (live) {
      const int n = static_cast<int>((I - i0) < ICH ? (I - i0) : ICH);
      // ii in order; the unrolled loads are in flight together
#pragma unroll 8
      for (int ii = 0; ii < n; ++ii) {
        T x = xp[(i0 + ii) * C];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) acc[k] += x * ms[ii][k];
      }
    }
  }
  if (live) {
    T* op = out + a * K * C + c;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < K) op[k * C] = acc[k];
  }
}

template <typename T, int KMAX>
int ttm_dispatch(const T* X, const T* M, T* out, int64_t A, int64_t I,
                 int64_t C, int K, hipStream_t s) {
  if (C == 1) {
    constexpr int ICH = 128 / sizeof(T);
    dim3 grid(static_cast<unsigned>(ceil_div(A, kThreads)));
    hipLaunchKernelGGL((ttm_rows_kernel<T, KMAX, ICH>), grid, dim3(kThreads), 0,
                       s, X, M, out, A, I, K);
  } else {
    dim3 grid(static_cast<unsigned>(ceil_div(A * C, kThreads)));
    hipLaunchKernelGGL((ttm_cols_kernel<T, KMAX>), grid, dim3(kThreads), 0, s,
                       X, M, out, A, I, C, K);
  }
  RT_LAUNCH_CHECK("ttm");
  return kOk;
}

// Z[i, r] = sum_{a, c} X[a, i, c] Om[a*C + c, r]; one thread per (i, r).
template <typename T>
__global__ __launch_bounds__(kThreads) void sketch_z_kernel(
    const T* __restrict__ X, const T* __restrict__ Om, T* __restrict__ Z,
    int64_t A, int64_t I, int64_t C, int R) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= I * R) return;
  const int64_t i = idx / R;
  const int r = static_cast<int>(idx % R);
  T acc = T(0);
  for (int64_t a = 0; a < A; ++a) {
    const T* xp = X + (a * I + i) * C;
    const T* op = Om + a * C * R + r;
    for (int64_t c = 0; c < C; ++c) acc += xp[c] * op[c * R];
  }
  Z[idx] = acc;
}

// S[i][j] = sum_{a, c} X[a, i, c] X[a, j, c] in FP64.
template <typename T>
__global__ __launch_bounds__(kThreads) void gram_unfold_kernel(
    const T* __restrict__ X, double* __restrict__ S, int64_t A, int I,
    int64_t C) {
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if (idx >= I * I) return;
  const int i = idx / I, j = idx % I;
  double acc = 0.0;
  for (int64_t a = 0; a < A; ++a) {
    const T* xi = X + (a * I + i) * C;
    const T* xj = X + (a * I + j) * C;
    for (int64_t c = 0; c < C; ++c)
      acc += static_cast<double>(xi[c]) * static_cast<double>(xj[c]);
  }
  S[idx] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void matmul_w_kernel(
    const T* __restrict__ Q, const double* __restrict__ W, T* __restrict__ out,
    int64_t I, int K, int J) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= I * J) return;
  const int64_t i = idx / J;
  const int j = static_cast<int>(idx % J);
  double acc = 0.0;
  // k in order; the unrolled loads of a chunk are in flight together
#pragma unroll 8
  for (int k = 0; k < K; ++k) acc += static_cast<double>(Q[i * K + k]) * W[k * J + j];
  out[idx] = static_cast<T>(acc);
}

// the batch: products first, then the FP32 copies of W
template <typename T>
__global__ __launch_bounds__(kThreads) void matmul_w_batch_kernel(MatWBatch<T> b) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < b.first[b.nb]) {
    int m = 0;
    while (m + 1 < b.nb && idx >= b.first[m + 1]) ++m;
    const int64_t e = idx - b.first[m];
    const int J = b.J[m], K = b.K[m];
    const int64_t i = e / J;
    const int j = static_cast<int>(e % J);
    const T* __restrict__ Q = b.Q[m];
    const double* __restrict__ W = b.W[m];
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < K; ++k) acc += static_cast<double>(Q[i * K + k]) * W[k * J + j];
    b.out[m][e] = static_cast<T>(acc);
    return;
  }
  const int64_t w = idx - b.first[b.nb];
  if (w >= b.wfirst[b.nb]) return;
  int m = 0;
  while (m + 1 < b.nb && w >= b.wfirst[m + 1]) ++m;
  const int64_t e = w - b.wfirst[m];
  b.WT[m][e] = static_cast<float>(b.W[m][e]);
}

template <typename T>
__device__ __forceinline__ double sq_val(T x) {
  double d = static_cast<double>(x);
  return d * d;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void norm2_kernel(
    const T* __restrict__ X, int64_t n, double* __restrict__ partial,
    int32_t* __restrict__ nonfinite) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int bad = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
       i < n; i += stride) {
    double d = static_cast<double>(X[i]);
    bad |= !isfinite(d);
    acc += d * d;
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  if (bad) atomicOr(nonfinite, 1);  // integer flag: order-independent
}

__global__ __launch_bounds__(kThreads) void norm2_bf16_kernel(
    const uint16_t* __restrict__ X, int64_t n, double* __restrict__ partial,
    int32_t* __restrict__ nonfinite) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int bad = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
       i < n; i += stride) {
    double d = static_cast<double>(bf16_to_f32(X[i]));
    bad |= !isfinite(d);
    acc += d * d;
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  if (bad) atomicOr(nonfinite, 1);
}

__global__ void sum_partials_kernel(const double* __restrict__ partial, int nb,
                                    double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += partial[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void convert_kernel(
    const Tin* __restrict__ in, Tout* __restrict__ out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) out[i] = static_cast<Tout>(in[i]);
}

__global__ void sum_partials_checked_kernel(const double* __restrict__ partial,
                                            int nb, double* __restrict__ out,
                                            int32_t* __restrict__ nonfinite) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += partial[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) {
    out[0] = s;
    if (!isfinite(s) && nonfinite) nonfinite[0] = 1;
  }
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

struct GramPtrs {
  const double* g[8];
};

__global__ void cp_fit_final_kernel(const float* __restrict__ X, int N, int R,
                                    const float* __restrict__ lambda,
                                    GramPtrs gp, const double* __restrict__ scal,
                                    double* __restrict__ out3) {
  __shared__ double red[kThreads / 64];
  int64_t stride = 0, pw = 1;
  for (int p = 0; p < N; ++p) {
    stride += pw;
    pw *= R;
  }
  double inner = 0.0;
  for (int r = threadIdx.x; r < R; r += kThreads) {
    const double lr = lambda ? static_cast<double>(lambda[r]) : 1.0;
    inner += lr * static_cast<double>(X[r * stride]);
  }
  inner = block_sum(inner, red);
  double yh = 0.0;
  for (int l = threadIdx.x; l < R * R; l += kThreads) {
    const int r = l / R, q = l % R;
    double v = lambda ? static_cast<double>(lambda[r]) * lambda[q] : 1.0;
    for (int p = 0; p < N; ++p) v *= gp.g[p][l];
    yh += v;
  }
  yh = block_sum(yh, red);
  if (threadIdx.x == 0) {
    const double y2 = scal[0];
    double res2 = y2 - 2.0 * inner + yh;
    res2 = res2 > 0.0 ? res2 : 0.0;
    out3[0] = 1.0 - sqrt(res2) / sqrt(y2);
    out3[1] = y2;
    out3[2] = inner;
  }
}

}  // namespace

int launch_sum_partials(const double* partial, int nb, double* out,
                        int32_t* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_checked_kernel, dim3(1), dim3(kThreads), 0, s,
                     partial, nb, out, nonfinite);
  RT_LAUNCH_CHECK("sum_partials");
  return kOk;
}

int launch_fill_i32(int32_t* p, int32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(ceil_div(n, kThreads))),
                     dim3(kThreads), 0, s, p, value, n);
  RT_LAUNCH_CHECK("fill");
  return kOk;
}

int launch_cp_fit_final(const float* X, int N, int R, const float* lambda,
                        double* const* grams, const double* scal, double* out3,
                        hipStream_t s) {
  GramPtrs gp{};
  for (int p = 0; p < N; ++p) gp.g[p] = grams[p];
  hipLaunchKernelGGL(cp_fit_final_kernel, dim3(1), dim3(kThreads), 0, s, X, N, R,
                     lambda, gp, scal, out3);
  RT_LAUNCH_CHECK("cp_fit_final");
  return kOk;
}

template <typename T>
int launch_ttm(const T* X, const T* M, T* out, int64_t A, int64_t I, int64_t C,
               int K, hipStream_t s) {
  if (A <= 0 || I <= 0 || C <= 0 || K <= 0) return kOk;
  if (K <= 8) return ttm_dispatch<T, 8>(X, M, out, A, I, C, K, s);
  if (K <= 16) return ttm_dispatch<T, 16>(X, M, out, A, I, C, K, s);
  if (K <= 32) return ttm_dispatch<T, 32>(X, M, out, A, I, C, K, s);
  if (K <= 64) return ttm_dispatch<T, 64>(X, M, out, A, I, C, K, s);
  set_error("ttm: K=%d exceeds 64", K);
  return kErrUnsupported;
}

template <typename T>
int launch_sketch_z(const T* X, const T* Om, T* Z, int64_t A, int64_t I,
                    int64_t C, int R, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(I * R, kThreads)));
  hipLaunchKernelGGL(sketch_z_kernel<T>, grid, dim3(kThreads), 0, s, X, Om, Z,
                     A, I, C, R);
  RT_LAUNCH_CHECK("sketch_z");
  return kOk;
}

template <typename T>
int launch_gram_unfold(const T* X, double* S, int64_t A, int I, int64_t C,
                       hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(static_cast<int64_t>(I) * I, kThreads)));
  hipLaunchKernelGGL(gram_unfold_kernel<T>, grid, dim3(kThreads), 0, s, X, S, A,
                     I, C);
  RT_LAUNCH_CHECK("gram_unfold");
  return kOk;
}

template <typename T>
int launch_matmul_w(const T* Q, const double* W, T* out, int64_t I, int K,
                    int J, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(I * J, kThreads)));
  hipLaunchKernelGGL(matmul_w_kernel<T>, grid, dim3(kThreads), 0, s, Q, W, out,
                     I, K, J);
  RT_LAUNCH_CHECK("matmul_w");
  return kOk;
}

template <typename T>
int launch_matmul_w_batch(const MatWBatch<T>& b, hipStream_t s) {
  if (b.nb < 1 || b.nb > kBatchModes) {
    set_error("matmul_w batch of %d modes", b.nb);
    return kErrUnsupported;
  }
  const int64_t total = b.first[b.nb] + b.wfirst[b.nb];
  if (total <= 0) return kOk;
  hipLaunchKernelGGL(matmul_w_batch_kernel<T>,
                     dim3(static_cast<unsigned>(ceil_div(total, kThreads))), dim3(kThreads),
                     0, s, b);
  RT_LAUNCH_CHECK("matmul_w_batch");
  return kOk;
}

int norm2_blocks() { return 1024; }

template <typename T>
int launch_norm2(const T* X, int64_t n, double* partial, int nblocks,
                 double* out, int32_t* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel<T>, dim3(nblocks), dim3(kThreads), 0, s, X, n,
                     partial, nonfinite);
  RT_LAUNCH_CHECK("norm2");
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kThreads), 0, s, partial,
                     nblocks, out);
  RT_LAUNCH_CHECK("norm2 sum");
  return kOk;
}

int launch_norm2_bf16(const uint16_t* X, int64_t n, double* partial,
                      int nblocks, double* out, int32_t* nonfinite,
                      hipStream_t s) {
  hipLaunchKernelGGL(norm2_bf16_kernel, dim3(nblocks), dim3(kThreads), 0, s, X,
                     n, partial, nonfinite);
  RT_LAUNCH_CHECK("norm2_bf16");
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kThreads), 0, s, partial,
                     nblocks, out);
  RT_LAUNCH_CHECK("norm2 sum");
  return kOk;
}

template <typename Tin, typename Tout>
int launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t s) {
  if (n <= 0) return kOk;
  hipLaunchKernelGGL((convert_kernel<Tin, Tout>),
                     dim3(static_cast<unsigned>(ceil_div(n, kThreads))),
                     dim3(kThreads), 0, s, in, out, n);
  RT_LAUNCH_CHECK("convert");
  return kOk;
}

#define RT_INST(T)                                                             \
  template int launch_ttm<T>(const T*, const T*, T*, int64_t, int64_t,         \
                             int64_t, int, hipStream_t);                        \
  template int launch_sketch_z<T>(const T*, const T*, T*, int64_t, int64_t,    \
                                  int64_t, int, hipStream_t);                   \
  template int launch_gram_unfold<T>(const T*, double*, int64_t, int, int64_t, \
                                     hipStream_t);                              \
  template int launch_matmul_w<T>(const T*, const double*, T*, int64_t, int,   \
                                  int, hipStream_t);                            \
  template int launch_matmul_w_batch<T>(const MatWBatch<T>&, hipStream_t);      \
  template int launch_norm2<T>(const T*, int64_t, double*, int, double*,       \
                               int32_t*, hipStream_t);
RT_INST(float)
RT_INST(double)
#undef RT_INST

template int launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template int launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);

}  // namespace rt
