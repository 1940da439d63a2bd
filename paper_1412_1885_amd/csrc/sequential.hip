// Sequential RandTucker (Algorithm 2, Section IV-A) with dense Gaussian test
// matrices drawn on the device.
//
// For n = 1..N: Z_n = Y_(n) Omega_n with a dense Gaussian Omega_n whose rows
// run over the other modes' current indices (modes < n already shrunk to
// R~_k), U_n = orth(Z_n) (the same FP64 QR as Algorithm 3's sketches), and
// Y <- Y x_n U_n^T, so the tensor shrinks mode by mode; the last tensor is
// the core.  The first sketch reads Y once and the first projection reads it
// again: two passes over the full tensor, plus the dense Omega_1
// (prod_{k>1} I_k x R~_1: 1e6 x 30 at 1000^3) written and read once.
//
// Test matrices.  Entry (r, k) of Omega_n comes from a counter-based
// generator, so any entry can be produced anywhere from (seed, n, r, k)
// alone (the parameter broadcast Section IV-B describes for generating the
// random matrices where the data lives): Philox4x32 with 10 rounds (Salmon,
// Moraes, Dror, Shaw, SC 2011) on counter (r mod 2^32, r div 2^32, k, n) and
// key (seed mod 2^32, seed div 2^32), then Box-Muller in FP64 on its first
// two words: u1 = (x0 + 1) 2^-32, u2 = (x1 + 1/2) 2^-32,
// value = sqrt(-2 ln u1) cos(2 pi u2).  Each matrix is materialized once and
// consumed by the split-K sketch product of sketch.hip.
#include <cmath>

#include "../../include/rtucker.h"
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kGenThreads = 256;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = static_cast<uint32_t>(p1);
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = static_cast<uint32_t>(p0);
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

// out[r * cols + k] = entry (r, k) of the test matrix of `mode`, r < rows.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void gaussian_fill_kernel(T* out, int64_t rows,
                                                                    int cols, int mode,
                                                                    uint64_t seed) {
  const int64_t total = rows * cols;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kGenThreads;
  for (int64_t l = static_cast<int64_t>(blockIdx.x) * kGenThreads + threadIdx.x; l < total;
       l += stride) {
    const int64_t r = l / cols;
    const int k = static_cast<int>(l - r * cols);
    uint32_t c[4] = {static_cast<uint32_t>(r), static_cast<uint32_t>(r >> 32),
                     static_cast<uint32_t>(k), static_cast<uint32_t>(mode)};
    philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double u1 = (static_cast<double>(c[0]) + 1.0) * 0x1p-32;
    const double u2 = (static_cast<double>(c[1]) + 0.5) * 0x1p-32;
    out[l] = static_cast<T>(sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
  }
}

template <typename T>
int launch_gaussian_fill(T* out, int64_t rows, int cols, int mode, uint64_t seed,
                         hipStream_t s) {
  const int64_t total = rows * cols;
  const int64_t blocks = ceil_div(total, kGenThreads);
  const unsigned grid = static_cast<unsigned>(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(gaussian_fill_kernel<T>, dim3(grid > 0 ? grid : 1), dim3(kGenThreads),
                     0, s, out, rows, cols, mode, seed);
  RT_LAUNCH_CHECK("gaussian fill");
  return kOk;
}

int validate_seq(const rt_sequential_desc* d) {
  if (!d) {
    set_error("desc is NULL");
    return kErrInvalid;
  }
  if (d->N < 2 || d->N > RT_MAX_MODES) {
    set_error("N=%d outside 2..%d", d->N, RT_MAX_MODES);
    return kErrInvalid;
  }
  if (d->precision != RT_F32 && d->precision != RT_F64) {
    set_error("sequential RandTucker runs in RT_F32 or RT_F64 (precision %d)", d->precision);
    return kErrUnsupported;
  }
  int64_t total = 1;
  for (int n = 0; n < d->N; ++n) {
    const int64_t I = d->dims[n];
    const int rt = d->ranks_tilde[n];
    if (I < 1 || rt < 1 || rt > RT_MAX_SKETCH || rt > I) {
      set_error("mode %d: I=%lld, R~=%d (need 1 <= R~ <= min(I, %d))", n, (long long)I, rt,
                RT_MAX_SKETCH);
      return kErrInvalid;
    }
    if (total > (int64_t(1) << 62) / I) {
      set_error("tensor size overflows 64 bits");
      return kErrInvalid;
    }
    total *= I;
  }
  return kOk;
}

template <typename T>
struct SeqPlan {
  int N;
  int64_t I[RT_MAX_MODES];
  int K[RT_MAX_MODES];
  int64_t rows[RT_MAX_MODES];   // rows of Omega_n
  T* Om;
  T* buf[2];
  T* Z;
  double* qrwork;
  T* zpart;
  int64_t zpart_cap;
  int32_t* iflags;
  size_t plan(const rt_sequential_desc* d, void* ws) {
    Arena ar(ws);
    N = d->N;
    int64_t om = 1, big = 1, zmax = 1, qrmax = 1, imax = 1;
    int kmax = 1;
    for (int n = 0; n < N; ++n) {
      I[n] = d->dims[n];
      K[n] = d->ranks_tilde[n];
      imax = I[n] > imax ? I[n] : imax;
      kmax = K[n] > kmax ? K[n] : kmax;
    }
    for (int n = 0; n < N; ++n) {
      int64_t r = 1, after = 1;
      for (int k = 0; k < N; ++k) {
        if (k != n) r *= k < n ? K[k] : I[k];
        after *= k <= n ? K[k] : I[k];
      }
      rows[n] = r;
      om = r * K[n] > om ? r * K[n] : om;
      big = after > big ? after : big;
      zmax = I[n] * K[n] > zmax ? I[n] * K[n] : zmax;
      const int64_t q = qr_work_doubles(I[n], K[n]);
      qrmax = q > qrmax ? q : qrmax;
    }
    Om = ar.take<T>(om);
    buf[0] = ar.take<T>(big);
    buf[1] = ar.take<T>(big);
    Z = ar.take<T>(zmax);
    qrwork = ar.take<double>(qrmax);
    zpart_cap = sketch_part_elems(imax, kmax);
    zpart = ar.take<T>(zpart_cap);
    iflags = ar.take<int32_t>(16);
    return ar.need;
  }
};

template <typename T>
int seq_run(const rt_sequential_desc* d, const T* Y, void* ws, size_t ws_bytes,
            void* const* U, T* G, void* const* Om_out, hipStream_t s) {
  SeqPlan<T> P;
  const size_t need = P.plan(d, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  P.plan(d, ws);
  const int N = P.N;
  RT_TRY(launch_fill_i32(P.iflags, 0, 16, s));
  int64_t D[RT_MAX_MODES];
  for (int n = 0; n < N; ++n) D[n] = P.I[n];
  const T* src = Y;
  for (int n = 0; n < N; ++n) {
    RT_TRY(launch_gaussian_fill<T>(P.Om, P.rows[n], P.K[n], n, d->seed, s));
    if (Om_out && Om_out[n] &&
        hipMemcpyAsync(Om_out[n], P.Om, P.rows[n] * P.K[n] * sizeof(T),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return hip_fail(hipGetLastError(), "Omega copy");
    int64_t Apre = 1, Cpost = 1;
    for (int k = 0; k < n; ++k) Apre *= D[k];
    for (int k = n + 1; k < N; ++k) Cpost *= D[k];
    // Z_n = Y_(n) Omega_n with Y viewed [Apre, I_n, Cpost]: row (a, c) of
    // Omega_n is a * Cpost + c, the row-major order of the other modes
    RT_TRY(launch_sketch_gemm<T>(src, P.Om, P.Z, P.zpart, P.zpart_cap, Apre, D[n], Cpost,
                                 P.K[n], s));
    QrBatch qb{};
    qb.nb = 1;
    qb.bit0 = n;
    qb.need = P.iflags + 4;
    qb.Z[0] = P.Z;
    qb.Q[0] = U[n];
    qb.work[0] = P.qrwork;
    qb.I[0] = D[n];
    qb.K[0] = P.K[n];
    RT_TRY(launch_qr<T>(qb, P.iflags + 1, s));
    // Y <- Y x_n U_n^T (the last product writes the core)
    T* dst = (n == N - 1) ? G : P.buf[n & 1];
    RT_TRY(launch_ttm<T>(src, static_cast<const T*>(U[n]), dst, Apre, D[n], Cpost, P.K[n],
                         s));
    D[n] = P.K[n];
    src = dst;
  }
  return kOk;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_gaussian_matrix(int32_t dtype, uint64_t seed, int32_t mode, int64_t rows, int32_t cols,
                       void* out, void* stream) {
  if (rows < 1 || cols < 1 || mode < 0) {
    set_error("rt_gaussian_matrix: rows, cols must be >= 1 and mode >= 0");
    return kErrInvalid;
  }
  if (!out || (reinterpret_cast<uintptr_t>(out) & 15u)) {
    set_error("rt_gaussian_matrix: out is NULL or not 16-byte aligned");
    return kErrInvalid;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == RT_F32)
    return launch_gaussian_fill<float>(static_cast<float*>(out), rows, cols, mode, seed, s);
  if (dtype == RT_F64)
    return launch_gaussian_fill<double>(static_cast<double*>(out), rows, cols, mode, seed, s);
  set_error("rt_gaussian_matrix: dtype %d unsupported", dtype);
  return kErrInvalid;
}

int rt_tucker_sequential_workspace(const rt_sequential_desc* desc, size_t* bytes) {
  RT_TRY(validate_seq(desc));
  if (!bytes) {
    set_error("bytes is NULL");
    return kErrInvalid;
  }
  if (desc->precision == RT_F64) {
    SeqPlan<double> p;
    *bytes = p.plan(desc, nullptr);
  } else {
    SeqPlan<float> p;
    *bytes = p.plan(desc, nullptr);
  }
  return kOk;
}

int rt_tucker_sequential(const rt_sequential_desc* desc, const void* Y, void* ws,
                         size_t ws_bytes, void* const* U, void* G, void* const* Omega_out,
                         void* stream) {
  RT_TRY(validate_seq(desc));
  auto bad = [](const void* p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15u); };
  if (bad(Y) || bad(ws) || bad(G) || !U) {
    set_error("Y, ws, G and U must be non-NULL, 16-byte aligned device pointers");
    return kErrInvalid;
  }
  for (int n = 0; n < desc->N; ++n) {
    if (bad(U[n])) {
      set_error("U[%d] is NULL or not 16-byte aligned", n);
      return kErrInvalid;
    }
    if (Omega_out && Omega_out[n] && bad(Omega_out[n])) {
      set_error("Omega_out[%d] is not 16-byte aligned", n);
      return kErrInvalid;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (desc->precision == RT_F64)
    return seq_run<double>(desc, static_cast<const double*>(Y), ws, ws_bytes, U,
                           static_cast<double*>(G), Omega_out, s);
  return seq_run<float>(desc, static_cast<const float*>(Y), ws, ws_bytes, U,
                        static_cast<float*>(G), Omega_out, s);
}

}  // extern "C"
