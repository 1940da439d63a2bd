// FFCP with the ALS update (Algorithm 1 with eq. (14), Section III-B) run
// entirely in the compressed space.
//
// For the unconstrained update every factor stays in the range of its Tucker
// basis: A_n = U_n H T^{-1} = U_n Vh_n with Vh_n = H T^{-1} (R_n x R).  With
// M_n = U_n^T U_n (computed once; the identity up to the rounding of U_n), all
// the quantities Algorithm 1 forms in the I_n-dimensional space have exact
// compressed-space counterparts:
//   V_n    = U_n^T A_n         = M_n Vh_n
//   Gram_n = A_n^T A_n         = Vh_n^T M_n Vh_n = Vh_n^T V_n
//   ||a_r||^2 (column norms)   = (Vh_n^T M_n Vh_n)_rr
// so one iteration costs O(N (R prod_p R_p + R^3)) independently of I_n
// (eq. (10): CP of the Tucker core), and A_n = U_n Vh_n is formed once at the
// end.  Results equal the I_n-space recursion up to FP64 rounding order.
//
// One workgroup runs the whole loop (the work per step is tiny and serial in
// the modes); the core (FP32, promoted on read), the MTTKRP intermediates and
// all R x R / R_n x R matrices live in LDS when they fit.  Per mode, wave 0
// forms T and solves Vh T = H by Gauss-Jordan with the working columns in
// registers (one per lane) and the pivot column broadcast through scalar
// registers (when R + R_n > 64 it inverts T the same way and Vh = H T^{-1}
// is a product over all threads).  Then one wave per column forms
// P = M_n Vh, the column norm and the normalized columns, and the Gram
// A_n^T A_n = Vh^T P follows: three barriers per mode after the MTTKRP.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kLdsMax = 160 * 1024;

struct InfoDev {
  int32_t iterations, converged, ridged, init_used;
  double fit, fit_prev;
};

struct CoreAlsArgs {
  FfcpArgs a;
  int RP;             // R rounded up to a multiple of 4: row stride of R-wide rows
  int64_t core;       // prod R_n
  int64_t x1_doubles; // first MTTKRP step (shared by modes 0..N-2)
  // LDS byte offsets
  int oV[8], oVh[8], oM[8], oGram[8];
  int oT, oL, oH, oVr, oRed, oG, oX1, oW1, oW2, oStage;
  // MTTKRP schedule: step st of mode n contracts mode sm with V_sm; the
  // operand is [sApre, R_sm, sCpost] (times RP after the first step)
  int sm[8][8], sApre[8][8], sCpost[8][8];
};

// 1/p from the hardware estimate refined by two Newton steps (within an ulp
// or two of the correctly rounded quotient; the IEEE division sequence is
// several times longer and sits on the pivot chain)
__device__ __forceinline__ double recip(double p) {
  double x = __builtin_amdgcn_rcp(p);
  double e = fma(-p, x, 1.0);
  x = fma(x, e, x);
  e = fma(-p, x, 1.0);
  return fma(x, e, x);
}

// value of v held by lane `lane` (uniform), through the scalar unit
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// v from the lane that the DPP control selects (within a row of 16 lanes)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over a row of 16 lanes (all active), the same bits in every lane of
// the row: butterflies on the DPP network (quad swaps, half-row and row
// mirrors).  No LDS traffic.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0xb1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}

// Sum over the 64 lanes, the same bits in every lane: the row sums, then
// the four of them in a fixed order through scalar registers.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = row_sum16(v);
  return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

// Wave-level in-place Gauss-Jordan inversion of the symmetric positive
// definite R x R matrix T + delta I (row stride RP) into Tinv.  Lane j holds
// column j in registers; step k broadcasts the pivot column from lane k
// through scalar registers, so no step waits on LDS.  Without pivoting the
// pivots are the Schur-complement diagonals, i.e. the squared diagonal of
// the Cholesky factor: a pivot <= 0 means T is not numerically positive
// definite (returns false).
template <int RMAX>
__device__ __forceinline__ bool gj_inverse_wave(const double* T, int RP, int R,
                                                double delta, double* Tinv) {
  const int j = threadIdx.x & 63;
  const int jc = j < R ? j : R - 1;   // clamped: every load is in bounds
  double col[RMAX];
#pragma unroll
  for (int i = 0; i < RMAX; ++i) {
    const int ic = i < R ? i : R - 1;
    const double v = T[ic * RP + jc] + (i == j ? delta : 0.0);
    col[i] = (i < R && j < R) ? v : 0.0;
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k < R) {
      double p = lane_bcast(col[k], k);
      if (!(p > 0.0)) {
        ok = false;
        p = 1.0;
      }
      const double rip = ((j == k) ? 1.0 : col[k]) * recip(p);
#pragma unroll
      for (int i = 0; i < RMAX; ++i) {
        if (i != k) {
          const double f = lane_bcast(col[i], k);   // zero for i >= R
          col[i] = ((j == k) ? 0.0 : col[i]) - f * rip;
        }
      }
      col[k] = rip;
    }
  }
  if (j < R) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < R) Tinv[i * RP + j] = col[i];
  }
  return ok;
}

// Wave-level Gauss-Jordan solve of X (T + delta I) = H for X (Rn x R), where
// T = hadamard_{p != n} Gram_p (R x R, symmetric positive definite) is formed
// here, each lane c < R building column c of T from the Grams (row stride
// RP), so no separate pass writes T.  The wave holds the augmented matrix
// [T + delta I | H^T] (R rows), lane c column c (R + Rn <= 64), and
// eliminates one pivot per step without pivoting: the pivot column comes
// from lane k through scalar registers (two readlanes per entry), which
// costs less than a round trip through LDS per step.  After the last step
// lane R + i holds column i of T^{-1} H^T, i.e. row i of X.  The pivots are
// the Schur-complement diagonals of an SPD matrix: a pivot <= 0 means
// T + delta I is not numerically positive definite (returns false).  *trace
// receives tr(T) (every lane).  gram(p) returns Gram_p.
template <int RMAX, class GramFn>
__device__ __forceinline__ bool gj_solve_wave(GramFn gram, int N, int n, int RP,
                                              int R, double delta, const double* H, int Rn,
                                              double* X, double* trace) {
  static_assert(RMAX <= 32, "two columns of RMAX rows per lane");
  const int c = threadIdx.x & 63;
  const bool isT = c < R, isH = c >= R && c < R + Rn;
  const int jt = isT ? c : 0, ih = isH ? c - R : 0;   // clamped: loads in bounds
  double col[RMAX];
#pragma unroll
  for (int i = 0; i < RMAX; ++i) col[i] = 1.0;
  for (int p = 0; p < N; ++p) {
    if (p == n) continue;
    const double* Gp = gram(p);
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      const int ic = i < R ? i : R - 1;
      col[i] *= Gp[ic * RP + jt];
    }
  }
  double dg = 0.0;
#pragma unroll
  for (int i = 0; i < RMAX; ++i) {
    const int ic = i < R ? i : R - 1;
    double v = 0.0;
    if (isT) {
      if (i == c) dg = col[i];
      v = col[i] + (i == c ? delta : 0.0);
    } else if (isH) {
      v = H[ih * RP + ic];
    }
    col[i] = i < R ? v : 0.0;
  }
  *trace = wave_sum(dg);
  bool ok = true;
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k < R) {
      double m[RMAX];   // the pivot column (zero below row R)
#pragma unroll
      for (int i = 0; i < RMAX; ++i) m[i] = lane_bcast(col[i], k);
      // a failed pivot spoils the result, which the caller then discards
      const double p = m[k];
      ok = ok && p > 0.0;
      const double f = col[k] * recip(p);
#pragma unroll
      for (int i = 0; i < RMAX; ++i)
        if (i != k) col[i] = fma(-m[i], f, col[i]);
      col[k] = f;
    }
  }
  if (isH) {
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < R) X[ih * RP + i] = col[i];
  }
  return ok;
}

// out (p x q, row stride ldo) = X^T Y over `rows` rows of the row-major
// float matrices X (rows x p) and Y (rows x q); 64-row blocks staged in LDS
// (st: 64 (p + q) doubles).  p, q <= 64.
template <int NT>
__device__ void cross_rows(const float* X, int p, const float* Y, int q,
                           int64_t rows, double* out, int ldo, double* st) {
  constexpr int kG = NT / 64;
  constexpr int kAcc = 64 / kG;
  const int t = threadIdx.x;
  const int v = t & 63, g = t >> 6;
  double acc[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k) acc[k] = 0.0;
  double* xs = st;
  double* ys = st + 64 * p;
  for (int64_t i0 = 0; i0 < rows; i0 += 64) {
    const int nr = static_cast<int>((rows - i0) < 64 ? (rows - i0) : 64);
    __syncthreads();
    for (int l = t; l < nr * p; l += NT) xs[l] = X[i0 * p + l];
    for (int l = t; l < nr * q; l += NT) ys[l] = Y[i0 * q + l];
    __syncthreads();
    if (v < q) {
      for (int ii = 0; ii < nr; ++ii) {
        const double yv = ys[ii * q + v];
#pragma unroll
        for (int k = 0; k < kAcc; ++k) {
          const int u = g + kG * k;
          if (u < p) acc[k] += xs[ii * p + u] * yv;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kAcc; ++k) {
    const int u = g + kG * k;
    if (u < p && v < q) out[u * ldo + v] = acc[k];
  }
  __syncthreads();
}

// C (m x n, ldc) = op(A) B with op(A) = A (m x k, lda) or A^T (A: k x m).
template <int NT>
__device__ void small_mm(const double* A, int lda, bool transA, const double* B,
                         int ldb, double* C, int ldc, int m, int k, int n) {
  for (int l = threadIdx.x; l < m * n; l += NT) {
    const int i = l / n, j = l % n;
    double acc = 0.0;
    for (int q = 0; q < k; ++q)
      acc += (transA ? A[q * lda + i] : A[i * lda + q]) * B[q * ldb + j];
    C[i * ldc + j] = acc;
  }
}

template <int RMAX, int NT, bool GLDS>
__global__ __launch_bounds__(NT) void ffcp_als_core_kernel(CoreAlsArgs c_arg) {
  extern __shared__ __align__(16) char smem[];
  // The argument is read in place from the kernel-argument segment: its
  // arrays are indexed with (uniform) runtime indices, which a by-value copy
  // would serve from per-thread scratch memory; here they are scalar loads.
  (void)c_arg;
  typedef const __attribute__((address_space(4))) CoreAlsArgs KArgs;
  KArgs& c = *reinterpret_cast<KArgs*>(
      reinterpret_cast<uintptr_t>(__builtin_amdgcn_kernarg_segment_ptr()));
  auto& a = c.a;
  const int t = threadIdx.x;
  const int N = a.N, R = a.R, RP = c.RP, R4 = RP / 4;
  const int64_t core = c.core;
  auto D = [&](int off) __attribute__((always_inline)) { return reinterpret_cast<double*>(smem + off); };
  InfoDev* info = static_cast<InfoDev*>(a.info);

  // ---- setup -------------------------------------------------------------
  const float* G;
  double* X1;
  double* W1;
  double* W2;
  // The core in LDS keeps its last mode's rows at an odd stride GP (a row
  // of R_{N-1} values padded by one when R_{N-1} is even), so lanes that
  // read the same position of consecutive rows hit different banks.
  const int RL = a.Rn[N - 1];
  const int GP = GLDS ? (RL | 1) : RL;
  auto gidx = [&](int64_t l) __attribute__((always_inline)) {
    return (l / RL) * GP + l % RL;
  };
  if constexpr (GLDS) {
    float* gs = reinterpret_cast<float*>(smem + c.oG);
    for (int64_t l = t; l < core; l += NT) gs[gidx(l)] = a.G[l];
    G = gs;
    X1 = D(c.oX1);
    W1 = D(c.oW1);
    W2 = D(c.oW2);
  } else {
    G = a.G;
    X1 = a.Qm;   // global scratch (sized for the first contraction)
    W1 = a.W1;
    W2 = a.W2;
  }
  // zero every R-wide row region (padding columns must stay zero)
  for (int n = 0; n < N; ++n) {
    for (int l = t; l < a.Rn[n] * RP; l += NT) {
      D(c.oV[n])[l] = 0.0;
      D(c.oVh[n])[l] = 0.0;
    }
    for (int l = t; l < R * RP; l += NT) D(c.oGram[n])[l] = 0.0;
  }
  __syncthreads();
  double* stage = D(c.oStage);
  for (int n = 0; n < N; ++n) {
    const int Rn = a.Rn[n];
    cross_rows<NT>(a.U[n], Rn, a.U[n], Rn, a.I[n], D(c.oM[n]), Rn, stage);
    if (a.A_init[n]) {
      cross_rows<NT>(a.U[n], Rn, a.A_init[n], R, a.I[n], D(c.oV[n]), RP, stage);
      cross_rows<NT>(a.A_init[n], R, a.A_init[n], R, a.I[n], D(c.oGram[n]), RP,
                     stage);
    }
  }
  __syncthreads();
  // coefficient starts (HOSVD or the caller's): A_n = U_n Vc_n
  // (alt: the HOSVD start kept beside the caller's, else the start)
  auto load_coeffs = [&](bool alt) __attribute__((always_inline)) {
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      double* Vh = D(c.oVh[n]);
      const double* Vc = alt ? a.V_alt[n] : a.V_init[n];
      for (int l = t; l < Rn * R; l += NT) Vh[(l / R) * RP + l % R] = Vc[l];
      __syncthreads();
      small_mm<NT>(D(c.oM[n]), Rn, false, Vh, RP, D(c.oV[n]), RP, Rn, Rn, R);
      __syncthreads();
      small_mm<NT>(Vh, RP, true, D(c.oV[n]), RP, D(c.oGram[n]), RP, R, Rn, R);
      __syncthreads();
    }
  };
  if (!a.A_init[0]) load_coeffs(false);

  // ||Yt||^2 = <G, G x_1 M_1 ... x_N M_N> unless given (global scratch)
  double nrm2 = a.normY2;
  double* red = D(c.oRed);
  if (!(nrm2 >= 0.0)) {
    const double* src = nullptr;
    double* bufs[2] = {a.W1, a.W2};  // core-sized, global
    int cur = 0;
    int64_t Apre = 1;
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      const int64_t Cpost = core / (Apre * Rn);
      const double* M = D(c.oM[n]);
      double* dst = bufs[cur];
      for (int64_t l = t; l < core; l += NT) {
        const int64_t cc = l % Cpost;
        const int64_t rest = l / Cpost;
        const int i = static_cast<int>(rest % Rn);
        const int64_t aa = rest / Rn;
        double acc = 0.0;
        for (int j = 0; j < Rn; ++j) {
          const int64_t idx = (aa * Rn + j) * Cpost + cc;
          const double x = src ? src[idx] : static_cast<double>(G[gidx(idx)]);
          acc += x * M[j * Rn + i];
        }
        dst[l] = acc;
      }
      __syncthreads();
      src = dst;
      cur ^= 1;
      Apre *= Rn;
    }
    double p = 0.0;
    for (int64_t l = t; l < core; l += NT) p += static_cast<double>(G[gidx(l)]) * src[l];
    nrm2 = block_sum(p, red);
    __syncthreads();
  }

  // ---- iterations ----------------------------------------------------------
  double* T = D(c.oT);
  double* L = D(c.oL);  // T^{-1}
  double* Hlast = D(c.oH);

  // H_n = G_(n) [KR_{p != n} V_p] into Hlast (returns it)
  auto mttkrp = [&](int n) __attribute__((always_inline)) -> const double* {
    // H = G_(n) [KR_{p != n} V_p]: contract the last remaining mode != n
    // (schedule precomputed on the host: mode, leading and trailing sizes).
    // The first step of modes 0..N-2 contracts mode N-1 with V_{N-1},
    // which only mode N-1 updates: it is computed once per iteration (X1).
    const double* src = nullptr;
    for (int st = 0; st < N - 1; ++st) {
      const int m = c.sm[n][st];
      const int Apre = c.sApre[n][st], Cpost = c.sCpost[n][st];
      const bool last = st == N - 2;
      const int Rm = a.Rn[m];
      const double* Vm = D(c.oV[m]);
      double* dst = last ? Hlast : (st == 0 ? X1 : (((st - 1) & 1) ? W2 : W1));
      const bool reuse = st == 0 && !last && n > 0 && n < N - 1;
      if (!reuse && src == nullptr) {
        // first step from the FP32 core (it contracts mode N-1 or N-2, so
        // Cpost is 1 or R_{N-1}): 4 positions (a, c) x 4 r per item, the
        // positions nq apart so that consecutive items read consecutive
        // rows of the core
        const int nac = Apre * Cpost;
        const int nq = (nac + 3) / 4;
        const int total = nq * R4;
        const int astride = Cpost == 1 ? GP : Rm * GP;   // padded strides
        const int jstride = Cpost == 1 ? 1 : GP;
        for (int item = t; item < total; item += NT) {
          const int rq = item % R4;
          const int ab = item / R4;
          int off[4];
          bool val[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ac = ab + u * nq;
            val[u] = ac < nac;
            const int acc_ = val[u] ? ac : nac - 1;   // clamped, in bounds
            const int cc = acc_ % Cpost, aa = acc_ / Cpost;
            off[u] = aa * astride + cc;
          }
          double acc[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
          const double* vp = Vm + 4 * rq;
          // operands of 4 consecutive j are loaded before any is used, so
          // four LDS round trips overlap; the last group of a length that is
          // not a multiple of 4 clamps j and weighs the extra terms zero
          auto group = [&](int j0, bool tail) __attribute__((always_inline)) {
            double2 v01[4], v23[4];
            float g[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = (!tail || j0 + q < Rm) ? j0 + q : Rm - 1;
              v01[q] = *reinterpret_cast<const double2*>(vp + j * RP);
              v23[q] = *reinterpret_cast<const double2*>(vp + j * RP + 2);
#pragma unroll
              for (int u = 0; u < 4; ++u) g[q][u] = G[off[u] + j * jstride];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const bool in = !tail || j0 + q < Rm;
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const double gv = in ? static_cast<double>(g[q][u]) : 0.0;
                acc[u][0] += gv * v01[q].x;
                acc[u][1] += gv * v01[q].y;
                acc[u][2] += gv * v23[q].x;
                acc[u][3] += gv * v23[q].y;
              }
            }
          };
          int j0 = 0;
          for (; j0 + 4 <= Rm; j0 += 4) group(j0, false);
          if (j0 < Rm) group(j0, true);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (val[u]) {
              double* dp = dst + (ab + u * nq) * RP + 4 * rq;
              *reinterpret_cast<double2*>(dp) = make_double2(acc[u][0], acc[u][1]);
              *reinterpret_cast<double2*>(dp + 2) = make_double2(acc[u][2], acc[u][3]);
            }
          }
        }
        __syncthreads();
      } else if (!reuse) {
        const int total = Apre * Cpost * R4;
        for (int item = t; item < total; item += NT) {
          const int rq = item % R4;
          const int ac = item / R4;
          const int cc = ac % Cpost, aa = ac / Cpost;
          double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
          const double* vp = Vm + 4 * rq;
          const double* sp = src + (aa * Rm * Cpost + cc) * RP + 4 * rq;
          const int sj = Cpost * RP;
          auto group = [&](int j0, bool tail) __attribute__((always_inline)) {
            double2 s01[4], s23[4], v01[4], v23[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = (!tail || j0 + q < Rm) ? j0 + q : Rm - 1;
              s01[q] = *reinterpret_cast<const double2*>(sp + j * sj);
              s23[q] = *reinterpret_cast<const double2*>(sp + j * sj + 2);
              v01[q] = *reinterpret_cast<const double2*>(vp + j * RP);
              v23[q] = *reinterpret_cast<const double2*>(vp + j * RP + 2);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (!tail || j0 + q < Rm) {
                acc0 += s01[q].x * v01[q].x;
                acc1 += s01[q].y * v01[q].y;
                acc2 += s23[q].x * v23[q].x;
                acc3 += s23[q].y * v23[q].y;
              }
            }
          };
          int j0 = 0;
          for (; j0 + 4 <= Rm; j0 += 4) group(j0, false);
          if (j0 < Rm) group(j0, true);
          double* dp = dst + ac * RP + 4 * rq;
          *reinterpret_cast<double2*>(dp) = make_double2(acc0, acc1);
          *reinterpret_cast<double2*>(dp + 2) = make_double2(acc2, acc3);
        }
        __syncthreads();
      }
      src = dst;
    }
    return src;
  };

  // closed-form fit of the current factors; uses the MTTKRP of the last
  // mode, which must be in Hlast
  auto fit_of_state = [&]() __attribute__((always_inline)) -> double {
    const int Rl = a.Rn[N - 1];
    const double* Vl = D(c.oV[N - 1]);
    double p = 0.0;
    for (int l = t; l < Rl * R; l += NT) {
      const int j = l / R, r = l % R;
      p += Hlast[j * RP + r] * Vl[j * RP + r];
    }
    const double inner = block_sum(p, red);
    double q = 0.0;
    for (int l = t; l < R * R; l += NT) {
      const int i = l / R, j = l % R;
      double v = 1.0;
      for (int pp = 0; pp < N; ++pp) v *= D(c.oGram[pp])[i * RP + j];
      q += v;
    }
    const double yh2 = block_sum(q, red);
    double res2 = nrm2 - 2.0 * inner + yh2;
    res2 = res2 > 0.0 ? res2 : 0.0;
    return 1.0 - sqrt(res2) / sqrt(nrm2);
  };

  // guarded start: keep the caller's coefficients only if their fit is at
  // least that of the HOSVD start
  int init_used = 0;
  if (!a.A_init[0] && a.V_alt[0]) {
    mttkrp(N - 1);
    const double f_user = fit_of_state();
    load_coeffs(true);
    mttkrp(N - 1);
    const double f_hosvd = fit_of_state();
    if (f_user >= f_hosvd) {
      load_coeffs(false);
      init_used = 1;
    }
  }

  double fit_prev = 0.0, fit = 0.0;
  int it = 0, converged = 0, ridged = 0;
  for (it = 1; it <= a.max_it; ++it) {
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      const double* H = mttkrp(n);  // Rn x RP (Hlast)

      // Vr = H T^{-1} with T = hadamard of the other Grams (ridge T + delta I
      // when T is not numerically positive definite)
      double* Vr = D(c.oVr);
      if (RMAX <= 32 && R + Rn <= 64) {
        // wave 0 forms T and solves
        if constexpr (RMAX <= 32) {
          if (t < 64) {
            auto gram = [&](int p) __attribute__((always_inline)) { return D(c.oGram[p]); };
            double delta = 0.0, tr = 0.0;
            for (int attempt = 0; attempt < 2; ++attempt) {
              if (gj_solve_wave<RMAX>(gram, N, n, RP, R, delta, H, Rn, Vr, &tr)) break;
              delta = 1e-12 * tr / R;
              ridged = 1;
            }
          }
        }
        __syncthreads();
      } else {
      // T in LDS, L <- T^{-1} by wave 0, then Vr = H L
      for (int l = t; l < R * R; l += NT) {
        const int i = l / R, j = l % R;
        double v = 1.0;
        for (int p = 0; p < N; ++p)
          if (p != n) v *= D(c.oGram[p])[i * RP + j];
        T[i * RP + j] = v;
      }
      __syncthreads();
      if (t < 64) {
        if (!gj_inverse_wave<RMAX>(T, RP, R, 0.0, L)) {
          double tr = 0.0;
          for (int k = 0; k < R; ++k) tr += T[k * RP + k];
          gj_inverse_wave<RMAX>(T, RP, R, 1e-12 * tr / R, L);
          ridged = 1;
        }
      }
      __syncthreads();
      for (int l = t; l < Rn * R4; l += NT) {
        const int i = l / R4, rq = l % R4;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        for (int q = 0; q < R; ++q) {
          const double hv = H[i * RP + q];
          const double2 v01 = *reinterpret_cast<const double2*>(L + q * RP + 4 * rq);
          const double2 v23 = *reinterpret_cast<const double2*>(L + q * RP + 4 * rq + 2);
          acc0 += hv * v01.x;
          acc1 += hv * v01.y;
          acc2 += hv * v23.x;
          acc3 += hv * v23.y;
        }
        double* vp = Vr + i * RP + 4 * rq;
        *reinterpret_cast<double2*>(vp) = make_double2(acc0, acc1);
        *reinterpret_cast<double2*>(vp + 2) = make_double2(acc2, acc3);
      }
      __syncthreads();
      }

      // One wave per column r: P(:, r) = M_n Vr(:, r) with lane j holding row
      // j (M_n is symmetric, so lane j reads row q of it at column j), the
      // squared column norm of the factor ||a_r||^2 = Vr(:, r)^T P(:, r) as a
      // wave sum, and the columns normalized for n < N-1 (zero columns stay
      // zero): Vh_n = Vr / nr, V_n = P / nr.
      double* Vh = D(c.oVh[n]);
      double* Vn = D(c.oV[n]);
      const double* M = D(c.oM[n]);
      const bool normalize = n < N - 1;
      {
        const int lane = t & 63, wave = t >> 6;
        const int jl = lane < Rn ? lane : 0;   // clamped: loads in bounds
        for (int r = wave; r < R; r += NT / 64) {
          double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
          int q = 0;
#pragma unroll 2
          for (; q + 4 <= Rn; q += 4) {
            const double m0 = M[q * Rn + jl], m1 = M[(q + 1) * Rn + jl];
            const double m2 = M[(q + 2) * Rn + jl], m3 = M[(q + 3) * Rn + jl];
            p0 = fma(m0, Vr[q * RP + r], p0);
            p1 = fma(m1, Vr[(q + 1) * RP + r], p1);
            p2 = fma(m2, Vr[(q + 2) * RP + r], p2);
            p3 = fma(m3, Vr[(q + 3) * RP + r], p3);
          }
          for (; q < Rn; ++q) p0 = fma(M[q * Rn + jl], Vr[q * RP + r], p0);
          const double pv = (p0 + p1) + (p2 + p3);
          const double vr = Vr[jl * RP + r];
          const double g = wave_sum_dpp(lane < Rn ? vr * pv : 0.0);
          const double nr = normalize && g > 0.0 ? sqrt(g) : 0.0;
          const double inv = nr > 0.0 ? 1.0 / nr : 1.0;
          if (lane < Rn) {
            Vh[lane * RP + r] = vr * inv;
            Vn[lane * RP + r] = pv * inv;
          }
        }
      }
      __syncthreads();
      // Gram_n = A_n^T A_n = Vh_n^T V_n
      {
        double* Gn = D(c.oGram[n]);
        for (int l = t; l < R * R; l += NT) {
          const int i = l / R, j = l % R;
          // four partial sums: independent LDS round trips and FMA chains
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
          int q = 0;
          for (; q + 4 <= Rn; q += 4) {
            a0 = fma(Vh[q * RP + i], Vn[q * RP + j], a0);
            a1 = fma(Vh[(q + 1) * RP + i], Vn[(q + 1) * RP + j], a1);
            a2 = fma(Vh[(q + 2) * RP + i], Vn[(q + 2) * RP + j], a2);
            a3 = fma(Vh[(q + 3) * RP + i], Vn[(q + 3) * RP + j], a3);
          }
          for (; q < Rn; ++q) a0 = fma(Vh[q * RP + i], Vn[q * RP + j], a0);
          Gn[i * RP + j] = (a0 + a1) + (a2 + a3);
        }
      }
      __syncthreads();
    }
    // ---- fit (the last mode's H is still in Hlast) -------------------------
    fit = fit_of_state();
    if (t == 0 && a.fit_trace) a.fit_trace[it - 1] = fit;
    if (it >= 2 && fabs(fit - fit_prev) < a.tol) {
      converged = 1;
      break;
    }
    if (it < a.max_it) fit_prev = fit;
    __syncthreads();
  }
  if (it > a.max_it) it = a.max_it;
  // ridged is known to wave 0 only
  __shared__ int ridged_any;
  if (t == 0) ridged_any = ridged;
  __syncthreads();

  // ---- outputs: A_n = U_n Vh_n; the last factor normalized, lambda -----------
  for (int n = 0; n < N; ++n) {
    const int Rn = a.Rn[n];
    const double* Vh = D(c.oVh[n]);
    const float* Un = a.U[n];
    const double* Gn = D(c.oGram[n]);
    const int64_t cnt = a.I[n] * R;
    for (int64_t l = t; l < cnt; l += NT) {
      const int64_t i = l / R;
      const int r = static_cast<int>(l % R);
      double acc = 0.0;
      for (int j = 0; j < Rn; ++j) acc += static_cast<double>(Un[i * Rn + j]) * Vh[j * RP + r];
      if (n == N - 1) {
        const double nr = sqrt(Gn[r * RP + r]);
        if (nr > 0.0) acc /= nr;
      }
      a.A_out[n][l] = static_cast<float>(acc);
    }
  }
  {
    const double* Gl = D(c.oGram[N - 1]);
    for (int r = t; r < R; r += NT) a.lambda[r] = static_cast<float>(sqrt(Gl[r * RP + r]));
  }
  if (t == 0 && info) {
    info->iterations = it;
    info->converged = converged;
    info->ridged = ridged_any;
    info->init_used = init_used;
    info->fit = fit;
    info->fit_prev = fit_prev;
  }
}

// LDS layout; returns the byte size or -1 when the small matrices alone do
// not fit.  glds selects the core and MTTKRP buffers in LDS as well.
int64_t layout(CoreAlsArgs& c, bool glds) {
  const FfcpArgs& a = c.a;
  const int N = a.N, R = a.R;
  c.RP = (R + 3) / 4 * 4;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off += (bytes + 15) / 16 * 16;
    return static_cast<int>(o);
  };
  int Rmax = 0;
  int64_t core = 1;
  for (int n = 0; n < N; ++n) {
    Rmax = a.Rn[n] > Rmax ? a.Rn[n] : Rmax;
    core *= a.Rn[n];
  }
  c.core = core;
  for (int n = 0; n < N; ++n) {
    c.oV[n] = take(8LL * a.Rn[n] * c.RP);
    c.oVh[n] = take(8LL * a.Rn[n] * c.RP);
    c.oM[n] = take(8LL * a.Rn[n] * a.Rn[n]);
    c.oGram[n] = take(8LL * R * c.RP);
  }
  c.oT = take(8LL * R * c.RP);
  c.oL = take(8LL * (R * c.RP > 64 ? R * c.RP : 64));   // also the pivot column
  c.oH = take(8LL * Rmax * c.RP);
  c.oVr = take(8LL * Rmax * c.RP);
  c.oRed = take(8LL * 64);
  // staging for the setup cross products: 64 rows of (p + q) <= 2 max(R, Rn);
  // with the MTTKRP buffers in LDS it shares the first-step buffer (X1 is
  // not in use before the iterations start)
  const int wmax = R > Rmax ? R : Rmax;
  const int64_t stage_bytes = 8LL * 64 * 2 * wmax;
  // MTTKRP intermediates: the first step (X1) and the alternating later
  // steps (W1, W2); the final step writes H
  int64_t x1 = 0, w[2] = {0, 0};
  for (int n = 0; n < N; ++n) {
    int rem[8], nrem = N;
    for (int p = 0; p < N; ++p) rem[p] = p;
    int step = 0;
    while (nrem > 1) {
      int pos = nrem - 1;
      if (rem[pos] == n) pos = nrem - 2;
      int Apre = 1, Cpost = 1;
      for (int q = 0; q < pos; ++q) Apre *= a.Rn[rem[q]];
      for (int q = pos + 1; q < nrem; ++q) Cpost *= a.Rn[rem[q]];
      c.sm[n][step] = rem[pos];
      c.sApre[n][step] = Apre;
      c.sCpost[n][step] = Cpost;
      if (nrem > 2) {  // the final step writes H
        const int64_t out = static_cast<int64_t>(Apre) * Cpost * c.RP;
        if (step == 0)
          x1 = out > x1 ? out : x1;
        else
          w[(step - 1) & 1] = out > w[(step - 1) & 1] ? out : w[(step - 1) & 1];
      }
      for (int q = pos; q < nrem - 1; ++q) rem[q] = rem[q + 1];
      --nrem;
      ++step;
    }
  }
  c.x1_doubles = x1;
  if (!glds) {
    c.oStage = take(stage_bytes);
    c.oG = c.oX1 = c.oW1 = c.oW2 = 0;
    return off;
  }
  {
    const int RL = a.Rn[a.N - 1];
    c.oG = take(4LL * (core / RL) * (RL | 1));   // padded rows (see the kernel)
  }
  c.oX1 = take(8LL * x1 > stage_bytes ? 8LL * x1 : stage_bytes);
  c.oStage = c.oX1;
  c.oW1 = take(8LL * (w[0] > 0 ? w[0] : 1));
  c.oW2 = take(8LL * (w[1] > 0 ? w[1] : 1));
  return off;
}

template <int RMAX, int NT, bool GLDS>
int launch_one(const CoreAlsArgs& c, int64_t lds, hipStream_t s) {
  auto k = ffcp_als_core_kernel<RMAX, NT, GLDS>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return hip_fail(e, "ffcp core LDS attribute");
  hipLaunchKernelGGL(k, dim3(1), dim3(NT), static_cast<size_t>(lds), s, c);
  RT_LAUNCH_CHECK("ffcp core ALS");
  return kOk;
}

template <int RMAX, int NT>
int launch_r(CoreAlsArgs& c, hipStream_t s) {
  int64_t lds = layout(c, true);
  if (lds + 64 <= kLdsMax) return launch_one<RMAX, NT, true>(c, lds, s);
  lds = layout(c, false);
  if (lds + 64 <= kLdsMax) return launch_one<RMAX, NT, false>(c, lds, s);
  return kErrUnsupported;
}

// ------------------------------------------------------------ three-way
// The iterations of the same method for three-way cores with R and every
// R_n at most K: the ranks are zero-padded to K, so every loop has a
// compile-time trip count and every matrix a fixed place in LDS (rows of K
// doubles), and no index arithmetic or schedule is read at run time.  The
// tall cross products of the start (M_n = U_n^T U_n; U_n^T A_n and A_n^T A_n
// for a start given as factors) come from the batched cross-product kernel;
// the kernel itself forms the coefficient start, ||Yt||^2 and the guarded
// choice, and the output kernel forms A_n = U_n Vh_n.  Zero padding changes
// no value: the padded rows and columns of V_n, Vh_n, M_n, H and the Grams
// stay zero, and the elimination takes only the first R pivots.
//
// Per mode, T_n = hadamard of the other two Grams is known before H_n, so
// the two run side by side: wave 0 factors T_n = L D L^T by forward
// elimination in registers (keeping E = L^{-1} and D) while waves 1-3 and
// 5-7 form the MTTKRP of eqs. (12)-(13) through the core
//   mode 0: X = G x_3 V_2 (all K^2 positions (i0, i1) in register blocks),
//           H_0 = X x_2 V_1;
//   mode 1: H_1 = X x_1 V_0 (X is still current: V_2 has not changed);
//   mode 2: Y = G x_2 V_1, H_2 = Y x_1 V_0;
// and M_n H_n.  Then T_n^{-1} = E^T D^{-1} E and the update of eq. (14):
// Vh_n = H_n T_n^{-1} and V_n = U_n^T A_n = (M_n H_n) T_n^{-1}, normalized
// by the column norms ||a_r||^2 = Vh_n(:, r)^T V_n(:, r) (16-lane DPP row
// sums), and the Gram A_n^T A_n = Vh_n^T V_n.  Six or seven barriers per
// mode, none waiting on a serial chain other than the elimination.
constexpr int kA3Threads = 512;

template <int K>
struct A3Layout {
  static constexpr int GP = K | 1;   // core rows (last mode) padded to an odd stride
  static constexpr int KK = K * K;
  static constexpr int oG = 0;                                   // float [K][K][GP]
  static constexpr int oV = (4 * KK * GP + 15) / 16 * 16;        // double [3][K][K]
  static constexpr int oVh = oV + 3 * 8 * KK;
  static constexpr int oM = oVh + 3 * 8 * KK;
  static constexpr int oGram = oM + 3 * 8 * KK;
  static constexpr int oW = oGram + 3 * 8 * KK;                  // double [K][K][K]
  static constexpr int oH = oW + 8 * K * KK;
  static constexpr int SP = K + 2;                               // pitch of the transposed arrays
  static constexpr int oTi = oH + 8 * KK;                        // T^{-1} by columns [K][SP]
  static constexpr int oMH = oTi + 8 * K * SP;                   // M_n H
  static constexpr int oS = oMH + 8 * KK;                        // Vr^T, P^T [K][SP] doubles each
  static constexpr int oSv = oS + 2 * 8 * K * SP;                // column scales, K doubles
  static constexpr int oRed = oSv + 8 * K;                       // 2 doubles per wave
  static constexpr int bytes = oRed + 8 * 2 * (kA3Threads / 64);
};

template <int K>
__global__ __launch_bounds__(kA3Threads) __attribute__((amdgpu_waves_per_eu(1, 2)))
void ffcp_als3_kernel(FfcpArgs a_arg) {
  static_assert(K % 4 == 0 && K <= 32, "rows of K doubles in 4-column quads");
  using L = A3Layout<K>;
  constexpr int GP = L::GP, KK = L::KK, RQ = K / 4, NT = kA3Threads;
  extern __shared__ __align__(16) char smem[];
  (void)a_arg;
  typedef const __attribute__((address_space(4))) FfcpArgs KArgs;
  KArgs& a = *reinterpret_cast<KArgs*>(
      reinterpret_cast<uintptr_t>(__builtin_amdgcn_kernarg_segment_ptr()));
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int R = a.R;
  float* G = reinterpret_cast<float*>(smem + L::oG);
  auto Vn = [&](int n) __attribute__((always_inline)) {
    return reinterpret_cast<double*>(smem + L::oV + 8 * KK * n);
  };
  auto Vhn = [&](int n) __attribute__((always_inline)) {
    return reinterpret_cast<double*>(smem + L::oVh + 8 * KK * n);
  };
  auto Mn = [&](int n) __attribute__((always_inline)) {
    return reinterpret_cast<double*>(smem + L::oM + 8 * KK * n);
  };
  auto Gramn = [&](int n) __attribute__((always_inline)) {
    return reinterpret_cast<double*>(smem + L::oGram + 8 * KK * n);
  };
  double* W = reinterpret_cast<double*>(smem + L::oW);
  double* H = reinterpret_cast<double*>(smem + L::oH);
  double* red = reinterpret_cast<double*>(smem + L::oRed);

  // ---- the start, zero-padded --------------------------------------------
  {
    double* z = reinterpret_cast<double*>(smem + L::oV);
    for (int l = t; l < (L::oRed - L::oV) / 8; l += NT) z[l] = 0.0;
    for (int l = t; l < KK * GP; l += NT) G[l] = 0.0f;
  }
  __syncthreads();
  {
    const int R0 = a.Rn[0], R1 = a.Rn[1], R2 = a.Rn[2];
    for (int l = t; l < R0 * R1 * R2; l += NT) {
      const int i0 = l / (R1 * R2), rem = l - i0 * (R1 * R2);
      const int i1 = rem / R2, i2 = rem - i1 * R2;
      G[(i0 * K + i1) * GP + i2] = a.G[l];
    }
  }
  // M_n = U_n^T U_n (dense R_n x R_n in a.U64); a start given as I_n x R
  // factors comes as V_n = U_n^T A_n (a.V) and Gram_n = A_n^T A_n (a.Gram)
  const bool user = a.A_init[0] != nullptr;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const int Rn = a.Rn[n];
    for (int l = t; l < Rn * Rn; l += NT) {
      const int j = l / Rn, q = l - j * Rn;
      Mn(n)[j * K + q] = a.U64[n][l];
    }
    if (user) {
      for (int l = t; l < Rn * R; l += NT) {
        const int j = l / R, r = l - j * R;
        Vn(n)[j * K + r] = a.V[n][l];
      }
      for (int l = t; l < R * R; l += NT) {
        const int i = l / R, j = l - i * R;
        Gramn(n)[i * K + j] = a.Gram[n][l];
      }
    }
  }
  __syncthreads();

  double* Ti = reinterpret_cast<double*>(smem + L::oTi);
  double* MH = reinterpret_cast<double*>(smem + L::oMH);
  // The MTTKRP steps run on waves 1-3 and 5-7 (worker u of NW = 384) while
  // wave 0 factors T; wave 4, which shares wave 0's SIMD when the waves are
  // placed round-robin, only meets the barriers.  Each step ends with a
  // barrier that wave 0 matches (or takes part in with no items, at the
  // start).
  constexpr int NW = NT - 128;
  const int u_w = (wave == 0 || wave == 4) ? (1 << 20) : (wave < 4 ? t - 64 : t - 128);
  // W[p][r] = sum_j G(p, j) Vm[j][r] over the contracted mode j; p runs over
  // the K^2 positions of the other two modes, PG positions KK/PG apart and
  // RG columns per item (5 x 5 when K = 20, so that the items fit the
  // workers once).  MID: the contracted mode is the middle one and
  // p = (i0, i2); else the last and p = (i0, i1).
  auto big_step = [&](auto mid, const double* Vm) __attribute__((always_inline)) {
    constexpr bool MID = decltype(mid)::value;
    constexpr int RG = K % 5 == 0 ? 5 : 4, NG = K / RG, PG = RG;
    constexpr int NQ = KK / PG, JS = MID ? GP : 1;
    for (int item = u_w; item < NQ * NG; item += NW) {
      const int rg = item % NG, pq = item / NG;
      int goff[PG];
#pragma unroll
      for (int u = 0; u < PG; ++u) {
        const int p = pq + u * NQ;
        const int i0 = p / K, x = p - i0 * K;
        goff[u] = MID ? i0 * K * GP + x : p * GP;
      }
      double acc[PG][RG];
#pragma unroll
      for (int u = 0; u < PG; ++u)
#pragma unroll
        for (int v = 0; v < RG; ++v) acc[u][v] = 0.0;
      const double* vp = Vm + RG * rg;
      // operands of step j + 2 are fetched while step j's products run
      // (three register sets), so the LDS latency is covered
      float gq[3][PG];
      double vq[3][RG];
      auto fetch = [&](int j, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < RG; ++v) vq[b][v] = vp[j * K + v];
#pragma unroll
        for (int u = 0; u < PG; ++u) gq[b][u] = G[goff[u] + j * JS];
      };
      fetch(0, 0);
      fetch(1, 1);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j + 2 < K) fetch(j + 2, (j + 2) % 3);
        const int b = j % 3;
#pragma unroll
        for (int u = 0; u < PG; ++u) {
          const double g = static_cast<double>(gq[b][u]);
#pragma unroll
          for (int v = 0; v < RG; ++v) acc[u][v] = fma(g, vq[b][v], acc[u][v]);
        }
      }
#pragma unroll
      for (int u = 0; u < PG; ++u) {
        double* dp = W + (pq + u * NQ) * K + RG * rg;
#pragma unroll
        for (int v = 0; v < RG; ++v) dp[v] = acc[u][v];
      }
    }
    __syncthreads();
  };
  // H[x][r] = sum_y W(x, y)[r] Vm[y][r] with W(x, y) = W[x][y] (XFIRST) or
  // W[y][x]; an item is one row x and a column pair, with the even and odd
  // y summed apart
  auto small_step = [&](auto xfirst, const double* Vm) __attribute__((always_inline)) {
    constexpr bool XF = decltype(xfirst)::value;
    constexpr int RP = K / 2;
    for (int item = u_w; item < K * RP; item += NW) {
      const int rp = item % RP, x = item / RP;
      double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
      for (int y = 0; y < K; y += 2) {
        const double2 w0 = *reinterpret_cast<const double2*>(
            W + (XF ? x * K + y : y * K + x) * K + 2 * rp);
        const double2 w1 = *reinterpret_cast<const double2*>(
            W + (XF ? x * K + y + 1 : (y + 1) * K + x) * K + 2 * rp);
        const double2 v0 = *reinterpret_cast<const double2*>(Vm + y * K + 2 * rp);
        const double2 v1 = *reinterpret_cast<const double2*>(Vm + (y + 1) * K + 2 * rp);
        a0 = fma(w0.x, v0.x, a0);
        a1 = fma(w0.y, v0.y, a1);
        b0 = fma(w1.x, v1.x, b0);
        b1 = fma(w1.y, v1.y, b1);
      }
      *reinterpret_cast<double2*>(H + x * K + 2 * rp) = make_double2(a0 + b0, a1 + b1);
    }
    __syncthreads();
  };

  // MH = M_n H (M_n symmetric, zero-padded), items as in the small step
  auto mh_step = [&](const double* M) __attribute__((always_inline)) {
    constexpr int RP = K / 2;
    for (int item = u_w; item < K * RP; item += NW) {
      const int rp = item % RP, x = item / RP;
      double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
      for (int y = 0; y < K; y += 2) {
        const double2 m = *reinterpret_cast<const double2*>(M + x * K + y);
        const double2 h0 = *reinterpret_cast<const double2*>(H + y * K + 2 * rp);
        const double2 h1 = *reinterpret_cast<const double2*>(H + (y + 1) * K + 2 * rp);
        a0 = fma(m.x, h0.x, a0);
        a1 = fma(m.x, h0.y, a1);
        b0 = fma(m.y, h1.x, b0);
        b1 = fma(m.y, h1.y, b1);
      }
      *reinterpret_cast<double2*>(MH + x * K + 2 * rp) = make_double2(a0 + b0, a1 + b1);
    }
    __syncthreads();
  };

  int ridged = 0;
  // Wave 0: forward Gaussian elimination without pivoting on [T + delta I |
  // I] for T = Gp .* Gq (R x R): lane c < R holds column c of T, lane R + c
  // column c of I; step k takes the pivot column's rows k.. from lane k
  // through scalar registers and clears the rows below k.  With T = L D L^T
  // the pivots are D and the right half becomes E = L^{-1}, so that
  // T^{-1} = E^T D^{-1} E (formed by all waves in ti_step).  Lane R + c
  // stores column c of E and of D^{-1} E transposed (rows of pitch SP, in
  // the pair S1, S2, free until the finishing passes).  A pivot <= 0 means
  // T is not numerically positive definite: the elimination is repeated
  // with the ridge delta = 1e-12 tr(T) / R.  With SPLIT the first attempt
  // meets one barrier after its first K/5 steps (the small step's, in the
  // mode without a big step: the M_n H step then runs beside the rest).
  auto eliminate_T = [&](const double* Gp, const double* Gq, bool split) __attribute__((always_inline)) {
    constexpr int KS = K / 5, SP = L::SP;
    double* Et = reinterpret_cast<double*>(smem + L::oS);
    double* EtD = Et + K * SP;
    const int c = lane;
    const bool isT = c < R, isI = c >= R && c < 2 * R;
    const int jt = isT ? c : 0;   // clamped: loads in bounds
    double dg = 0.0;
    double tcol[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      tcol[i] = Gp[i * K + jt] * Gq[i * K + jt];
      if (i == c) dg = tcol[i];
    }
    const double tr = wave_sum_dpp(isT ? dg : 0.0);
    double delta = 0.0;
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
      double col[K], rps[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        double v = 0.0;
        if (isT)
          v = tcol[i] + (i == c ? delta : 0.0);
        else if (isI)
          v = i == c - R ? 1.0 : 0.0;
        col[i] = i < R ? v : 0.0;
      }
      bool ok = true;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k == KS && split && attempt == 0) __syncthreads();
        rps[k] = 0.0;
        if (k < R) {
          double m[K];
#pragma unroll
          for (int i = k; i < K; ++i) m[i] = lane_bcast(col[i], k);
          const double piv = m[k];
          ok = ok && piv > 0.0;
          rps[k] = recip(piv);
          const double f = col[k] * rps[k];
#pragma unroll
          for (int i = k + 1; i < K; ++i) col[i] = fma(-m[i], f, col[i]);
        }
      }
      if (ok || attempt == 1) {
        if (isI) {
#pragma unroll
          for (int i = 0; i < K; i += 2) {
            *reinterpret_cast<double2*>(Et + (c - R) * SP + i) = make_double2(col[i], col[i + 1]);
            *reinterpret_cast<double2*>(EtD + (c - R) * SP + i) =
                make_double2(col[i] * rps[i], col[i + 1] * rps[i + 1]);
          }
        }
        break;
      }
      delta = 1e-12 * tr / R;
      ridged = 1;
    }
  };
  // T^{-1} = E^T D^{-1} E, stored by columns: Ti[c][y] = sum_i E(i, y)
  // E(i, c) / D_i.  Rows of the pair beyond R hold the last finishing pass's
  // values, so the padding of Ti is written as zero.
  auto ti_entry = [&](int l) __attribute__((always_inline)) {
    constexpr int SP = L::SP;
    const double* Et = reinterpret_cast<const double*>(smem + L::oS);
    const double* EtD = Et + K * SP;
    const int y = l / K, c = l - y * K;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < K; i += 2) {
      const double2 e = *reinterpret_cast<const double2*>(Et + y * SP + i);
      const double2 d = *reinterpret_cast<const double2*>(EtD + c * SP + i);
      a0 = fma(e.x, d.x, a0);
      a1 = fma(e.y, d.y, a1);
    }
    Ti[c * SP + y] = y < R && c < R ? a0 + a1 : 0.0;
  };
  // by all waves (the mode without a big step, where the elimination ends
  // last)
  auto ti_step = [&]() __attribute__((always_inline)) {
    for (int l = t; l < KK; l += NT) ti_entry(l);
    __syncthreads();
  };
  // by waves 0 and 4 beside the small step (H = 0) and the M_n H step
  // (H = 1), in a mode with a big step: wave 0's elimination ends before the
  // big step does, and the two waves share a SIMD that the steps leave idle
  static_assert(K * K <= 512, "two halves of 256 entries");
  auto ti_half = [&](int h) __attribute__((always_inline)) {
    const int u = (wave == 0 ? 0 : 64) + lane;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int l = 256 * h + 128 * r + u;
      if (l < KK) ti_entry(l);
    }
  };
  // Mode n after H_n, MH and Ti, in three passes over all waves.  First the
  // unnormalized Vr = H Ti (the coefficients Vh_n) and P = MH Ti (= M_n Vr,
  // the products U_n^T A_n), stored transposed.  Then the column scales
  // 1 / ||a_c|| with ||a_c||^2 = Vr(:, c)^T P(:, c): row c of 16 lanes sums
  // the products of its row pairs on the DPP network.  Then thread (i, j)
  // writes Gram_n(i, j) = (Vr^T P)(i, j) / (||a_i|| ||a_j||) and entry
  // (i, j) of the normalized Vh_n and V_n.
  auto finish_mode = [&](int n, bool normalize) __attribute__((always_inline)) {
    constexpr int SP = L::SP;
    double* S1 = reinterpret_cast<double*>(smem + L::oS);
    double* S2 = S1 + K * SP;
    for (int l = t; l < KK; l += NT) {
      const int x = l / K, c = l - x * K;
      double v0 = 0.0, v1 = 0.0, p0 = 0.0, p1 = 0.0;
#pragma unroll
      for (int y = 0; y < K; y += 2) {
        const double2 h = *reinterpret_cast<const double2*>(H + x * K + y);
        const double2 m = *reinterpret_cast<const double2*>(MH + x * K + y);
        const double2 tc = *reinterpret_cast<const double2*>(Ti + c * L::SP + y);
        const double t0 = tc.x, t1 = tc.y;
        v0 = fma(h.x, t0, v0);
        v1 = fma(h.y, t1, v1);
        p0 = fma(m.x, t0, p0);
        p1 = fma(m.y, t1, p1);
      }
      S1[c * SP + x] = v0 + v1;
      S2[c * SP + x] = p0 + p1;
    }
    __syncthreads();
    double* sv = reinterpret_cast<double*>(smem + L::oSv);
    {
      const int c = t >> 4, xp = t & 15;
      if (c < K) {   // whole 16-lane rows
        const bool on = xp < K / 2;
        const int x0 = on ? 2 * xp : 0;   // clamped: loads in bounds
        const double2 a = *reinterpret_cast<const double2*>(S1 + c * SP + x0);
        const double2 b = *reinterpret_cast<const double2*>(S2 + c * SP + x0);
        const double d = row_sum16(on ? fma(a.y, b.y, a.x * b.x) : 0.0);
        if (xp == 0) sv[c] = normalize && d > 0.0 ? 1.0 / sqrt(d) : 1.0;
      }
    }
    __syncthreads();
    double* Vh = Vhn(n);
    double* V = Vn(n);
    double* Gn = Gramn(n);
    for (int l = t; l < KK; l += NT) {
      const int i = l / K, j = l - i * K;
      const double* ri = S1 + i * SP;
      const double* pj = S2 + j * SP;
      double g0 = 0.0, g1 = 0.0;
#pragma unroll
      for (int x = 0; x < K; x += 2) {
        const double2 a = *reinterpret_cast<const double2*>(ri + x);
        const double2 b = *reinterpret_cast<const double2*>(pj + x);
        g0 = fma(a.x, b.x, g0);
        g1 = fma(a.y, b.y, g1);
      }
      const double si = sv[i], sj = sv[j];
      Gn[i * K + j] = (g0 + g1) * si * sj;
      Vh[i * K + j] = S1[j * SP + i] * sj;
      V[i * K + j] = S2[j * SP + i] * sj;
    }
    __syncthreads();
  };

  // closed-form fit from H_2 (in H) and the Grams; the same value in every
  // thread
  auto fit_now = [&](double nrm2) __attribute__((always_inline)) -> double {
    const double* V2 = Vn(2);
    const double* G0 = Gramn(0);
    const double* G1 = Gramn(1);
    const double* G2 = Gramn(2);
    double pin = 0.0, pyh = 0.0;
    for (int l = t; l < KK; l += NT) {
      pin = fma(H[l], V2[l], pin);
      pyh += G0[l] * G1[l] * G2[l];
    }
    pin = wave_sum_dpp(pin);
    pyh = wave_sum_dpp(pyh);
    if (lane == 0) {
      red[2 * wave] = pin;
      red[2 * wave + 1] = pyh;
    }
    __syncthreads();
    double inner = 0.0, yh2 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      inner += red[2 * w];
      yh2 += red[2 * w + 1];
    }
    __syncthreads();   // red is rewritten by the next call
    double res2 = nrm2 - 2.0 * inner + yh2;
    res2 = res2 > 0.0 ? res2 : 0.0;
    return 1.0 - sqrt(res2) / sqrt(nrm2);
  };
  // coefficient start: Vh_n = src[n] (dense R_n x R, FP64), V_n = M_n Vh_n,
  // Gram_n = Vh_n^T V_n
  auto coeff_start = [&](bool alt) __attribute__((always_inline)) {
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int Rn = a.Rn[n];
      const double* src = alt ? a.V_alt[n] : a.V_init[n];
      for (int l = t; l < Rn * R; l += NT) {
        const int j = l / R, r = l - j * R;
        Vhn(n)[j * K + r] = src[l];
      }
    }
    __syncthreads();
    for (int item = t; item < 3 * K * RQ; item += NT) {
      const int n = item / (K * RQ), rem = item - n * (K * RQ);
      const int rq = rem % RQ, x = rem / RQ;
      const double* M = Mn(n);
      const double* Vh = Vhn(n);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
      for (int y = 0; y < K; ++y) {
        const double mv = M[x * K + y];
        const double2 v01 = *reinterpret_cast<const double2*>(Vh + y * K + 4 * rq);
        const double2 v23 = *reinterpret_cast<const double2*>(Vh + y * K + 4 * rq + 2);
        a0 = fma(mv, v01.x, a0);
        a1 = fma(mv, v01.y, a1);
        a2 = fma(mv, v23.x, a2);
        a3 = fma(mv, v23.y, a3);
      }
      double* vp = Vn(n) + x * K + 4 * rq;
      *reinterpret_cast<double2*>(vp) = make_double2(a0, a1);
      *reinterpret_cast<double2*>(vp + 2) = make_double2(a2, a3);
    }
    __syncthreads();
    for (int l = t; l < 3 * KK; l += NT) {
      const int n = l / KK, e = l - n * KK;
      const int i = e / K, j = e - i * K;
      const double* Vh = Vhn(n);
      const double* V = Vn(n);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int q = 0; q < K; q += 4) {
        a0 = fma(Vh[q * K + i], V[q * K + j], a0);
        a1 = fma(Vh[(q + 1) * K + i], V[(q + 1) * K + j], a1);
        a2 = fma(Vh[(q + 2) * K + i], V[(q + 2) * K + j], a2);
        a3 = fma(Vh[(q + 3) * K + i], V[(q + 3) * K + j], a3);
      }
      Gramn(n)[i * K + j] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
  };
  // H_2 = G x_1 V_0 x_2 V_1 (the last mode's MTTKRP)
  auto mttkrp_last = [&]() __attribute__((always_inline)) {
    big_step(std::true_type{}, Vn(1));
    small_step(std::false_type{}, Vn(0));
  };

  // ||Yt||^2 = <G, G x_1 M_0 x_2 M_1 x_3 M_2> unless given: W = G x_3 M_2,
  // then the other two modes in place (a thread keeps its whole fibre in
  // registers), then the inner product with G
  double nrm2 = a.normY2;
  if (!(nrm2 >= 0.0)) {
    big_step(std::false_type{}, Mn(2));
#pragma unroll 1
    for (int md = 1; md >= 0; --md) {
      const double* M = Mn(md);
      // fibre along mode md through W[i0][i1][c]: the other position index
      // o and c fixed
      const int step = md == 0 ? KK : K;
      for (int l = t; l < KK; l += NT) {
        const int o = l / K, c = l - o * K;
        const int base = (md == 0 ? o * K : o * KK) + c;
        double f[K];
#pragma unroll
        for (int x = 0; x < K; ++x) f[x] = W[base + x * step];
#pragma unroll
        for (int x = 0; x < K; ++x) {
          double acc = 0.0;
#pragma unroll
          for (int y = 0; y < K; ++y) acc = fma(M[x * K + y], f[y], acc);
          W[base + x * step] = acc;
        }
      }
      __syncthreads();
    }
    double pl = 0.0;
    for (int l = t; l < K * KK; l += NT) {
      const int i0 = l / KK, rem = l - i0 * KK;
      const int i1 = rem / K, i2 = rem - i1 * K;
      pl = fma(static_cast<double>(G[(i0 * K + i1) * GP + i2]), W[l], pl);
    }
    pl = wave_sum_dpp(pl);
    if (lane == 0) red[2 * wave] = pl;
    __syncthreads();
    nrm2 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) nrm2 += red[2 * w];
    __syncthreads();
  }

  // the start: the caller's factors, or the coefficient start (guarded by
  // the HOSVD start when one is given: the caller's is kept only if its fit
  // is at least the HOSVD start's)
  int init_used = 0;
  if (!user) {
    coeff_start(false);
    if (a.V_alt[0]) {
      mttkrp_last();
      const double f_user = fit_now(nrm2);
      coeff_start(true);
      mttkrp_last();
      const double f_hosvd = fit_now(nrm2);
      if (f_user >= f_hosvd) {
        coeff_start(false);
        init_used = 1;
      }
    }
  }

  double fit_prev = 0.0, fit = 0.0;
  int it = 0, converged = 0;
  for (it = 1; it <= a.max_it; ++it) {
    // one copy of each step in the code (the loop over the modes is kept).
    // T_n needs only the other Grams, so wave 0 factors it while waves
    // 1..7 form H_n; the barriers of the two sides pair up (the branch is
    // uniform per wave).
#pragma unroll 1
    for (int n = 0; n < 3; ++n) {
      if (__builtin_amdgcn_readfirstlane(wave) == 0) {
        // in the mode without a big step the small step's barrier is met
        // inside the elimination
        eliminate_T(Gramn(n == 0 ? 1 : 0), Gramn(n == 2 ? 1 : 2), n == 1);
        if (n != 1) {
          __syncthreads();             // the big step's barrier
          ti_half(0);
          __syncthreads();             // the small step's barrier
          ti_half(1);
        }
        __syncthreads();               // the M_n H step's barrier
      } else {
        if (n == 0)
          big_step(std::false_type{}, Vn(2));   // X = G x_3 V_2
        else if (n == 2)
          big_step(std::true_type{}, Vn(1));    // Y = G x_2 V_1
        if (n != 1 && wave == 4) ti_half(0);
        if (n == 0)
          small_step(std::true_type{}, Vn(1));  // H_0 = X x_2 V_1
        else
          small_step(std::false_type{}, Vn(0)); // H_1 = X x_1 V_0, H_2 = Y x_1 V_0
        if (n != 1 && wave == 4) ti_half(1);
        mh_step(Mn(n));
      }
      if (n == 1) ti_step();
      finish_mode(n, n < 2);
    }
    fit = fit_now(nrm2);
    if (t == 0 && a.fit_trace) a.fit_trace[it - 1] = fit;
    if (it >= 2 && fabs(fit - fit_prev) < a.tol) {
      converged = 1;
      break;
    }
    if (it < a.max_it) fit_prev = fit;
  }
  if (it > a.max_it) it = a.max_it;
  // ridged is known to wave 0 only
  __shared__ int ridged_any;
  if (t == 0) ridged_any = ridged;
  __syncthreads();
  // Vh_n (dense R_n x R) and the last Gram for the output kernel
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const int Rn = a.Rn[n];
    for (int l = t; l < Rn * R; l += NT) {
      const int j = l / R, r = l - j * R;
      a.A[n][l] = Vhn(n)[j * K + r];
    }
  }
  for (int l = t; l < R * R; l += NT) {
    const int i = l / R, j = l - i * R;
    a.Gram[2][l] = Gramn(2)[i * K + j];
  }
  if (t == 0 && a.info) {
    InfoDev* info = static_cast<InfoDev*>(a.info);
    info->iterations = it;
    info->converged = converged;
    info->ridged = ridged_any;
    info->init_used = init_used;
    info->fit = fit;
    info->fit_prev = fit_prev;
  }
}

// A_n = U_n Vh_n (rows of the FP32 U_n, Vh_n dense R_n x R in a.A[n]); the
// last factor normalized, lambda = its column norms (from its Gram).
__global__ __launch_bounds__(256) void als_output_kernel(FfcpArgs a_arg) {
  (void)a_arg;
  typedef const __attribute__((address_space(4))) FfcpArgs KArgs;
  KArgs& a = *reinterpret_cast<KArgs*>(
      reinterpret_cast<uintptr_t>(__builtin_amdgcn_kernarg_segment_ptr()));
  const int n = blockIdx.y, R = a.R, Rn = a.Rn[n], last = a.N - 1;
  const int64_t cnt = a.I[n] * R;
  const double* Vh = a.A[n];
  const double* Gl = a.Gram[last];
  const float* Un = a.U[n];
  float* out = a.A_out[n];
  for (int64_t l = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; l < cnt;
       l += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t i = l / R;
    const int r = static_cast<int>(l - i * R);
    double acc = 0.0;
    for (int j = 0; j < Rn; ++j) acc += static_cast<double>(Un[i * Rn + j]) * Vh[j * R + r];
    if (n == last) {
      const double nr = sqrt(Gl[r * R + r]);
      if (nr > 0.0) acc /= nr;
    }
    out[l] = static_cast<float>(acc);
  }
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int r = threadIdx.x; r < R; r += 256) a.lambda[r] = static_cast<float>(sqrt(Gl[r * R + r]));
}

template <int K>
int launch_als3(const FfcpArgs& a, hipStream_t s) {
  constexpr int lds = A3Layout<K>::bytes;
  static_assert(lds + 64 <= kLdsMax, "three-way state in LDS");
  auto k = ffcp_als3_kernel<K>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return hip_fail(e, "ffcp three-way LDS attribute");
  hipLaunchKernelGGL(k, dim3(1), dim3(kA3Threads), static_cast<size_t>(lds), s, a);
  RT_LAUNCH_CHECK("ffcp three-way ALS");
  int64_t imax = 1;
  for (int n = 0; n < a.N; ++n) imax = a.I[n] > imax ? a.I[n] : imax;
  int64_t blocks = (imax * a.R + 255) / 256;
  blocks = blocks < 1024 ? blocks : 1024;
  hipLaunchKernelGGL(als_output_kernel, dim3(static_cast<unsigned>(blocks), a.N), dim3(256),
                     0, s, a);
  RT_LAUNCH_CHECK("ffcp ALS output");
  return kOk;
}

}  // namespace

bool ffcp_als_core_applicable(const FfcpArgs& a) {
  return a.update == 0 && !(a.l1 > 0.0) && a.R <= 64;
}

int launch_ffcp_als_core(const FfcpArgs& a, hipStream_t s) {
  CoreAlsArgs c{};
  c.a = a;
  int kmax = a.R;
  for (int n = 0; n < a.N; ++n) kmax = a.Rn[n] > kmax ? a.Rn[n] : kmax;
  if (a.N == 3 && kmax <= 20) {
    // the tall cross products of the start (M_n = U_n^T U_n, and for a
    // start given as factors U_n^T A_n and A_n^T A_n), then the three-way
    // kernel and the output kernel
    CrossBatch cb{};
    int nb = 0;
    for (int n = 0; n < 3; ++n) {
      cb.X[nb] = a.U[n];
      cb.Y[nb] = a.U[n];
      cb.out[nb] = a.U64[n];
      cb.I[nb] = a.I[n];
      cb.p[nb] = cb.q[nb] = a.Rn[n];
      ++nb;
      if (a.A_init[0]) {
        cb.X[nb] = a.U[n];
        cb.Y[nb] = a.A_init[n];
        cb.out[nb] = a.V[n];
        cb.I[nb] = a.I[n];
        cb.p[nb] = a.Rn[n];
        cb.q[nb] = a.R;
        ++nb;
        cb.X[nb] = a.A_init[n];
        cb.Y[nb] = a.A_init[n];
        cb.out[nb] = a.Gram[n];
        cb.I[nb] = a.I[n];
        cb.p[nb] = cb.q[nb] = a.R;
        ++nb;
      }
    }
    cb.nb = nb;
    RT_TRY(launch_cross_tall(cb, s));
    if (kmax <= 8) return launch_als3<8>(a, s);
    if (kmax <= 16) return launch_als3<16>(a, s);
    return launch_als3<20>(a, s);
  }
  if (a.R <= 16) return launch_r<16, 512>(c, s);
  if (a.R <= 20) return launch_r<20, 512>(c, s);
  if (a.R <= 24) return launch_r<24, 512>(c, s);
  if (a.R <= 32) return launch_r<32, 512>(c, s);
  return launch_r<64, 512>(c, s);
}

}  // namespace rt
