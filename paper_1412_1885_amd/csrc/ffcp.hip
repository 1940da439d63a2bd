// FFCP (Algorithm 1, Section III-B) on a Tucker format [[G; U]].
//
// The whole iteration loop runs inside one workgroup of 512 threads: every
// step is a small dense operation (R <= 64, R_n <= 64, the core has at most
// a few 10^5 entries) so the loop is latency bound, and keeping it on the
// device removes every launch and host round trip; the stopping test is
// evaluated on the device too.  Arithmetic is FP64: the stopping rule
// compares fits to 1e-6..1e-9, and the closed-form fit cancels
// ||Yt||^2 - 2<Yt,Yhat> + ||Yhat||^2, so its inputs need FP64 accumulation.
//
// Per iteration, for n = 0..N-1:
//   H   = G_(n) [KR_{p != n} V_p]            eq. (12)-(13), contracted one
//                                            mode at a time, last mode first
//   Q   = U_n H
//   T   = hadamard_{p != n} Gram_p          eq. (9)
//   A_n <- ALS (Cholesky solve of A T = Q, eq. (14)) | HALS (eq. (8), standard
//          form) | MU (eq. (15));  optional soft threshold S_c (eq. (16))
//   normalize columns if n < N-1;  V_n = U_n^T A_n;  Gram_n = A_n^T A_n
// then Fit = 1 - sqrt(||Yt||^2 - 2 sum(H_{N-1} * V_{N-1}) + 1^T(had Gram)1)
//            / ||Yt||.
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kFThreads = 512;
constexpr int kFWaves = kFThreads / 64;
constexpr int kRMax = 64;

struct InfoDev {
  int32_t iterations, converged, ridged, init_used;
  double fit, fit_prev;
};

__device__ __forceinline__ void bsync() { __syncthreads(); }

// Cross products of row-major FP64 matrices with packed rows:
//   out[a * q + b] = sum_i X[i * p + a] Y[i * q + b]   (a < p, b < q),
// or only the diagonal out[a] (diag; X = Y, p = q), over `rows` rows; with
// out2, also out2[a * q + b] = sum_i Y[i * q + a] Y[i * q + b] from the same
// staged rows (one pass over Y for U^T A and A^T A).
// One workgroup does it, so the cost is the number of dependent memory
// round trips: the rows go through LDS in blocks as large as the staging
// buffer holds (st: kXtyStage doubles; B rows of X and Y, one copy when
// X = Y), which the threads load with consecutive addresses (B p and B q
// contiguous doubles), about 16 loads in flight per thread.  When there are
// fewer outputs than threads, the threads form G = threads / outputs groups
// that take every G-th row of a block; the G partial sums of an output are
// added in group order at the end.  Every output is a sum in a fixed order:
// deterministic.
// KOUT bounds the outputs per thread: nout <= KOUT * threads.
constexpr int kXtyStage = 2 * 64 * kRMax;            // doubles (64 KB)

template <int KOUT>
__device__ void block_xty(const double* X, const double* Y, int64_t rows, int p,
                          int q, bool diag, double* out, double* st,
                          double* out2 = nullptr) {
  const int t = threadIdx.x;
  const bool same = X == Y;
  const int w = same ? p : p + q;              // staged doubles per row
  const int B = kXtyStage / w;                 // rows per block (>= 64)
  const int nout1 = diag ? p : p * q;
  const int nout = nout1 + (out2 ? q * q : 0);
  const int G = nout < kFThreads ? kFThreads / nout : 1;
  const int g = t / (nout < kFThreads ? nout : kFThreads);   // this thread's group
  double acc[KOUT];
#pragma unroll
  for (int u = 0; u < KOUT; ++u) acc[u] = 0.0;
  for (int64_t i0 = 0; i0 < rows; i0 += B) {
    const int nb = static_cast<int>(rows - i0 < B ? rows - i0 : B);
    const int nx = nb * p, ny = same ? 0 : nb * q;
    double* sY = same ? st : st + nx;
    const int64_t xb = i0 * p, yb = i0 * q;
    for (int e = t; e < nx + ny; e += kFThreads) {
      st[e] = e < nx ? X[xb + e] : Y[yb + (e - nx)];
    }
    bsync();
    // sum over rows g, g + G, ... of the block for output o (X or Y first)
    auto dot = [&](int o, bool batched) __attribute__((always_inline)) -> double {
      const bool two = o >= nout1;
      const int oo = two ? o - nout1 : o;
      const double* sA = two ? sY : st;
      const int pa = two ? q : p;
      const int ia = diag ? oo : oo / q, ib = diag ? oo : oo % q;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int i = g;
      if (batched) {
        // 8 rows' operands read from LDS before their products, so the
        // reads overlap instead of each waiting on the previous sum
        for (; i + 7 * G < nb; i += 8 * G) {
          double xa[8], yb[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            xa[k] = sA[(i + k * G) * pa + ia];
            yb[k] = sY[(i + k * G) * q + ib];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) s4[k & 3] += xa[k] * yb[k];
        }
      }
      for (; i < nb; i += G) s4[0] += sA[i * pa + ia] * sY[i * q + ib];
      return (s4[0] + s4[1]) + (s4[2] + s4[3]);
    };
    if (g < G) {
      if (G > 1) {
        acc[0] += dot(t - g * nout, true);   // one output per thread
      } else {
#pragma unroll
        for (int u = 0; u < KOUT; ++u) {
          const int o = t + u * kFThreads;
          if (o < nout) acc[u] += dot(o, false);
        }
      }
    }
    bsync();
  }
  if (G > 1) {
    // partial sums of the groups, added in group order
    if (g < G) st[g * nout + (t - g * nout)] = acc[0];
    bsync();
    for (int o = t; o < nout; o += kFThreads) {
      double v = 0.0;
      for (int k = 0; k < G; ++k) v += st[k * nout + o];
      if (o < nout1) out[o] = v; else out2[o - nout1] = v;
    }
    bsync();
  } else {
#pragma unroll
    for (int u = 0; u < KOUT; ++u) {
      const int o = t + u * kFThreads;
      if (o < nout1) out[o] = acc[u];
      else if (o < nout) out2[o - nout1] = acc[u];
    }
  }
}

// Mode product of a core by a square FP64 matrix M (S x S) in mode m:
// out[a, i, c] = sum_j X[a, j, c] M[j, i].
__device__ void core_ttm_sq(const double* X, double* out, const double* M,
                            int64_t Apre, int S, int64_t Cpost) {
  const int64_t total = Apre * S * Cpost;
  for (int64_t l = threadIdx.x; l < total; l += kFThreads) {
    int64_t c = l % Cpost;
    int64_t t = l / Cpost;
    int i = static_cast<int>(t % S);
    int64_t a = t / S;
    double acc = 0.0;
    for (int j = 0; j < S; ++j) acc += X[(a * S + j) * Cpost + c] * M[j * S + i];
    out[l] = acc;
  }
}

template <int RMAX>
__global__ __launch_bounds__(kFThreads) void ffcp_kernel(FfcpArgs a) {
  __shared__ double Ts[kRMax * kRMax];   // T, then its Cholesky factor
  __shared__ double st[kXtyStage];   // block_xty staging
  // outputs per thread of the fused U^T A, A^T A pass (R_n <= 64, R <= RMAX)
  constexpr int kVgOut = (kRMax * RMAX + RMAX * RMAX + kFThreads - 1) / kFThreads;
  __shared__ double red[kFWaves];
  __shared__ double sh[8];
  __shared__ int shi[4];
  const int t = threadIdx.x;
  const int N = a.N, R = a.R;
  InfoDev* info = static_cast<InfoDev*>(a.info);

  // ---- setup: FP64 copies of U, G; A from the initialization -------------
  int64_t coreSize = 1;
  for (int n = 0; n < N; ++n) coreSize *= a.Rn[n];
  for (int n = 0; n < N; ++n) {
    const int64_t cnt = a.I[n] * a.Rn[n];
    for (int64_t l = t; l < cnt; l += kFThreads) a.U64[n][l] = a.U[n][l];
  }
  for (int64_t l = t; l < coreSize; l += kFThreads) a.G64[l] = a.G[l];
  bsync();
  for (int n = 0; n < N; ++n) {
    const int64_t cnt = a.I[n] * R;
    if (a.A_init[n]) {
      for (int64_t l = t; l < cnt; l += kFThreads) a.A[n][l] = a.A_init[n][l];
    } else {  // A = U V_init
      for (int64_t l = t; l < cnt; l += kFThreads) {
        int64_t i = l / R;
        int r = static_cast<int>(l % R);
        double acc = 0.0;
        for (int j = 0; j < a.Rn[n]; ++j)
          acc += a.U64[n][i * a.Rn[n] + j] * a.V_init[n][j * R + r];
        a.A[n][l] = acc;
      }
    }
  }
  bsync();
  for (int n = 0; n < N; ++n) {
    const int Rn = a.Rn[n];
    const double* Un = a.U64[n];
    const double* An = a.A[n];
    block_xty<kVgOut>(Un, An, a.I[n], Rn, R, false, a.V[n], st, a.Gram[n]);
  }
  bsync();

  // ---- ||Yt||^2 = <G, G x_n U_n^T U_n> unless given ----------------------
  double nrm2 = a.normY2;
  if (!(nrm2 >= 0.0)) {
    // UtU_n into W2 (packed), G' chain in W1 <-> Qm buffers
    double* src = a.G64;
    double* bufs[2] = {a.W1, a.W2};
    int cur = 0;
    int64_t Apre = 1;
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      int64_t Cpost = coreSize / (Apre * Rn);
      // UtU in Ts (Rn <= 64)
      block_xty<kRMax * kRMax / kFThreads>(a.U64[n], a.U64[n], a.I[n], Rn, Rn, false,
                                            a.H, st);
      bsync();
      core_ttm_sq(src, bufs[cur], a.H, Apre, Rn, Cpost);
      bsync();
      src = bufs[cur];
      cur ^= 1;
      Apre *= Rn;
    }
    double p = 0.0;
    for (int64_t l = t; l < coreSize; l += kFThreads) p += a.G64[l] * src[l];
    nrm2 = block_sum(p, red);
    bsync();
  }

  // ---- iterations ---------------------------------------------------------
  double fit_prev = 0.0, fit = 0.0;
  int it = 0, converged = 0, ridged = 0;
  double inner = 0.0;
  for (it = 1; it <= a.max_it; ++it) {
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      const int64_t In = a.I[n];
      // H = G_(n) [KR_{p != n} V_p]: contract the last remaining mode != n
      int rem[8], nrem = N;
      for (int p = 0; p < N; ++p) rem[p] = p;
      const double* src = a.G64;
      double* bufs[2] = {a.W1, a.W2};
      int cur = 0;
      bool first = true;
      while (nrem > 1) {
        int pos = nrem - 1;
        if (rem[pos] == n) pos = nrem - 2;
        const int m = rem[pos];
        int64_t Apre = 1, Cpost = 1;
        for (int q = 0; q < pos; ++q) Apre *= a.Rn[rem[q]];
        for (int q = pos + 1; q < nrem; ++q) Cpost *= a.Rn[rem[q]];
        const int Rm = a.Rn[m];
        const double* Vm = a.V[m];
        double* dst = bufs[cur];
        const int64_t total = Apre * Cpost * R;
        for (int64_t l = t; l < total; l += kFThreads) {
          const int r = static_cast<int>(l % R);
          const int64_t ac = l / R;
          const int64_t c = ac % Cpost, aa = ac / Cpost;
          double acc = 0.0;
          if (first) {
            for (int j = 0; j < Rm; ++j)
              acc += src[(aa * Rm + j) * Cpost + c] * Vm[j * R + r];
          } else {
            for (int j = 0; j < Rm; ++j)
              acc += src[((aa * Rm + j) * Cpost + c) * R + r] * Vm[j * R + r];
          }
          dst[l] = acc;
        }
        bsync();
        for (int q = pos; q < nrem - 1; ++q) rem[q] = rem[q + 1];
        --nrem;
        src = dst;
        cur ^= 1;
        first = false;
      }
      const double* H = src;  // Rn x R
      // Q = U_n H: H staged in LDS, one thread per row of Q; the row of U_n
      // is loaded 16 values at a time, so a row costs ceil(R_n / 16) memory
      // round trips
      double* Qm = a.Qm;
      for (int l = t; l < Rn * R; l += kFThreads) st[l] = H[l];
      bsync();
      for (int64_t i = t; i < In; i += kFThreads) {
        double acc[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) acc[r] = 0.0;
        const double* urow = a.U64[n] + i * Rn;
        for (int j0 = 0; j0 < Rn; j0 += 16) {
          double uv[16];
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) uv[jj] = j0 + jj < Rn ? urow[j0 + jj] : 0.0;
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) {
            if (j0 + jj < Rn) {
#pragma unroll
              for (int r = 0; r < RMAX; ++r)
                if (r < R) acc[r] += uv[jj] * st[(j0 + jj) * R + r];
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RMAX; ++r)
          if (r < R) Qm[i * R + r] = acc[r];
      }
      // T = hadamard of the other Grams
      for (int l = t; l < R * R; l += kFThreads) {
        double v = 1.0;
        for (int p = 0; p < N; ++p)
          if (p != n) v *= a.Gram[p][l];
        Ts[l] = v;
      }
      if (n == N - 1) {
        // keep H of the last mode for the fit (copy before buffers reuse)
        for (int l = t; l < Rn * R; l += kFThreads) a.H[l] = H[l];
      }
      bsync();
      double* An = a.A[n];
      if (a.update == 0) {
        // ---- ALS: Cholesky of T (in place, lower), ridge on failure ------
        for (int attempt = 0; attempt < 2; ++attempt) {
          if (attempt == 1) {
            // rebuild T + delta I
            double tr = 0.0;
            for (int l = 0; l < R; ++l) {
              double v = 1.0;
              for (int p = 0; p < N; ++p)
                if (p != n) v *= a.Gram[p][l * R + l];
              tr += v;
            }
            const double delta = 1e-12 * tr / R;
            bsync();
            for (int l = t; l < R * R; l += kFThreads) {
              double v = 1.0;
              for (int p = 0; p < N; ++p)
                if (p != n) v *= a.Gram[p][l];
              if (l / R == l % R) v += delta;
              Ts[l] = v;
            }
            bsync();
          }
          if (t == 0) shi[0] = 0;
          bsync();
          for (int k = 0; k < R; ++k) {
            if (t == 0) {
              double d = Ts[k * R + k];
              if (!(d > 0.0)) {
                shi[0] = 1;
                d = 1.0;
              }
              Ts[k * R + k] = sqrt(d);
            }
            bsync();
            const double dk = Ts[k * R + k];
            for (int i = k + 1 + t; i < R; i += kFThreads) Ts[i * R + k] /= dk;
            bsync();
            const int rem2 = R - k - 1;
            for (int l = t; l < rem2 * rem2; l += kFThreads) {
              const int i = k + 1 + l / rem2, j = k + 1 + l % rem2;
              if (j <= i) Ts[i * R + j] -= Ts[i * R + k] * Ts[j * R + k];
            }
            bsync();
          }
          const int failed = shi[0];
          bsync();
          if (!failed) break;
          ridged = 1;
        }
        // solve A_n[i,:] L L^T = Q[i,:] row by row
        for (int64_t i = t; i < In; i += kFThreads) {
          double y[RMAX];
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            if (r < R) {
              double s = Qm[i * R + r];
              for (int q = 0; q < r; ++q) s -= Ts[r * R + q] * y[q];
              y[r] = s / Ts[r * R + r];
            }
          }
#pragma unroll
          for (int r = RMAX - 1; r >= 0; --r) {
            if (r < R) {
              double s = y[r];
              for (int q = r + 1; q < R; ++q) s -= Ts[q * R + r] * y[q];
              y[r] = s / Ts[r * R + r];
            }
          }
#pragma unroll
          for (int r = 0; r < RMAX; ++r)
            if (r < R) An[i * R + r] = y[r];
        }
      } else if (a.update == 1) {
        // ---- HALS: columns in order, in place per row --------------------
        for (int64_t i = t; i < In; i += kFThreads) {
          double row[RMAX], qrow[RMAX];   // both rows loaded before any use
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            row[r] = (r < R) ? An[i * R + r] : 0.0;
            qrow[r] = (r < R) ? Qm[i * R + r] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            if (r < R) {
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < RMAX; ++q)
                if (q < R) s += row[q] * Ts[q * R + r];
              double v = row[r] + (qrow[r] - s) / Ts[r * R + r];
              row[r] = v > 1e-16 ? v : 1e-16;
            }
          }
#pragma unroll
          for (int r = 0; r < RMAX; ++r)
            if (r < R) An[i * R + r] = row[r];
        }
      } else {
        // ---- MU: A <- A * max(Q,0) / (A T + eps) -------------------------
        for (int64_t i = t; i < In; i += kFThreads) {
          double row[RMAX];
#pragma unroll
          for (int r = 0; r < RMAX; ++r) row[r] = (r < R) ? An[i * R + r] : 0.0;
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            if (r < R) {
              double s = 0.0;
#pragma unroll
              for (int q = 0; q < RMAX; ++q)
                if (q < R) s += row[q] * Ts[q * R + r];
              double qv = Qm[i * R + r];
              An[i * R + r] = row[r] * (qv > 0.0 ? qv : 0.0) / (s + 1e-16);
            }
          }
        }
      }
      bsync();
      if (a.l1 > 0.0) {
        // sparsity step S_c of eq. (16); under HALS the result goes back onto
        // the feasible set a >= 1e-16 so that no column (and no t_rr) vanishes
        const double c = a.l1;
        const double lo = a.update == 1 ? 1e-16 : -INFINITY;
        for (int64_t l = t; l < In * R; l += kFThreads) {
          const double x = An[l];
          const double y = x > c ? x - c : (x < -c ? x + c : 0.0);
          An[l] = y > lo ? y : lo;
        }
        bsync();
      }
      if (n < N - 1) {
        block_xty<1>(An, An, In, R, R, true, a.scal + 8, st);
        bsync();
        // column norms in LDS; 8 elements per thread and step, loads first
        for (int r = t; r < R; r += kFThreads) st[r] = sqrt(a.scal[8 + r]);
        bsync();
        const int64_t cnt = In * R;
        for (int64_t l0 = t; l0 < cnt; l0 += 8 * kFThreads) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int64_t l = l0 + u * kFThreads;
            v[u] = l < cnt ? An[l] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int64_t l = l0 + u * kFThreads;
            const double nr = st[l % R];
            if (l < cnt && nr > 0.0) An[l] = v[u] / nr;
          }
        }
        bsync();
      }
      block_xty<kVgOut>(a.U64[n], An, In, Rn, R, false, a.V[n], st, a.Gram[n]);
      bsync();
    }
    // ---- fit ----------------------------------------------------------------
    {
      double p = 0.0;
      const int Rl = a.Rn[N - 1];
      for (int l = t; l < Rl * R; l += kFThreads) p += a.H[l] * a.V[N - 1][l];
      inner = block_sum(p, red);
      double q = 0.0;
      for (int l = t; l < R * R; l += kFThreads) {
        double v = 1.0;
        for (int pp = 0; pp < N; ++pp) v *= a.Gram[pp][l];
        q += v;
      }
      const double yh2 = block_sum(q, red);
      double res2 = nrm2 - 2.0 * inner + yh2;
      res2 = res2 > 0.0 ? res2 : 0.0;
      fit = 1.0 - sqrt(res2) / sqrt(nrm2);
    }
    if (t == 0 && a.fit_trace) a.fit_trace[it - 1] = fit;
    if (it >= 2 && fabs(fit - fit_prev) < a.tol) {
      converged = 1;
      break;
    }
    if (it < a.max_it) fit_prev = fit;
    bsync();
  }
  if (it > a.max_it) it = a.max_it;
  bsync();
  // ---- outputs --------------------------------------------------------------
  for (int n = 0; n < N - 1; ++n) {
    const int64_t cnt = a.I[n] * R;
    for (int64_t l = t; l < cnt; l += kFThreads)
      a.A_out[n][l] = static_cast<float>(a.A[n][l]);
  }
  {
    const int n = N - 1;
    const double* An = a.A[n];
    block_xty<1>(An, An, a.I[n], R, R, true, a.scal + 8, st);
    bsync();
    const int64_t cnt = a.I[n] * R;
    for (int64_t l = t; l < cnt; l += kFThreads) {
      const double nr = sqrt(a.scal[8 + l % R]);
      a.A_out[n][l] = static_cast<float>(nr > 0.0 ? An[l] / nr : An[l]);
    }
    for (int r = t; r < R; r += kFThreads)
      a.lambda[r] = static_cast<float>(sqrt(a.scal[8 + r]));
  }
  if (t == 0 && info) {
    info->iterations = it;
    info->converged = converged;
    info->ridged = ridged;
    info->init_used = 0;
    info->fit = fit;
    info->fit_prev = fit_prev;
  }
}

}  // namespace

int launch_ffcp(const FfcpArgs& a, hipStream_t s) {
  if (a.R <= 16) {
    hipLaunchKernelGGL(ffcp_kernel<16>, dim3(1), dim3(kFThreads), 0, s, a);
  } else if (a.R <= 32) {
    hipLaunchKernelGGL(ffcp_kernel<32>, dim3(1), dim3(kFThreads), 0, s, a);
  } else if (a.R <= 64) {
    hipLaunchKernelGGL(ffcp_kernel<64>, dim3(1), dim3(kFThreads), 0, s, a);
  } else {
    set_error("ffcp: R=%d exceeds 64", a.R);
    return kErrUnsupported;
  }
  RT_LAUNCH_CHECK("ffcp");
  return kOk;
}

}  // namespace rt
