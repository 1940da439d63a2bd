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

// ---------------------------------------------------------------------------
// The same iteration over the whole chip, for large I_n (the 10^4-per-mode
// workload of Section V-A): one cooperative launch of G workgroups (at most
// one per CU, all resident), grid-wide barriers between the steps that need
// every row.
//   * I_n-sized steps: the rows of each mode are split into G contiguous
//     chunks, one per workgroup.  A row's Q = U_n H and its update (ALS /
//     HALS / MU, soft threshold) need only that row, so they run back to
//     back without a barrier (Q is never written out).
//   * Cross products over the rows (U_n^T A_n, A_n^T A_n, column norms,
//     U_n^T U_n): each workgroup sums its chunk (the single-workgroup code),
//     the partials go to global memory, and after a barrier every output is
//     the sum of the G partials in workgroup order: deterministic, and the
//     same in every workgroup.
//   * Core-sized steps (the MTTKRP chain through the core) are spread over
//     all threads of the grid, one barrier per contracted mode; the R x R
//     steps (T, its Cholesky factor) are repeated in every workgroup from
//     the same data.
//   * The fit and the stopping decision are made by workgroup 0 and
//     broadcast through global memory behind a barrier, so every workgroup
//     leaves the loop at the same iteration.
constexpr int kGridMax = 256;        // workgroups of the cooperative launch (partials' rows)
constexpr int kGridMinRows = 2048;   // below this the single-workgroup kernel is used
constexpr int kGridRows = 128;       // rows of the longest mode per workgroup
constexpr unsigned kSpinLimit = 1u << 24;

// Grid-wide barrier of the cooperative launch (every workgroup resident):
// after the workgroup's barrier, thread 0 counts the arrival in bar[0] with
// an agent-scope release (the L2 write-back that makes this workgroup's
// stores visible to the other XCDs) and polls bar[0] with acquire loads
// until all G workgroups of this phase have arrived.  The poll is bounded:
// after kSpinLimit polls bar[1] records the failure and the workgroup goes
// on, so the kernel always finishes; the host reports it.  (The runtime's
// cooperative-groups grid barrier took 9-27 us at 79-256 workgroups, this one
// 3-7.5 us.)
struct GridCtx {
  unsigned* bar;
  int G, wg;
  int64_t gtid, gthreads;
  unsigned phase;
  __device__ void sync() {
    __syncthreads();
    ++phase;
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = phase * static_cast<unsigned>(G);
      unsigned n = 0;
      while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++n > kSpinLimit) {
          __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __syncthreads();
  }
};

// rows [r0, r1) of this workgroup for a mode of I rows
__device__ __forceinline__ void grid_rows(const GridCtx& g, int64_t I, int64_t& r0, int64_t& r1) {
  const int64_t per = (I + g.G - 1) / g.G;
  r0 = g.wg * per;
  r1 = r0 + per < I ? r0 + per : I;
  if (r0 > I) r0 = I;
}

// out (p x q, or its diagonal) [and out2 = Y^T Y] over all rows: chunk
// partials, a barrier, the fixed-order sum of the G partials spread over the
// grid, a barrier
template <int KOUT>
__device__ void grid_xty(GridCtx& g, const double* X, const double* Y, int64_t rows,
                         int p, int q, bool diag, double* out, double* st, double* part,
                         double* out2 = nullptr) {
  const int nout1 = diag ? p : p * q;
  const int nout = nout1 + (out2 ? q * q : 0);
  int64_t r0, r1;
  grid_rows(g, rows, r0, r1);
  double* mine = part + static_cast<int64_t>(g.wg) * nout;
  block_xty<KOUT>(X + r0 * p, Y + r0 * q, r1 - r0, p, q, diag, mine, st,
                  out2 ? mine + nout1 : nullptr);
  g.sync();
  // one wavefront per output: lane l adds the partials of workgroups
  // l, l + 64, ... in order, then the lanes are summed in a fixed tree
  const int lane = threadIdx.x & 63;
  const int64_t wave = g.gtid >> 6, nwaves = g.gthreads >> 6;
  for (int64_t o = wave; o < nout; o += nwaves) {
    double v = 0.0;
    for (int w = lane; w < g.G; w += 64) v += part[static_cast<int64_t>(w) * nout + o];
    v = wave_sum(v);
    if (lane == 0) {
      if (o < nout1) out[o] = v; else out2[o - nout1] = v;
    }
  }
  g.sync();
}

// V_n = U_n^T A_n and Gram_n = A_n^T A_n of the factor with unit columns,
// from its rows as stored (not normalized): per-workgroup partials of U^T A
// and A^T A, a barrier, then each output summed over the workgroups (one
// wavefront per output, fixed order) and divided by the column norms, which
// the same wavefront takes from the sums of the diagonal entries it needs.
// The norms go to nr (R values; ones when normalize is false).  The rows are
// divided by them where they are read next.
template <int KOUT>
__device__ void grid_vg(GridCtx& g, const double* U, const double* A, int64_t rows, int p,
                        int q, bool normalize, double* V, double* Gram, double* nr, double* st,
                        double* part) {
  const int nout1 = p * q;
  const int nout = nout1 + q * q;
  int64_t r0, r1;
  grid_rows(g, rows, r0, r1);
  double* mine = part + static_cast<int64_t>(g.wg) * nout;
  block_xty<KOUT>(U + r0 * p, A + r0 * q, r1 - r0, p, q, false, mine, st, mine + nout1);
  g.sync();
  const int lane = threadIdx.x & 63;
  const int64_t wave = g.gtid >> 6, nwaves = g.gthreads >> 6;
  auto total = [&](int o) __attribute__((always_inline)) {
    double v = 0.0;
    for (int w = lane; w < g.G; w += 64) v += part[static_cast<int64_t>(w) * nout + o];
    return wave_sum(v);
  };
  for (int64_t o = wave; o < nout; o += nwaves) {
    const double v = total(static_cast<int>(o));
    const bool isV = o < nout1;
    const int rr = isV ? static_cast<int>(o % q) : static_cast<int>((o - nout1) / q);
    const int cc = isV ? rr : static_cast<int>((o - nout1) % q);
    double s1 = 1.0, s2 = 1.0;
    if (normalize) {
      s1 = sqrt(total(nout1 + rr * q + rr));
      s2 = isV ? 1.0 : (cc == rr ? s1 : sqrt(total(nout1 + cc * q + cc)));
      s1 = s1 > 0.0 ? s1 : 1.0;
      s2 = s2 > 0.0 ? s2 : 1.0;
    }
    if (lane == 0) {
      if (isV) {
        V[o] = v / s1;
      } else {
        Gram[o - nout1] = v / (s1 * s2);
        if (rr == cc) nr[rr] = s1;
      }
    }
  }
  g.sync();
}

// Row i of mode n: q = U_n[i,:] H (H staged in LDS, R_n x R), then the
// update of A_n[i,:] (ALS: the Cholesky factor of T in Ts; HALS, MU: T in
// Ts) and the soft threshold of eq. (16).  Only row i is read and written.
template <int RMAX>
__device__ __forceinline__ void update_row(const FfcpArgs& a, int n, int64_t i, int Rn, int R,
                                           const double* Hs, const double* Ts,
                                           const double* nr_old) {
  double* An = a.A[n];
  const double c1 = a.l1;
  const double lo = a.update == 1 ? 1e-16 : -INFINITY;
  double q[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) q[r] = 0.0;
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
          if (r < R) q[r] += uv[jj] * Hs[(j0 + jj) * R + r];
      }
    }
  }
  double row[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) row[r] = 0.0;
  if (a.update == 0) {
    // A_n[i,:] L L^T = Q[i,:]
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < R) {
        double s = q[r];
        for (int qq = 0; qq < r; ++qq) s -= Ts[r * R + qq] * row[qq];
        row[r] = s / Ts[r * R + r];
      }
    }
#pragma unroll
    for (int r = RMAX - 1; r >= 0; --r) {
      if (r < R) {
        double s = row[r];
        for (int qq = r + 1; qq < R; ++qq) s -= Ts[qq * R + r] * row[qq];
        row[r] = s / Ts[r * R + r];
      }
    }
  } else if (a.update == 1) {
    // HALS: columns in order, in place (the old row normalized)
#pragma unroll
    for (int r = 0; r < RMAX; ++r) row[r] = (r < R) ? An[i * R + r] / nr_old[r] : 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < R) {
        double s = 0.0;
#pragma unroll
        for (int qq = 0; qq < RMAX; ++qq)
          if (qq < R) s += row[qq] * Ts[qq * R + r];
        const double v = row[r] + (q[r] - s) / Ts[r * R + r];
        row[r] = v > 1e-16 ? v : 1e-16;
      }
    }
  } else {
    // MU: A <- A * max(Q,0) / (A T + eps), from the old (normalized) row
    double old[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) old[r] = (r < R) ? An[i * R + r] / nr_old[r] : 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < R) {
        double s = 0.0;
#pragma unroll
        for (int qq = 0; qq < RMAX; ++qq)
          if (qq < R) s += old[qq] * Ts[qq * R + r];
        row[r] = old[r] * (q[r] > 0.0 ? q[r] : 0.0) / (s + 1e-16);
      }
    }
  }
  if (c1 > 0.0) {
    // sparsity step S_c of eq. (16); under HALS back onto a >= 1e-16
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const double x = row[r];
      const double y = x > c1 ? x - c1 : (x < -c1 ? x + c1 : 0.0);
      row[r] = y > lo ? y : lo;
    }
  }
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    if (r < R) An[i * R + r] = row[r];
}

template <int RMAX>
__global__ __launch_bounds__(kFThreads) void ffcp_grid_kernel(FfcpArgs a) {
  __shared__ double Ts[kRMax * kRMax];   // T, then its Cholesky factor
  __shared__ double st[kXtyStage];       // chunk staging; H of the mode
  constexpr int kVgOut = (kRMax * RMAX + RMAX * RMAX + kFThreads - 1) / kFThreads;
  __shared__ double red[kFWaves];
  __shared__ int shi[4];
  GridCtx g{a.bar, static_cast<int>(gridDim.x), static_cast<int>(blockIdx.x),
            static_cast<int64_t>(blockIdx.x) * kFThreads + threadIdx.x,
            static_cast<int64_t>(gridDim.x) * kFThreads, 0u};
  const int t = threadIdx.x;
  const int N = a.N, R = a.R;
  InfoDev* info = static_cast<InfoDev*>(a.info);
  double* part = a.part;
  double* bcast = a.scal;   // [0] fit, [1] stop flag, [2] ||Yt||^2 (workgroup 0 writes)

  // ---- setup: FP64 copies of U, G; A from the initialization -------------
  int64_t coreSize = 1;
  for (int n = 0; n < N; ++n) coreSize *= a.Rn[n];
  for (int n = 0; n < N; ++n) {
    const int64_t cnt = a.I[n] * a.Rn[n];
    for (int64_t l = g.gtid; l < cnt; l += g.gthreads) a.U64[n][l] = a.U[n][l];
  }
  for (int64_t l = g.gtid; l < coreSize; l += g.gthreads) a.G64[l] = a.G[l];
  g.sync();
  for (int n = 0; n < N; ++n) {
    const int64_t cnt = a.I[n] * R;
    if (a.A_init[n]) {
      for (int64_t l = g.gtid; l < cnt; l += g.gthreads) a.A[n][l] = a.A_init[n][l];
    } else {  // A = U V_init
      for (int64_t l = g.gtid; l < cnt; l += g.gthreads) {
        const int64_t i = l / R;
        const int r = static_cast<int>(l % R);
        double acc = 0.0;
        for (int j = 0; j < a.Rn[n]; ++j)
          acc += a.U64[n][i * a.Rn[n] + j] * a.V_init[n][j * R + r];
        a.A[n][l] = acc;
      }
    }
  }
  g.sync();
  // V_n, Gram_n of the start (not normalized: its norms are ones)
  for (int n = 0; n < N; ++n)
    grid_vg<kVgOut>(g, a.U64[n], a.A[n], a.I[n], a.Rn[n], R, false, a.V[n], a.Gram[n],
                    a.nrm + n * R, st, part);

  // ---- ||Yt||^2 = <G, G x_n U_n^T U_n> unless given ----------------------
  double nrm2 = a.normY2;
  if (!(nrm2 >= 0.0)) {
    double* src = a.G64;
    double* bufs[2] = {a.W1, a.W2};
    int cur = 0;
    int64_t Apre = 1;
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      const int64_t Cpost = coreSize / (Apre * Rn);
      grid_xty<kRMax * kRMax / kFThreads>(g, a.U64[n], a.U64[n], a.I[n], Rn, Rn, false,
                                          a.H, st, part);
      // out[a, i, c] = sum_j src[a, j, c] UtU[j, i], spread over the grid
      const int64_t total = Apre * Rn * Cpost;
      for (int64_t l = g.gtid; l < total; l += g.gthreads) {
        const int64_t c = l % Cpost, tt = l / Cpost;
        const int i = static_cast<int>(tt % Rn);
        const int64_t aa = tt / Rn;
        double acc = 0.0;
        for (int j = 0; j < Rn; ++j) acc += src[(aa * Rn + j) * Cpost + c] * a.H[j * Rn + i];
        bufs[cur][l] = acc;
      }
      g.sync();
      src = bufs[cur];
      cur ^= 1;
      Apre *= Rn;
    }
    if (g.wg == 0) {
      double p = 0.0;
      for (int64_t l = t; l < coreSize; l += kFThreads) p += a.G64[l] * src[l];
      p = block_sum(p, red);
      if (t == 0) bcast[2] = p;
    }
    g.sync();
    nrm2 = bcast[2];
  }

  // ---- iterations ---------------------------------------------------------
  double fit_prev = 0.0, fit = 0.0;
  int it = 0, converged = 0, ridged = 0;
  for (it = 1; it <= a.max_it; ++it) {
    for (int n = 0; n < N; ++n) {
      const int Rn = a.Rn[n];
      const int64_t In = a.I[n];
      // H = G_(n) [KR_{p != n} V_p]: contract the last remaining mode != n.
      // The first step (core-sized) is spread over the grid, the later ones
      // (each R_m times smaller) are repeated in every workgroup's LDS when
      // they fit half of the staging buffer: no barrier after them.
      int rem[8], nrem = N;
      for (int p = 0; p < N; ++p) rem[p] = p;
      const double* src = a.G64;
      double* bufs[2] = {a.W1, a.W2};
      int cur = 0, step = 0;
      while (nrem > 1) {
        int pos = nrem - 1;
        if (rem[pos] == n) pos = nrem - 2;
        const int m = rem[pos];
        int64_t Apre = 1, Cpost = 1;
        for (int q = 0; q < pos; ++q) Apre *= a.Rn[rem[q]];
        for (int q = pos + 1; q < nrem; ++q) Cpost *= a.Rn[rem[q]];
        const int Rm = a.Rn[m];
        const double* Vm = a.V[m];
        const int64_t total = Apre * Cpost * R;
        const bool first = step == 0;
        const bool local = !first && total <= kXtyStage / 2;   // the same in every workgroup
        double* dst = local ? st + (step & 1) * (kXtyStage / 2) : bufs[cur];
        const int64_t l0 = local ? t : g.gtid, dl = local ? kFThreads : g.gthreads;
        for (int64_t l = l0; l < total; l += dl) {
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
        if (local) {
          bsync();
        } else {
          g.sync();
          cur ^= 1;
        }
        for (int q = pos; q < nrem - 1; ++q) rem[q] = rem[q + 1];
        --nrem;
        src = dst;
        ++step;
      }
      const double* H = src;  // Rn x R, complete in every workgroup's view
      // H staged in LDS (already there when the chain ended in LDS, then
      // moved to the start of the buffer); T = hadamard of the other Grams
      if (H != st) {
        double hv[8];
        for (int l0 = 0; l0 < Rn * R; l0 += 8 * kFThreads) {
          // read everything of this round before writing (H may overlap st)
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int l = l0 + u * kFThreads + t;
            hv[u] = l < Rn * R ? H[l] : 0.0;
          }
          bsync();
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int l = l0 + u * kFThreads + t;
            if (l < Rn * R) st[l] = hv[u];
          }
          bsync();
        }
      }
      for (int l = t; l < R * R; l += kFThreads) {
        double v = 1.0;
        for (int p = 0; p < N; ++p)
          if (p != n) v *= a.Gram[p][l];
        Ts[l] = v;
      }
      if (n == N - 1 && g.wg == 0) {
        // H of the last mode, kept for the fit (the chain buffers are reused)
        for (int l = t; l < Rn * R; l += kFThreads) a.H[l] = st[l];
      }
      bsync();
      double* An = a.A[n];
      if (a.update == 0) {
        // ---- ALS: Cholesky of T (in place, lower), ridge on failure; every
        // workgroup factors the same T the same way --------------------------
        for (int attempt = 0; attempt < 2; ++attempt) {
          if (attempt == 1) {
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
      }
      // ---- the rows of this workgroup: Q = U_n H, the update, the soft
      // threshold ------------------------------------------------------------
      int64_t r0, r1;
      grid_rows(g, In, r0, r1);
      for (int64_t i = r0 + t; i < r1; i += kFThreads)
        update_row<RMAX>(a, n, i, Rn, R, st, Ts, a.nrm + n * R);
      bsync();
      // V_n, Gram_n of the normalized factor (n < N - 1) and its norms
      grid_vg<kVgOut>(g, a.U64[n], An, In, Rn, R, n < N - 1, a.V[n], a.Gram[n],
                      a.nrm + n * R, st, part);
    }
    // ---- fit (workgroup 0), broadcast with the stopping decision -------------
    if (g.wg == 0) {
      double p = 0.0;
      const int Rl = a.Rn[N - 1];
      for (int l = t; l < Rl * R; l += kFThreads) p += a.H[l] * a.V[N - 1][l];
      const double inner = block_sum(p, red);
      double q = 0.0;
      for (int l = t; l < R * R; l += kFThreads) {
        double v = 1.0;
        for (int pp = 0; pp < N; ++pp) v *= a.Gram[pp][l];
        q += v;
      }
      const double yh2 = block_sum(q, red);
      double res2 = nrm2 - 2.0 * inner + yh2;
      res2 = res2 > 0.0 ? res2 : 0.0;
      const double f = 1.0 - sqrt(res2) / sqrt(nrm2);
      if (t == 0) {
        bcast[0] = f;
        bcast[1] = (it >= 2 && fabs(f - fit_prev) < a.tol) ? 1.0 : 0.0;
        if (a.fit_trace) a.fit_trace[it - 1] = f;
      }
    }
    g.sync();
    fit = bcast[0];
    const bool stop = bcast[1] != 0.0;
    g.sync();   // every workgroup has read the broadcast before it is rewritten
    if (stop) {
      converged = 1;
      break;
    }
    if (it < a.max_it) fit_prev = fit;
  }
  if (it > a.max_it) it = a.max_it;
  // ---- outputs: the stored rows divided by their norms; the last factor's
  // norms (its Gram's diagonal) are lambda -------------------------------------
  for (int n = 0; n < N; ++n) {
    const double* nr = a.nrm + n * R;
    const double* Gl = a.Gram[N - 1];
    const int64_t cnt = a.I[n] * R;
    for (int64_t l = g.gtid; l < cnt; l += g.gthreads) {
      const int r = static_cast<int>(l % R);
      double d = n < N - 1 ? nr[r] : sqrt(Gl[r * R + r]);
      d = d > 0.0 ? d : 1.0;
      a.A_out[n][l] = static_cast<float>(a.A[n][l] / d);
    }
  }
  if (g.wg == 0)
    for (int r = t; r < R; r += kFThreads)
      a.lambda[r] = static_cast<float>(sqrt(a.Gram[N - 1][r * R + r]));
  g.sync();   // every earlier barrier's failure flag is final
  if (g.wg == 0 && t == 0 && info) {
    // a barrier that gave up (not expected: the launch keeps every
    // workgroup resident) leaves the results undefined: converged = -1
    const bool failed = __hip_atomic_load(g.bar + 1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) != 0;
    info->iterations = it;
    info->converged = failed ? -1 : converged;
    info->ridged = ridged;
    info->init_used = 0;
    info->fit = fit;
    info->fit_prev = fit_prev;
  }
}

}  // namespace

namespace {

// Workgroups of the cooperative launch on the current device: at most one
// per CU (every workgroup must be resident), at most kGridMax (the rows of
// the partials buffers), and about `rows` rows of the largest mode each.
int grid_size(const void* kernel, int64_t Imax, int rows, int* G) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kFThreads, 0);
  if (e != hipSuccess) return hip_fail(e, "ffcp grid size");
  int64_t g = (Imax + rows - 1) / rows;
  const int64_t lim = static_cast<int64_t>(cus) * (per < 1 ? 1 : per);
  if (g > lim) g = lim;
  if (g > kGridMax) g = kGridMax;
  *G = static_cast<int>(g < 1 ? 1 : g);
  return kOk;
}

template <int RMAX>
int launch_ffcp_r(const FfcpArgs& a, hipStream_t s) {
  int64_t Imax = 0;
  for (int n = 0; n < a.N; ++n) Imax = a.I[n] > Imax ? a.I[n] : Imax;
  if (Imax >= kGridMinRows && a.part && a.bar && a.nrm) {
    const void* k = reinterpret_cast<const void*>(ffcp_grid_kernel<RMAX>);
    int G = 1;
    RT_TRY(grid_size(k, Imax, kGridRows, &G));
    // the barrier's counter and failure flag start at zero (a fill kernel:
    // the call may be captured in a graph)
    RT_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(a.bar), 0, 2, s));
    FfcpArgs arg = a;
    void* args[] = {&arg};
    hipError_t e = hipLaunchCooperativeKernel(k, dim3(G), dim3(kFThreads), args, 0, s);
    if (e != hipSuccess) return hip_fail(e, "ffcp cooperative launch");
    RT_LAUNCH_CHECK("ffcp grid");
    return kOk;
  }
  hipLaunchKernelGGL(ffcp_kernel<RMAX>, dim3(1), dim3(kFThreads), 0, s, a);
  RT_LAUNCH_CHECK("ffcp");
  return kOk;
}

}  // namespace

int64_t ffcp_grid_part_doubles(int64_t nout_max) { return kGridMax * nout_max + 64; }

int launch_ffcp(const FfcpArgs& a, hipStream_t s) {
  if (a.R <= 16) return launch_ffcp_r<16>(a, s);
  if (a.R <= 32) return launch_ffcp_r<32>(a, s);
  if (a.R <= 64) return launch_ffcp_r<64>(a, s);
  set_error("ffcp: R=%d exceeds 64", a.R);
  return kErrUnsupported;
}

}  // namespace rt
