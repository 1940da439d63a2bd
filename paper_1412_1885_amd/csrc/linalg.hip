// Small FP64 factorizations of the method:
//  * orthonormal basis of a sketch Z_n (Section IV-A, step 3 of the range
//    finder; the orthonormalization in Algorithm 3) with diag(R) >= 0: CholeskyQR2 in FP64,
//    falling back to Householder QR when the sketch is numerically rank
//    deficient;
//  * symmetric eigen-decomposition (cyclic Jacobi, parallel ordering) of the
//    R~ x R~ Gram matrices used to truncate the core and to build the HOSVD
//    initialization of FFCP.
// One workgroup per matrix; matrices of one call are batched over the grid.
#include "common.hpp"
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kQrThreads = 256;
constexpr int kQrWaves = kQrThreads / 64;

// Block reduction of KMAX per-thread partial sums (entries c in [lo, hi)).
template <int KMAX>
__device__ void block_reduce_vec(double (&part)[KMAX], double* red /*[waves][KMAX]*/,
                                 double* outv /*[KMAX]*/, int lo, int hi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < KMAX; ++c) {
    if (c >= lo && c < hi) {
      double v = wave_sum(part[c]);
      if (lane == 0) red[wave * KMAX + c] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < KMAX; c += kQrThreads) {
    if (c >= lo && c < hi) {
      double s = 0.0;
      for (int w = 0; w < kQrWaves; ++w) s += red[w * KMAX + c];
      outv[c] = s;
    }
  }
  __syncthreads();
}

// Householder QR of matrix m of the batch (LAPACK geqrf/orgqr scheme).
// W: I x K working copy, column-major (W[c*I + i]); P: I x K output Q,
// column-major FP64 scratch.
template <typename T, int KMAX>
__global__ __launch_bounds__(kQrThreads) void householder_kernel(
    QrBatch b, int32_t* rank_flag, const int32_t* need) {
  const int m = blockIdx.x;
  if (need[m] == 0) return;  // CholeskyQR2 succeeded for this matrix
  __shared__ double red[kQrWaves * KMAX];
  __shared__ double wv[KMAX];
  __shared__ double tau[KMAX];
  __shared__ double rdiag[KMAX];
  __shared__ double sc[4];
  const int64_t I = b.I[m];
  const int K = b.K[m];
  const T* Z = static_cast<const T*>(b.Z[m]);
  T* Qo = static_cast<T*>(b.Q[m]);
  double* W = b.work[m];
  double* P = W + I * K;
  const int t = threadIdx.x;

  for (int64_t l = t; l < I * K; l += kQrThreads) {
    int64_t i = l / K;
    int c = static_cast<int>(l % K);
    W[c * I + i] = static_cast<double>(Z[l]);
  }
  __syncthreads();

  for (int j = 0; j < K; ++j) {
    // norm of the sub-diagonal part of column j
    double part = 0.0;
    for (int64_t i = j + 1 + t; i < I; i += kQrThreads) {
      double x = W[j * I + i];
      part += x * x;
    }
    double xnorm2 = block_sum(part, red);
    if (t == 0) {
      double alpha = W[j * I + j];
      double beta, tj, scale;
      if (xnorm2 == 0.0) {
        tj = 0.0;  // H_j = I (LAPACK convention)
        beta = alpha;
        scale = 0.0;
      } else {
        double nrm = sqrt(alpha * alpha + xnorm2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      tau[j] = tj;
      rdiag[j] = beta;
      sc[0] = scale;
      W[j * I + j] = beta;
      if (beta == 0.0 && rank_flag) atomicOr(rank_flag, 1 << (b.bit0 + m));
    }
    __syncthreads();
    const double scale = sc[0];
    const double tj = tau[j];
    for (int64_t i = j + 1 + t; i < I; i += kQrThreads) W[j * I + i] *= scale;
    __syncthreads();
    if (tj == 0.0) continue;
    // w_c = v^T W[:, c] for c > j, with v_j = 1 and v_i = W[j*I+i] (i > j)
    double acc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
    for (int64_t i = j + t; i < I; i += kQrThreads) {
      double v = (i == j) ? 1.0 : W[j * I + i];
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c > j && c < K) acc[c] += v * W[c * I + i];
    }
    block_reduce_vec<KMAX>(acc, red, wv, j + 1, K);
    for (int64_t l = t; l < (I - j) * (K - j - 1); l += kQrThreads) {
      int64_t i = j + l % (I - j);
      int c = j + 1 + static_cast<int>(l / (I - j));
      double v = (i == j) ? 1.0 : W[j * I + i];
      W[c * I + i] -= tj * wv[c] * v;
    }
    __syncthreads();
  }

  // Form Q = H_0 ... H_{K-1} [I_K; 0] (backward accumulation).
  for (int64_t l = t; l < I * K; l += kQrThreads) {
    int c = static_cast<int>(l / I);
    int64_t i = l % I;
    P[l] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = K - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    double acc[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
    for (int64_t i = j + t; i < I; i += kQrThreads) {
      double v = (i == j) ? 1.0 : W[j * I + i];
#pragma unroll
      for (int c = 0; c < KMAX; ++c)
        if (c >= j && c < K) acc[c] += v * P[c * I + i];
    }
    block_reduce_vec<KMAX>(acc, red, wv, j, K);
    for (int64_t l = t; l < (I - j) * (K - j); l += kQrThreads) {
      int64_t i = j + l % (I - j);
      int c = j + static_cast<int>(l / (I - j));
      double v = (i == j) ? 1.0 : W[j * I + i];
      P[c * I + i] -= tj * wv[c] * v;
    }
    __syncthreads();
  }
  // diag(R) >= 0: flip the matching columns of Q.
  for (int64_t l = t; l < I * K; l += kQrThreads) {
    int64_t i = l / K;
    int c = static_cast<int>(l % K);
    double sgn = rdiag[c] < 0.0 ? -1.0 : 1.0;
    Qo[l] = static_cast<T>(sgn * P[c * I + i]);
  }
}

// Cholesky of the K x K symmetric matrix S (LDS, row-major) in place into
// its upper factor R (S = R^T R).  Returns false if a pivot is not
// sufficiently positive (the sketch is numerically rank deficient).
template <int KMAX>
__device__ bool chol_upper(double* S, int K, double* flag) {
  const int t = threadIdx.x;
  if (t == 0) {
    double tr = 0.0;
    for (int j = 0; j < K; ++j) tr += S[j * KMAX + j];
    flag[0] = 1e-11 * tr / K;  // pivot floor
    flag[1] = 1.0;
  }
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    if (t == 0) {
      double d = S[j * KMAX + j];
      if (!(d > flag[0])) {
        flag[1] = 0.0;
        d = 1.0;
      }
      S[j * KMAX + j] = sqrt(d);
    }
    __syncthreads();
    const double rjj = S[j * KMAX + j];
    for (int c = j + 1 + t; c < K; c += kQrThreads) S[j * KMAX + c] /= rjj;
    __syncthreads();
    const int n = K - j - 1;
    for (int l = t; l < n * n; l += kQrThreads) {
      const int r = j + 1 + l / n, c = j + 1 + l % n;
      if (c >= r) S[r * KMAX + c] -= S[j * KMAX + r] * S[j * KMAX + c];
    }
    __syncthreads();
  }
  return flag[1] > 0.5;
}

// CholeskyQR2 in FP64: R1 = chol(Z^T Z), Q1 = Z R1^{-1}, R2 = chol(Q1^T Q1),
// Q = Q1 R2^{-1}.  diag(R2 R1) > 0 by construction, so Q is the same unique
// factor Householder QR with a positive diagonal gives (up to rounding).
// Falls back to Householder when a Gram matrix is not positive definite.
//
// Sketches of at most kQfMaxI rows and K <= 32 take the fused one-workgroup
// form below; for larger ones the row work is spread over many workgroups
// (row chunks x matrices):
//   rows(0): partial Gram of Z per chunk
//   chol(0): sum of the partials (fixed order), R1, R1^{-1}
//   rows(1): Q1 = Z R1^{-1} (FP64, kept in work) and its partial Gram
//   chol(1): R2, R2^{-1}
//   rows(2): Q = Q1 R2^{-1}, written in the output type
// Work layout per matrix (doubles): [0, IK) Q1 | [IK, 2IK) Householder
// scratch | kQrChunks x K x K partial Grams | K x K inverse factor.
constexpr int kQrChunks = 64;
constexpr int kQrBlock = 64;  // rows staged in LDS at a time

__host__ __device__ inline int64_t qr_rows_per_chunk(int64_t I) {
  int64_t r = (I + kQrChunks - 1) / kQrChunks;
  r = (r + kQrBlock - 1) / kQrBlock * kQrBlock;
  return r < kQrBlock ? kQrBlock : r;
}

template <typename T, int KMAX>
__global__ __launch_bounds__(kQrThreads) void qr_rows_kernel(QrBatch b, int phase) {
  // thread -> (row group g, column c): c = t % KMAX, g = t / KMAX
  constexpr int kG = kQrThreads / KMAX;
  constexpr int kRowsPerThread = kQrBlock / kG;   // transform rows
  constexpr int kGramRows = (KMAX + kG - 1) / kG; // Gram rows r = g + kG*q
  __shared__ double zs[kQrBlock][KMAX + 1];
  __shared__ double zo[kQrBlock][KMAX + 1];
  __shared__ double Ri[KMAX][KMAX + 1];
  const int m = blockIdx.y;
  if (phase > 0 && b.need[m] != 0) return;
  const int64_t I = b.I[m];
  const int K = b.K[m];
  const int64_t rpc = qr_rows_per_chunk(I);
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rpc;
  if (r0 >= I) return;
  const int64_t r1 = (r0 + rpc) < I ? (r0 + rpc) : I;
  const T* Z = static_cast<const T*>(b.Z[m]);
  T* Qo = static_cast<T*>(b.Q[m]);
  double* W = b.work[m];
  double* part = W + 2 * I * K;
  const double* rinv = part + static_cast<int64_t>(kQrChunks) * K * K;
  const int t = threadIdx.x;
  const int c = t % KMAX, g = t / KMAX;
  if (phase > 0) {
    for (int l = t; l < KMAX * KMAX; l += kQrThreads) {
      const int i = l / KMAX, j = l % KMAX;
      Ri[i][j] = (i < K && j < K) ? rinv[i * K + j] : 0.0;
    }
  }
  double acc[kGramRows];
#pragma unroll
  for (int q = 0; q < kGramRows; ++q) acc[q] = 0.0;
  for (int64_t i0 = r0; i0 < r1; i0 += kQrBlock) {
    const int rows = static_cast<int>((r1 - i0) < kQrBlock ? (r1 - i0) : kQrBlock);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) {
      const int ii = g + kG * q;
      double v = 0.0;
      if (ii < rows && c < K)
        v = phase == 2 ? W[(i0 + ii) * K + c]
                       : static_cast<double>(Z[(i0 + ii) * K + c]);
      zs[ii][c] = v;
    }
    __syncthreads();
    double (*src)[KMAX + 1] = zs;
    if (phase > 0) {
      // row transform: out[ii][c] = sum_{l <= c} z[ii][l] Rinv[l][c]
#pragma unroll
      for (int q = 0; q < kRowsPerThread; ++q) {
        const int ii = g + kG * q;
        double v = 0.0;
#pragma unroll 8
        for (int l = 0; l < KMAX; ++l)
          if (l <= c) v += zs[ii][l] * Ri[l][c];
        zo[ii][c] = v;
        if (ii < rows && c < K) {
          if (phase == 1)
            W[(i0 + ii) * K + c] = v;
          else
            Qo[(i0 + ii) * K + c] = static_cast<T>(v);
        }
      }
      __syncthreads();
      src = zo;
    }
    if (phase < 2) {
      // Gram rows r = g + kG*q, column c (padding rows/columns are zero)
      for (int ii = 0; ii < rows; ++ii) {
        const double zc = src[ii][c];
#pragma unroll
        for (int q = 0; q < kGramRows; ++q) {
          const int r = g + kG * q;
          if (r < KMAX) acc[q] += src[ii][r] * zc;
        }
      }
    }
  }
  if (phase < 2) {
    double* pc = part + static_cast<int64_t>(blockIdx.x) * K * K;
#pragma unroll
    for (int q = 0; q < kGramRows; ++q) {
      const int r = g + kG * q;
      if (r < K && c < K) pc[r * K + c] = acc[q];
    }
  }
}

template <int KMAX>
__global__ __launch_bounds__(kQrThreads) void qr_chol_kernel(QrBatch b, int pass) {
  __shared__ double S[KMAX * KMAX];
  __shared__ double Rs[KMAX * KMAX];
  __shared__ double fl[4];
  const int m = blockIdx.x;
  if (pass > 0 && b.need[m] != 0) return;
  const int64_t I = b.I[m];
  const int K = b.K[m];
  double* part = b.work[m] + 2 * I * K;
  double* rinv = part + static_cast<int64_t>(kQrChunks) * K * K;
  const int64_t rpc = qr_rows_per_chunk(I);
  const int chunks = static_cast<int>((I + rpc - 1) / rpc);
  const int t = threadIdx.x;
  for (int l = t; l < K * K; l += kQrThreads) {
    const int r = l / K, cc = l % K;
    double v = 0.0;
    for (int ch = 0; ch < chunks; ++ch) v += part[static_cast<int64_t>(ch) * K * K + l];
    S[r * KMAX + cc] = v;
  }
  __syncthreads();
  const bool ok = chol_upper<KMAX>(S, K, fl);
  __syncthreads();
  if (!ok) {
    if (t == 0) b.need[m] = 1;
    return;
  }
  if (pass == 0 && t == 0) b.need[m] = 0;
  // R^{-1}: thread j back-substitutes column j (upper triangular)
  for (int j = t; j < K; j += kQrThreads) {
    for (int i = j; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) v -= S[i * KMAX + k] * Rs[k * KMAX + j];
      Rs[i * KMAX + j] = v / S[i * KMAX + i];
    }
  }
  __syncthreads();
  for (int l = t; l < K * K; l += kQrThreads) {
    const int i = l / K, j = l % K;
    rinv[l] = (i <= j) ? Rs[i * KMAX + j] : 0.0;
  }
}

__device__ __forceinline__ double wave_read(double v, int src) {   // src uniform
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(u), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// (the rotations need c^2 + s^2 = 1 to working precision)
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- Jacobi
// One workgroup of four wavefronts per matrix.  The pairs of a round
// partition the indices, so S and V split into disjoint 2 x 2 blocks
// (pair a) x (pair b); a thread owns such blocks (at most kBlk, indices
// computed once).  S is double-buffered: a round reads every value it needs
// from the previous copy, each thread derives the rotations of its own two
// pairs from that copy (the same arithmetic on the same values gives every
// thread the same rotation), writes its block of S J^T..J into the other
// copy and rotates its block of V in place.  One barrier per round.  The
// round-robin pair schedule is arithmetic.
constexpr int kEigThreads = 256;
constexpr int kEigMax = 64;

// Pair p of round r in the round-robin schedule over np players (np even;
// every index >= n is the dummy).  With p < np/2 and r < np - 1 both
// arguments of the reductions mod np - 1 lie in [0, 2(np - 1)), so one
// conditional subtraction replaces them.
__device__ __forceinline__ void jacobi_pair(int p, int r, int np, int& lo, int& hi) {
  const int m = np - 1;
  int x = p - 1 + r;
  x = x >= m ? x - m : x;
  int y = np - 2 - p + r;
  y = y >= m ? y - m : y;
  const int a = (p == 0) ? 0 : 1 + x;
  const int q = 1 + y;
  lo = a < q ? a : q;
  hi = a < q ? q : a;
}

// Rotation (c, s) of the pair (lo, hi) from a_pp = Spp, a_qq = Sqq,
// a_pq = Spq: the smaller angle that annihilates a_pq,
// tan = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = a_qq - a_pp, e = 2 a_pq.
// A pair is rotated only while |a_pq| > thresh; returns whether it is.
__device__ __forceinline__ bool jacobi_rotation(double app, double aqq, double apq,
                                                bool real, double thresh, double& c,
                                                double& s) {
  c = 1.0;
  s = 0.0;
  if (!real || !(fabs(apq) > thresh)) return false;
  const double d = aqq - app, e = 2.0 * apq;
  const double tt = (d >= 0.0 ? e : -e) / (fabs(d) + sqrt(d * d + e * e));
  c = rsqrt_nr(1.0 + tt * tt);
  s = tt * c;
  return true;
}

__global__ __launch_bounds__(kEigThreads) void eig_kernel(EigBatch b) {
  __shared__ double S2[2][kEigMax][kEigMax + 1];
  __shared__ double V[kEigMax][kEigMax + 1];
  __shared__ double red[kEigThreads / 64];
  __shared__ int rankpos[kEigMax];
  const int m = blockIdx.x;
  const int n = b.n[m];
  const int k = b.k[m];
  const int t = threadIdx.x;
  const double* Sin = b.S[m];
  for (int l = t; l < n * n; l += kEigThreads) {
    int i = l / n, j = l % n;
    S2[0][i][j] = 0.5 * (Sin[i * n + j] + Sin[j * n + i]);
    V[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = (n + 1) & ~1;  // even number of players (dummy = n)
  const int hp = np / 2;
  double fro = 0.0;
  for (int l = t; l < n * n; l += kEigThreads) {
    const double x = S2[0][l / n][l % n];
    fro += x * x;
  }
  // Threshold Jacobi: |a_pq| > 1e-14 ||S||_F.  A per-element test stays
  // above the rounding floor of the 2 x 2 updates (a few ulps of ||S||),
  // where a test on the whole off-diagonal norm can sit at that floor and
  // never pass.  The sweeps end after one in which no pair was rotated.
  const double thresh = 1e-14 * sqrt(block_sum(fro, red)) + 1e-300;
  constexpr int kBlk = kEigMax * kEigMax / 4 / kEigThreads;   // 4
  int bpa[kBlk], bpb[kBlk];
#pragma unroll
  for (int u = 0; u < kBlk; ++u) {
    const int blk = u * kEigThreads + t;
    bpa[u] = blk < hp * hp ? blk / hp : -1;
    bpb[u] = blk < hp * hp ? blk - (blk / hp) * hp : 0;
  }
  const int nblk = (hp * hp + kEigThreads - 1) / kEigThreads;   // slots in use
  int cur = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;   // this thread saw a rotation in this sweep
    for (int r = 0; r < np - 1; ++r) {
      const double(*Sc)[kEigMax + 1] = S2[cur];
      double(*Sn)[kEigMax + 1] = S2[cur ^ 1];
#pragma unroll
      for (int u = 0; u < kBlk; ++u) {
        if (u >= nblk) break;
        if (bpa[u] < 0) continue;
        int i0, i1, j0, j1;
        jacobi_pair(bpa[u], r, np, i0, i1);
        jacobi_pair(bpb[u], r, np, j0, j1);
        const bool r1 = i1 < n, c1 = j1 < n;
        const int i1c = r1 ? i1 : i0, j1c = c1 ? j1 : j0;
        // every load of the block first: its four entries, the three
        // entries of each pair's 2 x 2 diagonal block, its V entries
        const double b00 = Sc[i0][j0], b01 = Sc[i0][j1c];
        const double b10 = Sc[i1c][j0], b11 = Sc[i1c][j1c];
        const double ap0 = Sc[i0][i0], ap1 = Sc[i1c][i1c], apx = Sc[i0][i1c];
        const double bp0 = Sc[j0][j0], bp1 = Sc[j1c][j1c], bpx = Sc[j0][j1c];
        const double v00 = V[i0][j0], v01 = V[i0][j1c];
        const double v10 = V[i1c][j0], v11 = V[i1c][j1c];
        double ca, sa, cb, sb;
        rotated |= jacobi_rotation(ap0, ap1, apx, r1, thresh, ca, sa);
        rotated |= jacobi_rotation(bp0, bp1, bpx, c1, thresh, cb, sb);
        // a dummy row or column holds zeros
        const double e01 = c1 ? b01 : 0.0, e10 = r1 ? b10 : 0.0;
        const double e11 = (r1 && c1) ? b11 : 0.0;
        const double x00 = ca * b00 - sa * e10, x01 = ca * e01 - sa * e11;
        const double x10 = sa * b00 + ca * e10, x11 = sa * e01 + ca * e11;
        Sn[i0][j0] = cb * x00 - sb * x01;
        if (c1) Sn[i0][j1] = sb * x00 + cb * x01;
        if (r1) Sn[i1][j0] = cb * x10 - sb * x11;
        if (r1 && c1) Sn[i1][j1] = sb * x10 + cb * x11;
        // V <- V J on rows {i0, i1}, columns {j0, j1}
        if (c1) {
          V[i0][j0] = cb * v00 - sb * v01;
          V[i0][j1] = sb * v00 + cb * v01;
          if (r1) {
            V[i1][j0] = cb * v10 - sb * v11;
            V[i1][j1] = sb * v10 + cb * v11;
          }
        }
      }
      cur ^= 1;
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  const double(*S)[kEigMax + 1] = S2[cur];
  // descending order, ties by ascending index
  if (t < n) {
    double lt = S[t][t];
    int pos = 0;
    for (int j = 0; j < n; ++j) {
      double lj = S[j][j];
      if (lj > lt || (lj == lt && j < t)) ++pos;
    }
    rankpos[t] = pos;
  }
  __syncthreads();
  double* W = b.W[m];
  for (int src = t; src < n; src += kEigThreads) {
    int pos = rankpos[src];
    if (pos >= k) continue;
    // sign: largest |entry| positive, lowest index on ties
    int jm = 0;
    double vm = fabs(V[0][src]);
    for (int j = 1; j < n; ++j) {
      double a = fabs(V[j][src]);
      if (a > vm) { vm = a; jm = j; }
    }
    double sgn = V[jm][src] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j < n; ++j) W[j * k + pos] = sgn * V[j][src];
    if (b.evals[m]) b.evals[m][pos] = S[src][src];
  }
}

// The same cyclic Jacobi for n <= 32: the matrix is zero-padded to the even
// size np = n or n + 1 (a zero row and column is never rotated, since its
// off-diagonal entries stay 0 and fail the threshold), so np/2 pairs,
// np - 1 rounds per sweep and one 2 x 2 block per thread of the first
// (np/2)^2, with no dummy player.  The rotation angles
// come from the hardware reciprocal and reciprocal square root refined by
// Newton steps (c^2 + s^2 = 1 to working precision) instead of an IEEE
// division and square root, and the LDS addresses from 24-bit products:
// the round is about half the instructions of the general kernel.
__device__ __forceinline__ double recip_nr(double p) {
  double x = __builtin_amdgcn_rcp(p);
  double e = fma(-p, x, 1.0);
  x = fma(x, e, x);
  e = fma(-p, x, 1.0);
  return fma(x, e, x);
}

__device__ __forceinline__ bool jacobi_rotation_fast(double app, double aqq, double apq,
                                                     double thresh, double& c, double& s) {
  const double d = aqq - app, e = 2.0 * apq;
  const bool on = fabs(apq) > thresh;
  const double x = on ? fma(d, d, e * e) : 1.0;
  const double r = x * rsqrt_nr(x);   // sqrt(d^2 + e^2)
  const double tt = on ? (d >= 0.0 ? e : -e) * recip_nr(fabs(d) + r) : 0.0;
  const double cr = rsqrt_nr(fma(tt, tt, 1.0));
  c = on ? cr : 1.0;   // an unrotated pair is copied exactly
  s = on ? tt * cr : 0.0;
  return on;
}

__global__ __launch_bounds__(kEigThreads) void eig32_kernel(EigBatch b) {
  constexpr int NP = 32, L = NP + 1;
  __shared__ double S2[2][NP * L];
  __shared__ double V[NP * L];
  __shared__ double red[kEigThreads / 64];
  __shared__ int rankpos[NP];
  const int m = blockIdx.x;
  const int n = b.n[m];
  const int k = b.k[m];
  const int t = threadIdx.x;
  const double* Sin = b.S[m];
  for (int l = t; l < NP * NP; l += kEigThreads) {
    const int i = l / NP, j = l % NP;
    S2[0][i * L + j] = (i < n && j < n) ? 0.5 * (Sin[i * n + j] + Sin[j * n + i]) : 0.0;
    V[i * L + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro = 0.0;
  for (int l = t; l < NP * NP; l += kEigThreads) {
    const double x = S2[0][(l / NP) * L + l % NP];
    fro += x * x;
  }
  const double thresh = 1e-14 * sqrt(block_sum(fro, red)) + 1e-300;
  const int pa = t >> 4, pb = t & 15;   // the thread's block: pairs pa x pb
  // the round-robin schedule runs over the even size np >= n (np - 1
  // rounds per sweep); entries beyond np are never read
  const int np = n + (n & 1);
  const bool on = pa < np / 2 && pb < np / 2;
  int cur = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < np - 1; ++r) {
      const double* Sc = S2[cur];
      double* Sn = S2[cur ^ 1];
      if (!on) {
        cur ^= 1;
        __syncthreads();
        continue;
      }
      int i0, i1, j0, j1;
      jacobi_pair(pa, r, np, i0, i1);
      jacobi_pair(pb, r, np, j0, j1);
      const int ri0 = __mul24(i0, L), ri1 = __mul24(i1, L);
      const int rj0 = __mul24(j0, L), rj1 = __mul24(j1, L);
      const double b00 = Sc[ri0 + j0], b01 = Sc[ri0 + j1];
      const double b10 = Sc[ri1 + j0], b11 = Sc[ri1 + j1];
      const double ap0 = Sc[ri0 + i0], ap1 = Sc[ri1 + i1], apx = Sc[ri0 + i1];
      const double bp0 = Sc[rj0 + j0], bp1 = Sc[rj1 + j1], bpx = Sc[rj0 + j1];
      const double v00 = V[ri0 + j0], v01 = V[ri0 + j1];
      const double v10 = V[ri1 + j0], v11 = V[ri1 + j1];
      double ca, sa, cb, sb;
      rotated |= jacobi_rotation_fast(ap0, ap1, apx, thresh, ca, sa);
      rotated |= jacobi_rotation_fast(bp0, bp1, bpx, thresh, cb, sb);
      const double x00 = ca * b00 - sa * b10, x01 = ca * b01 - sa * b11;
      const double x10 = sa * b00 + ca * b10, x11 = sa * b01 + ca * b11;
      Sn[ri0 + j0] = cb * x00 - sb * x01;
      Sn[ri0 + j1] = sb * x00 + cb * x01;
      Sn[ri1 + j0] = cb * x10 - sb * x11;
      Sn[ri1 + j1] = sb * x10 + cb * x11;
      // V <- V J on rows {i0, i1}, columns {j0, j1}
      V[ri0 + j0] = cb * v00 - sb * v01;
      V[ri0 + j1] = sb * v00 + cb * v01;
      V[ri1 + j0] = cb * v10 - sb * v11;
      V[ri1 + j1] = sb * v10 + cb * v11;
      cur ^= 1;
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  const double* S = S2[cur];
  // descending order over the n real indices, ties by ascending index
  if (t < n) {
    const double lt = S[t * L + t];
    int pos = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = S[j * L + j];
      if (lj > lt || (lj == lt && j < t)) ++pos;
    }
    rankpos[t] = pos;
  }
  __syncthreads();
  double* W = b.W[m];
  for (int src = t; src < n; src += kEigThreads) {
    const int pos = rankpos[src];
    if (pos >= k) continue;
    // sign: largest |entry| positive, lowest index on ties
    int jm = 0;
    double vm = fabs(V[src]);
    for (int j = 1; j < n; ++j) {
      const double a = fabs(V[j * L + src]);
      if (a > vm) {
        vm = a;
        jm = j;
      }
    }
    const double sgn = V[jm * L + src] < 0.0 ? -1.0 : 1.0;
    for (int j = 0; j < n; ++j) W[j * k + pos] = sgn * V[j * L + src];
    if (b.evals[m]) b.evals[m][pos] = S[src * L + src];
  }
}

// ------------------------------------------------- fused CholeskyQR2
// The same CholeskyQR2 for sketches of at most kQfMaxI rows and K <= 32 in
// ONE workgroup per matrix, so that no step waits on a global round trip or
// a kernel boundary (the multi-kernel form spends most of its time there):
//   G1 = Z^T Z  (FP64 MFMA over 4-row groups read straight from Z)
//   R1^{-1} for R1 = chol(G1), by Gaussian elimination on [G1 | I]
//                                               (one wavefront, registers)
//   Q1 = Z R1^{-1} tile by tile, G2 = Q1^T Q1   (Q1 never leaves registers)
//   R2^{-1} likewise, M = R1^{-1} R2^{-1}
//   Q  = Z M     (= Q1 R2^{-1} up to FP64 rounding; M is upper triangular)
// v_mfma_f64_16x16x4_f64 lane layout (checked on the device): A (16 x 4)
// lane l holds A[l%16][l/16], B (4 x 16) lane l holds B[l/16][l%16], D
// (16 x 16) lane l element e holds D[4e + l/16][l%16].  A D tile of Q1 rows
// therefore serves directly as both operands of the Gram product: its
// element e is the 4-row slice 4e..4e+3 of the tile (k = l/16) in operand
// layout.
constexpr int kQfThreads = 512;
constexpr int kQfWaves = kQfThreads / 64;
constexpr int kQfMaxI = 4096;
constexpr int kQfLd = 33;   // LDS row stride of the 32 x 32 FP64 matrices

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// R^{-1} for the upper Cholesky factor R of the K x K SPD matrix S, by one
// wavefront, through Gaussian elimination without pivoting on [S | I]:
// lane c < K holds column c of S, lane K + c column c of I, all in
// registers.  Step k broadcasts the pivot and the multipliers of column k
// (rows below k) from lane k through scalar registers and subtracts the
// row multiples in every lane.  With S = L D L^T the pivots are D (= the
// squared diagonal of R) and the right half becomes E = L^{-1}; since
// R = D^{1/2} L^T, R^{-1} = E^T D^{-1/2}, upper triangular with a positive
// diagonal: lane K + i writes row i.  A pivot at or below 1e-11 of the mean
// diagonal of S fails (returns false, wave-uniform).  Writes R^{-1} to Ri
// ([32][kQfLd], zero outside the upper K x K part).
__device__ __forceinline__ bool chol_inv_ge_wave(const double* S, int K, double* Ri) {
  const int c = threadIdx.x & 63;
  const bool isS = c < K, isI = c >= K && c < 2 * K;
  const int cs = isS ? c : 0;   // clamped: loads in bounds
  const double floor_ = 1e-11 * wave_sum(isS ? S[cs * kQfLd + cs] : 0.0) / K;
  double col[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    double v = 0.0;
    if (isS)
      v = S[r * kQfLd + cs];
    else if (isI)
      v = (r == c - K) ? 1.0 : 0.0;
    col[r] = r < K ? v : 0.0;
  }
  double dinv[32];   // 1 / sqrt(pivot k), uniform
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    dinv[k] = 0.0;
    if (k < K) {
      const double p = wave_read(col[k], k);
      ok = ok && p > floor_;
      dinv[k] = rsqrt_nr(p);
      const double rp = dinv[k] * dinv[k];   // 1 / p
      const double ck = col[k];
      // rows at or past K are zero in every lane: no guard, straight-line code
      double mv[32];
#pragma unroll
      for (int i = k + 1; i < 32; ++i) mv[i] = wave_read(col[i], k);
#pragma unroll
      for (int i = k + 1; i < 32; ++i) col[i] = fma(-(mv[i] * rp), ck, col[i]);
    }
  }
  // rows of R^{-1}: lane K + i holds column i of E, R^{-1}[i][j] = E[j][i] / sqrt(d_j)
  if (isI) {
    const int i = c - K;
#pragma unroll
    for (int j = 0; j < 32; ++j) Ri[i * kQfLd + j] = j < K ? col[j] * dinv[j] : 0.0;
  }
  // rows K .. 31 of R^{-1} are zero
  if (c >= K && c < 32) {
#pragma unroll
    for (int j = 0; j < 32; ++j) Ri[c * kQfLd + j] = 0.0;
  }
  return ok;
}

// Fixed-order sum of the waves' Gram tiles (red: [waves][3][64][4]) into
// the symmetric 32 x 32 matrix G (row stride kQfLd).
__device__ void gram_reduce(const double* red, double* G) {
  for (int o = threadIdx.x; o < 3 * 256; o += kQfThreads) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kQfWaves; ++w) v += red[w * 768 + o];
    const int tile = o / 256, l = (o % 256) / 4, e = o % 4;
    const int a = 4 * e + l / 16, bcol = l % 16;
    if (tile == 0) {
      G[a * kQfLd + bcol] = v;
    } else if (tile == 1) {
      G[a * kQfLd + 16 + bcol] = v;
      G[(16 + bcol) * kQfLd + a] = v;
    } else {
      G[(16 + a) * kQfLd + 16 + bcol] = v;
    }
  }
}

__device__ __forceinline__ void gram_store(double* red, const v4d& g00, const v4d& g01,
                                           const v4d& g11) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    red[w * 768 + l * 4 + i] = g00[i];
    red[w * 768 + 256 + l * 4 + i] = g01[i];
    red[w * 768 + 512 + l * 4 + i] = g11[i];
  }
}

// Tile (16 rows from r0, column tile ct) of Z X for the upper triangular X
// whose operand values the lane holds in bx[ct][ks]; az[ks] = Z[r0 + l%16][4ks + l/16].
template <typename T>
__device__ __forceinline__ v4d tile_times(const T (&az)[8], const double (&bx)[2][8], int ct) {
  // two accumulators: consecutive products do not wait on each other
  v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  if (ct == 0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)   // X[k][c] = 0 for k > c
      acc[ks & 1] = mfma_f64(static_cast<double>(az[ks]), bx[0][ks], acc[ks & 1]);
  } else {
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
      acc[ks & 1] = mfma_f64(static_cast<double>(az[ks]), bx[1][ks], acc[ks & 1]);
  }
  return acc[0] + acc[1];
}

template <typename T>
__device__ __forceinline__ void load_rows(const T* Z, int64_t I, int K, int64_t r0, T (&az)[8]) {
  const int l = threadIdx.x & 63;
  const int64_t r = r0 + (l & 15);
  // unconditional loads from clamped (valid) addresses, zeroed afterwards:
  // no branches, so a batch of loads is in flight together
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const int k = 4 * ks + (l >> 4);
    const bool ok = r < I && k < K;
    const T v = Z[ok ? r * K + k : 0];
    az[ks] = ok ? v : T(0);
  }
}

// Register batches: the loads of a wave's next NG row groups (first Gram)
// or NB row blocks (transforms) are all issued before any of them is used,
// so a pass waits for global memory once per batch, not once per block.
template <typename T> struct QfBatch { static constexpr int NG = 16, NB = 4; };
template <> struct QfBatch<double> { static constexpr int NG = 16, NB = 4; };

__device__ __forceinline__ void load_bx(const double* X, double (&bx)[2][8]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) bx[ct][ks] = X[(4 * ks + (l >> 4)) * kQfLd + 16 * ct + (l & 15)];
}

template <typename T>
__global__ __launch_bounds__(kQfThreads) void qr_fused_kernel(QrBatch b) {
  __shared__ double red[kQfWaves * 768];
  __shared__ double S[32 * kQfLd];
  __shared__ double Ri1[32 * kQfLd];
  __shared__ double Ri2[32 * kQfLd];
  __shared__ double scal[2];
  const int m = blockIdx.x;
  const int64_t I = b.I[m];
  const int K = b.K[m];
  const T* Z = static_cast<const T*>(b.Z[m]);
  T* Qo = static_cast<T*>(b.Q[m]);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const bool wide = K > 16;   // second column tile
  for (int e = t; e < 32 * kQfLd; e += kQfThreads) S[e] = 0.0;
  __syncthreads();

  // G1 = Z^T Z over 4-row groups: lane l holds Z[4g + l/16][l%16] (and +16)
  constexpr int NG = QfBatch<T>::NG, NB = QfBatch<T>::NB;
  {
    v4d g00[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}, g01[2] = {g00[0], g00[0]},
        g11[2] = {g00[0], g00[0]};
    const int64_t ng = (I + 3) / 4;
    const int k0 = l & 15, k1 = 16 + (l & 15);
    for (int64_t gb = w; gb < ng; gb += NG * kQfWaves) {
      T a0[NG], a1[NG];
#pragma unroll
      for (int j = 0; j < NG; ++j) {   // clamped loads, zeroed: see load_rows
        const int64_t r = 4 * (gb + j * kQfWaves) + (l >> 4);
        const bool ok0 = r < I && k0 < K, ok1 = r < I && k1 < K;
        const T v0 = Z[ok0 ? r * K + k0 : 0];
        const T v1 = Z[ok1 ? r * K + k1 : 0];
        a0[j] = ok0 ? v0 : T(0);
        a1[j] = ok1 ? v1 : T(0);
      }
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const double x0 = static_cast<double>(a0[j]), x1 = static_cast<double>(a1[j]);
        g00[j & 1] = mfma_f64(x0, x0, g00[j & 1]);
        if (wide) {
          g01[j & 1] = mfma_f64(x0, x1, g01[j & 1]);
          g11[j & 1] = mfma_f64(x1, x1, g11[j & 1]);
        }
      }
    }
    gram_store(red, g00[0] + g00[1], g01[0] + g01[1], g11[0] + g11[1]);
  }
  __syncthreads();
  gram_reduce(red, S);
  __syncthreads();
  if (w == 0) {
    const bool ok = chol_inv_ge_wave(S, K, Ri1);
    if (l == 0) scal[0] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  if (scal[0] < 0.5) {
    if (t == 0) b.need[m] = 1;   // Householder QR takes over
    return;
  }

  // Q1 = Z R1^{-1} (registers only) and G2 = Q1^T Q1
  const int64_t nrb = (I + 15) / 16;
  {
    double bx[2][8];
    load_bx(Ri1, bx);
    v4d g00[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}, g01[2] = {g00[0], g00[0]},
        g11[2] = {g00[0], g00[0]};
    for (int64_t b0 = w; b0 < nrb; b0 += NB * kQfWaves) {
      T az[NB][8];
#pragma unroll
      for (int j = 0; j < NB; ++j) load_rows(Z, I, K, 16 * (b0 + j * kQfWaves), az[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (b0 + j * kQfWaves >= nrb) break;   // zero rows: nothing to add
        const v4d q0 = tile_times(az[j], bx, 0);
        const v4d q1 = wide ? tile_times(az[j], bx, 1) : q0 * 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          g00[i & 1] = mfma_f64(q0[i], q0[i], g00[i & 1]);
          if (wide) {
            g01[i & 1] = mfma_f64(q0[i], q1[i], g01[i & 1]);
            g11[i & 1] = mfma_f64(q1[i], q1[i], g11[i & 1]);
          }
        }
      }
    }
    gram_store(red, g00[0] + g00[1], g01[0] + g01[1], g11[0] + g11[1]);
  }
  __syncthreads();
  for (int e = t; e < 32 * kQfLd; e += kQfThreads) S[e] = 0.0;
  __syncthreads();
  gram_reduce(red, S);
  __syncthreads();
  if (w == 0) {
    const bool ok = chol_inv_ge_wave(S, K, Ri2);
    if (l == 0) scal[0] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  if (scal[0] < 0.5) {
    if (t == 0) b.need[m] = 1;
    return;
  }
  // M = R1^{-1} R2^{-1} (upper triangular) into S
  for (int e = t; e < 32 * 32; e += kQfThreads) {
    const int i = e / 32, c = e % 32;
    double v = 0.0;
    for (int k = i; k <= c; ++k) v += Ri1[i * kQfLd + k] * Ri2[k * kQfLd + c];
    S[i * kQfLd + c] = v;
  }
  __syncthreads();
  // Q = Z M
  {
    double bx[2][8];
    load_bx(S, bx);
    for (int64_t b0 = w; b0 < nrb; b0 += NB * kQfWaves) {
      T az[NB][8];
#pragma unroll
      for (int j = 0; j < NB; ++j) load_rows(Z, I, K, 16 * (b0 + j * kQfWaves), az[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int64_t rb = b0 + j * kQfWaves;
        if (rb >= nrb) break;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          if (ct == 1 && !wide) break;
          const v4d q = tile_times(az[j], bx, ct);
          const int cidx = 16 * ct + (l & 15);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t r = 16 * rb + 4 * i + (l >> 4);
            if (r < I && cidx < K) Qo[r * K + cidx] = static_cast<T>(q[i]);
          }
        }
      }
    }
  }
  if (t == 0) b.need[m] = 0;
}

// ------------------------------------------------- tall cross products
// out = X^T Y for tall FP32 X (I x p) and Y (I x q), p, q <= 32, by the
// FP64 MFMA of the fused CholeskyQR2's first Gram: waves take 4-row groups
// in turn (a batch of NG groups' loads in flight), each holds the 2 x 2
// tiles of 16 x 16 of its partial product, and the waves' tiles are summed
// in wave order.  Operand lane layout as there: lane l holds row
// 4g + l/16, column l%16 (+16 for the second tile) of X and of Y.
__global__ __launch_bounds__(kQfThreads) void cross_tall_kernel(CrossBatch b) {
  __shared__ double red[kQfWaves * 4 * 256];
  const int m = blockIdx.x;
  const int64_t I = b.I[m];
  const int p = b.p[m], q = b.q[m];
  const float* X = b.X[m];
  const float* Y = b.Y[m];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  constexpr int NG = 16;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t ng = (I + 3) / 4;
  const int c0 = l & 15, c1 = 16 + (l & 15);
  for (int64_t gb = w; gb < ng; gb += NG * kQfWaves) {
    float x0[NG], x1[NG], y0[NG], y1[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) {   // clamped loads, zeroed afterwards
      const int64_t r = 4 * (gb + j * kQfWaves) + (l >> 4);
      const bool in = r < I;
      const float a0 = X[in && c0 < p ? r * p + c0 : 0];
      const float a1 = X[in && c1 < p ? r * p + c1 : 0];
      const float b0 = Y[in && c0 < q ? r * q + c0 : 0];
      const float b1 = Y[in && c1 < q ? r * q + c1 : 0];
      x0[j] = in && c0 < p ? a0 : 0.0f;
      x1[j] = in && c1 < p ? a1 : 0.0f;
      y0[j] = in && c0 < q ? b0 : 0.0f;
      y1[j] = in && c1 < q ? b1 : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const double a0 = x0[j], a1 = x1[j], b0 = y0[j], b1 = y1[j];
      acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
      if (q > 16) acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
      if (p > 16) {
        acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
        if (q > 16) acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[((w * 4 + 2 * a + c) * 64 + l) * 4 + e] = acc[a][c][e];
  __syncthreads();
  double* out = b.out[m];
  for (int o = t; o < 4 * 256; o += kQfThreads) {
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < kQfWaves; ++ww) v += red[ww * 1024 + o];
    const int tile = o / 256, ln = (o % 256) / 4, e = o % 4;
    const int i = 16 * (tile >> 1) + 4 * e + ln / 16, j = 16 * (tile & 1) + ln % 16;
    if (i < p && j < q) out[i * q + j] = v;
  }
}

template <typename T, int KMAX>
int qr_dispatch(const QrBatch& b, int32_t* flag, hipStream_t s) {
  const dim3 rows_grid(kQrChunks, b.nb);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL((qr_rows_kernel<T, KMAX>), rows_grid, dim3(kQrThreads), 0, s,
                       b, pass);
    RT_LAUNCH_CHECK("qr rows");
    hipLaunchKernelGGL((qr_chol_kernel<KMAX>), dim3(b.nb), dim3(kQrThreads), 0, s,
                       b, pass);
    RT_LAUNCH_CHECK("qr chol");
  }
  hipLaunchKernelGGL((qr_rows_kernel<T, KMAX>), rows_grid, dim3(kQrThreads), 0, s, b,
                     2);
  RT_LAUNCH_CHECK("qr rows");
  hipLaunchKernelGGL((householder_kernel<T, KMAX>), dim3(b.nb), dim3(kQrThreads),
                     0, s, b, flag, static_cast<const int32_t*>(b.need));
  RT_LAUNCH_CHECK("qr fallback");
  return kOk;
}

}  // namespace

int64_t qr_work_doubles(int64_t I, int K) {
  return 2 * I * K + static_cast<int64_t>(kQrChunks + 1) * K * K;
}

template <typename T>
int launch_qr(const QrBatch& b, int32_t* flag, hipStream_t s) {
  int kmax = 0;
  int64_t imax = 0;
  for (int i = 0; i < b.nb; ++i) {
    kmax = b.K[i] > kmax ? b.K[i] : kmax;
    imax = b.I[i] > imax ? b.I[i] : imax;
  }
  if (kmax <= 32 && imax <= kQfMaxI) {
    // one workgroup per sketch; Householder for any that CholeskyQR2 rejects
    hipLaunchKernelGGL(qr_fused_kernel<T>, dim3(b.nb), dim3(kQfThreads), 0, s, b);
    RT_LAUNCH_CHECK("qr fused");
    hipLaunchKernelGGL((householder_kernel<T, 32>), dim3(b.nb), dim3(kQrThreads), 0, s, b,
                       flag, static_cast<const int32_t*>(b.need));
    RT_LAUNCH_CHECK("qr fallback");
    return kOk;
  }
  if (kmax <= 16) return qr_dispatch<T, 16>(b, flag, s);
  if (kmax <= 32) return qr_dispatch<T, 32>(b, flag, s);
  if (kmax <= 64) return qr_dispatch<T, 64>(b, flag, s);
  set_error("qr: width %d exceeds 64", kmax);
  return kErrUnsupported;
}

template int launch_qr<float>(const QrBatch&, int32_t*, hipStream_t);
template int launch_qr<double>(const QrBatch&, int32_t*, hipStream_t);

int launch_cross_tall(const CrossBatch& b, hipStream_t s) {
  for (int i = 0; i < b.nb; ++i) {
    if (b.p[i] < 1 || b.p[i] > 32 || b.q[i] < 1 || b.q[i] > 32 || b.I[i] < 1) {
      set_error("cross product: widths %d x %d unsupported", b.p[i], b.q[i]);
      return kErrUnsupported;
    }
  }
  hipLaunchKernelGGL(cross_tall_kernel, dim3(b.nb), dim3(kQfThreads), 0, s, b);
  RT_LAUNCH_CHECK("cross products");
  return kOk;
}

int launch_eig(const EigBatch& b, hipStream_t s) {
  for (int i = 0; i < b.nb; ++i) {
    if (b.n[i] > kEigMax || b.k[i] > b.n[i]) {
      set_error("eig: size %d (k=%d) unsupported", b.n[i], b.k[i]);
      return kErrUnsupported;
    }
  }
  int nmax = 0;
  for (int i = 0; i < b.nb; ++i) nmax = b.n[i] > nmax ? b.n[i] : nmax;
  if (nmax <= 32)
    hipLaunchKernelGGL(eig32_kernel, dim3(b.nb), dim3(kEigThreads), 0, s, b);
  else
    hipLaunchKernelGGL(eig_kernel, dim3(b.nb), dim3(kEigThreads), 0, s, b);
  RT_LAUNCH_CHECK("eig");
  return kOk;
}

}  // namespace rt
