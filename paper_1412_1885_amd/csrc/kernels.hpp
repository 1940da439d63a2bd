// Host-side launchers of the device kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt {

// modes per batched launch (at least the library's largest N)
constexpr int kBatchModes = 8;

// ---- generic mode-n product (ttm.hip) ------------------------------------
// out[a, k, c] = sum_i X[a, i, c] * M[i, k];  X: [A, I, C], M: I x K.
template <typename T>
int launch_ttm(const T* X, const T* M, T* out, int64_t A, int64_t I, int64_t C,
               int K, hipStream_t s);

// Z[i, r] = sum_{a, c} X[a, i, c] * Om[a*C + c, r]  (X_(n) Omega~_n).
template <typename T>
int launch_sketch_z(const T* X, const T* Om, T* Z, int64_t A, int64_t I,
                    int64_t C, int R, hipStream_t s);

// ---- sketch products from streamed intermediates (sketch.hip) ------------
// out[a, i, c] = sum_j B[i, j] X[a, j, c]  (expand mode: J -> I)
template <typename T>
int launch_expand(const T* X, const T* B, T* out, int64_t A, int64_t I, int J,
                  int64_t C, hipStream_t s);
// Z[i, r] = sum_{a, c} Tm[a, i, c] W[a*C + c, r]; part: split-K scratch of
// part_cap elements, at least sketch_part_elems(I, R). The split count aims
// at kSketchTargetBlocks workgroups of 64 rows, so S * I <= 64 * target + I.
constexpr int64_t kSketchTargetBlocks = 1024;
inline int64_t sketch_part_elems(int64_t I, int64_t R) {
  return (64 * kSketchTargetBlocks + I) * R;
}
template <typename T>
int launch_sketch_gemm(const T* Tm, const T* W, T* Z, T* part, int64_t part_cap,
                       int64_t A, int64_t I, int64_t C, int R, hipStream_t s);
// out[c][r] = in[r][c] (R x C matrix).
template <typename T>
int launch_transpose(const T* in, T* out, int64_t R, int64_t C, hipStream_t s);
// S = X_(n) X_(n)^T (FP64) for X viewed [A, I, C], one wavefront per entry.
template <typename T>
int launch_gram_waves(const T* X, double* S, int64_t A, int I, int64_t C,
                      hipStream_t s);
// The same for several views of one X in one launch: S[m] for the view
// [A[m], I[m], C[m]]; first[m] numbers mode m's upper-triangle entries
// (first[nb] is the total).
struct GramWavesBatch {
  double* S[kBatchModes];
  int64_t A[kBatchModes], C[kBatchModes];
  int I[kBatchModes];
  int first[kBatchModes + 1];
  int nb;
};
template <typename T>
int launch_gram_waves_batch(const T* X, const GramWavesBatch& b, hipStream_t s);
// out[a, k, c] = sum_i X[a, i, c] M[i, k] for C <= 64, K <= 64.
template <typename T>
int launch_ttm_small_c(const T* X, const T* M, T* out, int64_t A, int64_t I,
                       int C, int K, hipStream_t s);

// S = X_(n) X_(n)^T in FP64 for X viewed [A, I, C] (I <= 64).
template <typename T>
int launch_gram_unfold(const T* X, double* S, int64_t A, int I, int64_t C,
                       hipStream_t s);

// out[i, j] = sum_k Q[i, k] * W[k, j];  Q: I x K (T), W: K x J (FP64).
template <typename T>
int launch_matmul_w(const T* Q, const double* W, T* out, int64_t I, int K,
                    int J, hipStream_t s);

// Several modes in one launch: out[m] = Q[m] W[m] as in launch_matmul_w,
// then WT[m] = float(W[m]) (K[m] x J[m]) where WT[m] is set.  first[m] and
// wfirst[m] number the elements of each mode's product and copy (first[nb]
// and wfirst[nb] are the totals).
template <typename T>
struct MatWBatch {
  const T* Q[kBatchModes];
  const double* W[kBatchModes];
  T* out[kBatchModes];
  float* WT[kBatchModes];
  int64_t I[kBatchModes];
  int K[kBatchModes], J[kBatchModes];
  int64_t first[kBatchModes + 1], wfirst[kBatchModes + 1];
  int nb;
};
template <typename T>
int launch_matmul_w_batch(const MatWBatch<T>& b, hipStream_t s);

// partial[b] = sum of squares (FP64) over a grid-stride slice; flag |= !finite.
// Then out[0] = sum partials (fixed order).  n elements of T.
template <typename T>
int launch_norm2(const T* X, int64_t n, double* partial, int nblocks,
                 double* out, int32_t* nonfinite, hipStream_t s);
int launch_norm2_bf16(const uint16_t* X, int64_t n, double* partial,
                      int nblocks, double* out, int32_t* nonfinite,
                      hipStream_t s);
int norm2_blocks();

// out[0] = sum of nb partials (fixed order); flag |= 1 if it is not finite.
int launch_sum_partials(const double* partial, int nb, double* out,
                        int32_t* nonfinite, hipStream_t s);

int launch_fill_i32(int32_t* p, int32_t value, int64_t n, hipStream_t s);

// Fit of a CP model from X = Y x_1 A_1^T ... x_N A_N^T (an R^N tensor):
// <Y,Yhat> = sum_r lambda_r X[r,..,r]; ||Yhat||^2 from the Grams (eq. 9);
// ||Y||^2 = scal[0].  out3 = {fit, ||Y||^2, <Y,Yhat>}.
int launch_cp_fit_final(const float* X, int N, int R, const float* lambda,
                        double* const* grams, const double* scal, double* out3,
                        hipStream_t s);

// convert FP64 <-> T copies
template <typename Tin, typename Tout>
int launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t s);

// ---- small FP64 linear algebra (linalg.hip) -------------------------------
// Batched Householder QR: for b < nb, Zin[b] is I_b x K_b (row-major, T),
// Q_out[b] receives the orthonormal factor (diag(R) >= 0), T.  ws64 is a
// FP64 scratch of sum_b I_b*K_b*2 doubles.  rank_flag bit b set on a zero
// pivot.
struct QrBatch {
  const void* Z[16];
  void* Q[16];
  double* work[16];
  int64_t I[16];
  int K[16];
  int nb;
  int32_t* need;  // per-matrix flag: CholeskyQR2 failed, Householder ran
  int bit0;       // matrix m reports rank deficiency as bit bit0 + m
};
template <typename T>
int launch_qr(const QrBatch& b, int32_t* rank_flag, hipStream_t s);
// FP64 work doubles launch_qr needs per matrix (work[b])
int64_t qr_work_doubles(int64_t I, int K);

// Batched symmetric eigen-decomposition by cyclic Jacobi (FP64).
// S[b] is n_b x n_b (n_b <= 64), W[b] receives the top-k_b eigenvectors as
// an n_b x k_b row-major matrix (descending eigenvalues, ties by index,
// largest-|.| entry of each column positive); evals[b] (may be null) the
// sorted eigenvalues.
struct EigBatch {
  const double* S[16];
  double* W[16];
  double* evals[16];
  int n[16];
  int k[16];
  int nb;
};
int launch_eig(const EigBatch& b, hipStream_t s);

// out_m = X_m^T Y_m in FP64 (p_m x q_m, dense row-major) for row-major FP32
// X_m (I_m x p_m) and Y_m (I_m x q_m), p_m, q_m <= 32: one workgroup per
// product, FP64 matrix cores, a fixed summation order.
struct CrossBatch {
  const float* X[16];
  const float* Y[16];
  double* out[16];
  int64_t I[16];
  int p[16], q[16];
  int nb;
};
int launch_cross_tall(const CrossBatch& b, hipStream_t s);

// ---- FFCP (ffcp.hip) ------------------------------------------------------
struct FfcpArgs {
  int N, R, update, max_it;
  double tol, l1, normY2;
  int64_t I[8];
  int Rn[8];
  const float* U[8];
  const float* G;
  const float* A_init[8];  // user init (null when HOSVD)
  const double* V_init[8]; // coefficient start R_n x R in FP64 (HOSVD, padded, or caller's)
  const double* V_alt[8];  // guarded start: the HOSVD alternative, or null
  float* A_out[8];
  float* lambda;
  double* fit_trace;
  void* info;              // rt_ffcp_info*
  // FP64 workspace pointers
  double* A[8];
  double* V[8];
  double* Gram[8];
  double* U64[8];
  double* G64;
  double* H;       // max R_n x R
  double* Qm;      // max I_n x R
  double* T;       // R x R (+ Cholesky factor)
  double* W1;      // prod R / min R_p * R  (MTTKRP partial)
  double* W2;      // same size
  double* scal;    // scalars
  double* part;    // partial sums of the multi-workgroup kernel (null: one workgroup)
  unsigned* bar;   // its grid barrier: [0] arrivals, [1] failure flag (zeroed per launch)
  double* nrm;     // its column norms of each factor's last normalization (N x R)
};
int launch_ffcp(const FfcpArgs& a, hipStream_t s);
// doubles of FfcpArgs::part for cross products of at most nout_max outputs
int64_t ffcp_grid_part_doubles(int64_t nout_max);
// ALS without the l1 term, run in the compressed space (one workgroup, LDS
// resident); kErrUnsupported when the problem does not fit.
bool ffcp_als_core_applicable(const FfcpArgs& a);
int launch_ffcp_als_core(const FfcpArgs& a, hipStream_t s);

}  // namespace rt
