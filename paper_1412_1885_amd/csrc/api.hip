// C ABI of librtucker (declared in include/rtucker.h): argument validation,
// workspace planning and the launch sequence of RandTucker2i and FFCP.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/rtucker.h"
#include "common.hpp"
#include "kernels.hpp"
#include "profile.hpp"
#include "stream.hpp"

namespace rt {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("HIP error in %s: %s", what, hipGetErrorString(e));
  return kErrHip;
}

namespace {

bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

int check_ptr(const void* p, const char* name) {
  if (!p) {
    set_error("%s is NULL", name);
    return kErrInvalid;
  }
  if (!aligned16(p)) {
    set_error("%s is not 16-byte aligned", name);
    return kErrInvalid;
  }
  return kOk;
}

// ------------------------------------------------------------ tucker_rand

int validate_tucker(const rt_tucker_desc* d) {
  if (!d) {
    set_error("desc is NULL");
    return kErrInvalid;
  }
  if (d->N < 2 || d->N > RT_MAX_MODES) {
    set_error("N=%d outside 2..%d", d->N, RT_MAX_MODES);
    return kErrInvalid;
  }
  if (d->sweeps < 1 || d->sweeps > 2) {
    set_error("sweeps=%d (must be 1 or 2)", d->sweeps);
    return kErrInvalid;
  }
  if (d->precision != RT_F32 && d->precision != RT_BF16_MIXED &&
      d->precision != RT_F64) {
    set_error("unknown precision %d", d->precision);
    return kErrInvalid;
  }
  if (d->flags & ~(RT_FLAG_NO_TRUNCATE | RT_FLAG_BF16_INPUT | RT_FLAG_GAUSS_SEIDEL)) {
    set_error("unknown flag bits 0x%x", d->flags);
    return kErrInvalid;
  }
  if ((d->flags & RT_FLAG_BF16_INPUT) && d->precision != RT_BF16_MIXED) {
    set_error("RT_FLAG_BF16_INPUT requires RT_BF16_MIXED");
    return kErrInvalid;
  }
  int64_t total = 1;
  int64_t core = 1;
  for (int n = 0; n < d->N; ++n) {
    const int64_t I = d->dims[n];
    const int rt = d->ranks_tilde[n];
    if (I < 1) {
      set_error("dims[%d]=%lld < 1", n, (long long)I);
      return kErrInvalid;
    }
    if (rt < 1 || rt > RT_MAX_SKETCH || rt > I) {
      set_error("ranks_tilde[%d]=%d outside 1..min(I_n=%lld, %d)", n, rt,
                (long long)I, RT_MAX_SKETCH);
      return kErrInvalid;
    }
    if (!(d->flags & RT_FLAG_NO_TRUNCATE)) {
      if (d->ranks[n] < 1 || d->ranks[n] > rt) {
        set_error("ranks[%d]=%d outside 1..R~_n=%d", n, d->ranks[n], rt);
        return kErrInvalid;
      }
    }
    if (total > (int64_t(1) << 62) / I) {
      set_error("tensor size overflows 64 bits");
      return kErrInvalid;
    }
    total *= I;
    core *= rt;
  }
  if (core > (int64_t(1) << 26)) {
    set_error("sketch core prod R~_n = %lld too large", (long long)core);
    return kErrUnsupported;
  }
  if (d->precision == RT_BF16_MIXED)
    RT_TRY(bf16_check_shape(total / (d->dims[d->N - 2] * d->dims[d->N - 1]),
                            d->dims[d->N - 2], d->dims[d->N - 1],
                            d->ranks_tilde[d->N - 2], d->ranks_tilde[d->N - 1],
                            (d->flags & RT_FLAG_BF16_INPUT) != 0));
  return kOk;
}

template <typename T>
struct TuckerPlan {
  int N;
  int64_t I[RT_MAX_MODES];
  int K[RT_MAX_MODES];
  int Rn[RT_MAX_MODES];
  int64_t total, core, core_out;
  int64_t sizeTA, sizeTB, chain;
  // workspace carves
  double* partial;
  double* scal;   // [0] normY2 [1] normG2
  int32_t* iflags; // [0] nonfinite [1] rank
  T* TA;
  T* TB;
  T* Cs;   // TA x_{N-1} B_{N-1}^T per slab, [prod_{p<N-1} I_p, R~_{N-1}, R~_N]
  T* X0;
  T* X1;
  T* Z[RT_MAX_MODES];
  T* Q[RT_MAX_MODES];
  double* qrwork[RT_MAX_MODES];
  T* Gt;
  T* Gtmp;
  T* W0;
  T* W1;
  T* zpart;
  int64_t zpart_cap;
  double* gram[RT_MAX_MODES];
  double* W[RT_MAX_MODES];
  T* WT[RT_MAX_MODES];
  uint16_t* stream_scratch;
  size_t stream_bytes;
  void* stream_ws;

  size_t plan(const rt_tucker_desc* d, void* ws) {
    Arena ar(ws);
    N = d->N;
    total = 1;
    core = 1;
    core_out = 1;
    const bool trunc = !(d->flags & RT_FLAG_NO_TRUNCATE);
    for (int n = 0; n < N; ++n) {
      I[n] = d->dims[n];
      K[n] = d->ranks_tilde[n];
      Rn[n] = trunc ? d->ranks[n] : K[n];
      total *= I[n];
      core *= K[n];
      core_out *= Rn[n];
    }
    const int last = N - 1, second = N - 2;
    sizeTA = total / I[last] * K[last];
    sizeTB = total / I[second] * K[second];
    chain = sizeTA > sizeTB ? sizeTA : sizeTB;
    partial = ar.take<double>(norm2_blocks());
    scal = ar.take<double>(8);
    iflags = ar.take<int32_t>(8 + 16);
    TA = ar.take<T>(sizeTA);
    TB = ar.take<T>(sizeTB);
    Cs = ar.take<T>(sizeTA / I[second] * K[second]);
    X0 = ar.take<T>(chain);
    X1 = ar.take<T>(chain);
    for (int n = 0; n < N; ++n) {
      Z[n] = ar.take<T>(I[n] * K[n]);
      Q[n] = ar.take<T>(I[n] * K[n]);
      qrwork[n] = ar.take<double>(qr_work_doubles(I[n], K[n]));
      gram[n] = ar.take<double>(K[n] * K[n]);
      W[n] = ar.take<double>(K[n] * K[n]);
      WT[n] = ar.take<T>(K[n] * K[n]);
    }
    Gt = ar.take<T>(core);
    Gtmp = ar.take<T>(core);
    // expanded test matrices W_n and split-K partials of the sketch product
    int64_t wmax = 0, imax = 0;
    int kmax = 0;
    for (int n = 0; n < N; ++n) {
      const int64_t tsize = (n == last) ? sizeTB : sizeTA;
      const int64_t w = tsize / I[n] * K[n];
      wmax = w > wmax ? w : wmax;
      imax = I[n] > imax ? I[n] : imax;
      kmax = K[n] > kmax ? K[n] : kmax;
    }
    W0 = ar.take<T>(wmax);
    W1 = ar.take<T>(wmax);
    // the last core contraction also runs through the split-K product with
    // prod_{p>1} R~_p rows
    const int64_t rows_max = imax > core / K[0] ? imax : core / K[0];
    zpart_cap = sketch_part_elems(rows_max, kmax);
    zpart = ar.take<T>(zpart_cap);
    stream_bytes = stream_workspace_bytes(d);
    stream_ws = ar.take<char>(stream_bytes);
    return ar.need;
  }
};

// X_n = base x_{p in modes} B_p^T, contracting in increasing p; dims `D`
// are updated in place.  Returns the buffer holding the result.
template <typename T>
int contract_chain(const T* base, int64_t* D, int N, const int* modes,
                   int nmodes, const T* const* B, const int* K, T* buf0,
                   T* buf1, const T** result, hipStream_t s) {
  const T* src = base;
  T* bufs[2] = {buf0, buf1};
  int cur = 0;
  for (int q = 0; q < nmodes; ++q) {
    const int p = modes[q];
    int64_t Apre = 1, Cpost = 1;
    for (int r = 0; r < p; ++r) Apre *= D[r];
    for (int r = p + 1; r < N; ++r) Cpost *= D[r];
    RT_TRY(launch_ttm<T>(src, B[p], bufs[cur], Apre, D[p], Cpost, K[p], s));
    D[p] = K[p];
    src = bufs[cur];
    cur ^= 1;
  }
  *result = src;
  return kOk;
}

// Z_n = X_(n) Omega~_n from the streamed intermediate T (TA for n < N-1,
// TB for n = N-1; for n < N-2, when the pass made it, C = TA x_{N-1}
// B_{N-1}^T, 1/I_{N-1}-th of TA's size): W_n = Omega~_n expanded by B_p in
// every mode p that T still holds at full size (p != n), then
// Z_n[i, r] = sum_{a,c} T[a,i,c] W_n[a,c,r] (split-K product).
template <typename T, typename Plan>
int sketch_from_intermediate(Plan& P, int n, const T* const* B, const T* Omt, bool use_c,
                             hipStream_t s) {
  const int N = P.N, last = N - 1, second = N - 2;
  int64_t D[RT_MAX_MODES];
  for (int p = 0; p < N; ++p) D[p] = P.I[p];
  const T* base;
  // modes the intermediate already holds at R~_p
  const bool from_c = use_c && n < second;
  const int contracted = (n != last) ? last : second;
  if (from_c) {
    base = P.Cs;
    D[last] = P.K[last];
    D[second] = P.K[second];
  } else if (n != last) {
    base = P.TA;
    D[last] = P.K[last];
  } else {
    base = P.TB;
    D[second] = P.K[second];
  }
  // W dims: modes p != n in order (all K_p initially), then R~_n.
  int64_t Wd[RT_MAX_MODES];
  int wm[RT_MAX_MODES], nw = 0;
  for (int p = 0; p < N; ++p)
    if (p != n) {
      wm[nw] = p;
      Wd[nw++] = P.K[p];
    }
  const T* src = Omt;
  T* bufs[2] = {P.W0, P.W1};
  int cur = 0;
  for (int q = 0; q < nw; ++q) {
    const int p = wm[q];
    if (p == contracted || (from_c && p == second)) continue;  // held at K_p
    int64_t Apre = 1, Cpost = P.K[n];
    for (int r = 0; r < q; ++r) Apre *= Wd[r];
    for (int r = q + 1; r < nw; ++r) Cpost *= Wd[r];
    RT_TRY(launch_expand<T>(src, B[p], bufs[cur], Apre, P.I[p], P.K[p], Cpost, s));
    Wd[q] = P.I[p];
    src = bufs[cur];
    cur ^= 1;
  }
  int64_t Apre = 1, Cpost = 1;
  for (int p = 0; p < n; ++p) Apre *= D[p];
  for (int p = n + 1; p < N; ++p) Cpost *= D[p];
  return launch_sketch_gemm<T>(base, src, P.Z[n], P.zpart, P.zpart_cap, Apre, P.I[n], Cpost,
                               P.K[n], s);
}

template <typename T>
int tucker_run(const rt_tucker_desc* d, const void* Yv, const void* const* Om,
               const void* const* Omt, void* ws, size_t ws_bytes,
               void* const* Uout, void* Gout, uint16_t* Ybf16,
               rt_tucker_info* info, const rt_tucker_trace* trace,
               hipStream_t s) {
  TuckerPlan<T> P;
  const size_t need = P.plan(d, ws);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  const int N = P.N, last = N - 1, second = N - 2;
  RT_TRY(launch_fill_i32(P.iflags, 0, 8, s));

  // ||Y||^2 and the non-finite flag come from the first streamed pass.
  const T* B[RT_MAX_MODES];
  for (int n = 0; n < N; ++n) B[n] = static_cast<const T*>(Om[n]);
  StreamCtx sc = make_stream_ctx(d, Yv, Ybf16, P.stream_ws, P.stream_bytes,
                                 P.scal + 0, P.iflags + 0);

  // QR of the sketches of modes n0..n1-1 into Q (one batched launch)
  auto qr_modes = [&](int n0, int n1) {
    ProfScope ps(kStageQr, s);
    QrBatch qb{};
    qb.nb = n1 - n0;
    qb.bit0 = n0;
    qb.need = P.iflags + 4;
    for (int n = n0; n < n1; ++n) {
      qb.Z[n - n0] = P.Z[n];
      qb.Q[n - n0] = P.Q[n];
      qb.work[n - n0] = P.qrwork[n];
      qb.I[n - n0] = P.I[n];
      qb.K[n - n0] = P.K[n];
    }
    return launch_qr<T>(qb, P.iflags + 1, s);
  };
  const bool gauss_seidel = (d->flags & RT_FLAG_GAUSS_SEIDEL) != 0;
  int pass = 0;   // streamed passes so far (the first one converts / takes ||Y||^2)

  for (int sw = 0; sw < d->sweeps; ++sw) {
    const T* const* Omt_s = reinterpret_cast<const T* const*>(Omt) + sw * N;
    if (!gauss_seidel) {
      // Jacobi: one streamed pass, TA = Y x_last B_last^T and
      // TB = Y x_second B_second^T, serves every mode of the sweep
      bool cdone = false;
      RT_TRY(stream_dual<T>(sc, pass++, B[last], P.K[last], B[second], P.K[second], P.TA,
                            P.TB, N >= 3 ? P.Cs : nullptr, &cdone, s));
      {
        ProfScope ps(kStageContract, s);
        for (int n = 0; n < N; ++n)
          RT_TRY(sketch_from_intermediate<T>(P, n, B, Omt_s[n], cdone, s));
      }
      RT_TRY(qr_modes(0, N));
    } else {
      // Gauss-Seidel (the loop of Algorithm 3 as printed): mode n's sketch
      // uses the bases modes < n received in this sweep.  Modes < N-1 are
      // reached from TA = Y x_last B_last^T, which only mode N-1 changes, so
      // one pass serves them one after the other; mode N-1 needs
      // TB = Y x_second Q_second^T with the new basis of mode N-2: a second
      // pass (its TA is not used).
      // (C = TA x_{N-1} B_{N-1}^T holds the previous basis of mode N-1,
      // which is what modes < N-1 use in this order)
      bool cdone = false;
      RT_TRY(stream_dual<T>(sc, pass++, B[last], P.K[last], B[second], P.K[second], P.TA,
                            P.TB, N >= 3 ? P.Cs : nullptr, &cdone, s));
      for (int n = 0; n < last; ++n) {
        {
          ProfScope ps(kStageContract, s);
          RT_TRY(sketch_from_intermediate<T>(P, n, B, Omt_s[n], cdone, s));
        }
        RT_TRY(qr_modes(n, n + 1));
        B[n] = P.Q[n];
      }
      RT_TRY(stream_dual<T>(sc, pass++, B[last], P.K[last], B[second], P.K[second], P.TA,
                            P.TB, nullptr, nullptr, s));
      {
        ProfScope ps(kStageContract, s);
        RT_TRY(sketch_from_intermediate<T>(P, last, B, Omt_s[last], false, s));
      }
      RT_TRY(qr_modes(last, N));
    }
    if (trace) {
      for (int n = 0; n < N; ++n) {
        const size_t bytes = P.I[n] * P.K[n] * sizeof(T);
        if (trace->Z[sw * N + n] &&
            hipMemcpyAsync(trace->Z[sw * N + n], P.Z[n], bytes,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
          return hip_fail(hipGetLastError(), "trace copy");
        if (trace->Q[sw * N + n] &&
            hipMemcpyAsync(trace->Q[sw * N + n], P.Q[n], bytes,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
          return hip_fail(hipGetLastError(), "trace copy");
      }
    }
    for (int n = 0; n < N; ++n) B[n] = P.Q[n];
  }

  // core G~ = Y x_1 Q_1^T ... x_N Q_N^T: streamed mode first (with mode
  // N-1 inside the pass where it can), then the rest
  bool cdone = false;
  RT_TRY(stream_single<T>(sc, pass, B[last], P.K[last], B[second], P.K[second], P.TA,
                          N >= 3 ? P.Cs : nullptr, &cdone, s));
  {
    ProfScope ps(kStageContract, s);
    int64_t D[RT_MAX_MODES];
    for (int p = 0; p < N; ++p) D[p] = P.I[p];
    D[last] = P.K[last];
    const T* src = P.TA;
    int pstart = last - 1;
    if (cdone) {
      src = P.Cs;
      D[second] = P.K[second];
      pstart = second - 1;
    }
    T* bufs[2] = {P.X0, P.X1};
    int cur = 0;
    for (int p = pstart; p >= 1; --p) {  // innermost remaining mode first
      int64_t Apre = 1, Cpost = 1;
      for (int q = 0; q < p; ++q) Apre *= D[q];
      for (int q = p + 1; q < N; ++q) Cpost *= D[q];
      if (Cpost <= 64)
        RT_TRY(launch_ttm_small_c<T>(src, B[p], bufs[cur], Apre, D[p],
                                     static_cast<int>(Cpost), P.K[p], s));
      else
        RT_TRY(launch_ttm<T>(src, B[p], bufs[cur], Apre, D[p], Cpost, P.K[p], s));
      D[p] = P.K[p];
      src = bufs[cur];
      cur ^= 1;
    }
    // mode 1 last, as one split-K product over I_1 (rows = the other core
    // indices), then transposed into G~ = [R~_1, ...].
    const int64_t rest = P.core / P.K[0];
    RT_TRY(launch_sketch_gemm<T>(src, B[0], bufs[cur], P.zpart, P.zpart_cap, P.I[0], rest, 1,
                                 P.K[0], s));
    RT_TRY(launch_transpose<T>(bufs[cur], P.Gt, rest, P.K[0], s));
  }
  if (trace && trace->Gt &&
      hipMemcpyAsync(trace->Gt, P.Gt, P.core * sizeof(T),
                     hipMemcpyDeviceToDevice, s) != hipSuccess)
    return hip_fail(hipGetLastError(), "trace copy");

  if (d->flags & RT_FLAG_NO_TRUNCATE) {
    for (int n = 0; n < N; ++n)
      if (hipMemcpyAsync(Uout[n], P.Q[n], P.I[n] * P.K[n] * sizeof(T),
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return hip_fail(hipGetLastError(), "U copy");
    if (hipMemcpyAsync(Gout, P.Gt, P.core * sizeof(T), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
      return hip_fail(hipGetLastError(), "G copy");
  } else {
    ProfScope ps(kStageTruncate, s);
    EigBatch eb{};
    eb.nb = N;
    static_assert(kBatchModes >= RT_MAX_MODES, "a batch holds every mode");
    GramWavesBatch gb{};
    gb.nb = N;
    int64_t Apre = 1;
    for (int n = 0; n < N; ++n) {
      gb.S[n] = P.gram[n];
      gb.A[n] = Apre;
      gb.I[n] = P.K[n];
      gb.C[n] = P.core / (Apre * P.K[n]);
      gb.first[n + 1] = gb.first[n] + P.K[n] * (P.K[n] + 1) / 2;
      Apre *= P.K[n];
      eb.S[n] = P.gram[n];
      eb.W[n] = P.W[n];
      eb.evals[n] = nullptr;
      eb.n[n] = P.K[n];
      eb.k[n] = P.Rn[n];
    }
    RT_TRY(launch_gram_waves_batch<T>(P.Gt, gb, s));
    RT_TRY(launch_eig(eb, s));
    // U_n = Q_n W_n for every mode, and the FP32 copies of W_n, in one launch
    const T* WT[RT_MAX_MODES];
    MatWBatch<T> mb{};
    mb.nb = N;
    for (int n = 0; n < N; ++n) {
      mb.Q[n] = P.Q[n];
      mb.W[n] = P.W[n];
      mb.out[n] = static_cast<T*>(Uout[n]);
      mb.I[n] = P.I[n];
      mb.K[n] = P.K[n];
      mb.J[n] = P.Rn[n];
      mb.first[n + 1] = mb.first[n] + P.I[n] * P.Rn[n];
      if (sizeof(T) == sizeof(double)) {
        mb.WT[n] = nullptr;
        mb.wfirst[n + 1] = mb.wfirst[n];
        WT[n] = reinterpret_cast<const T*>(P.W[n]);
      } else {
        mb.WT[n] = reinterpret_cast<float*>(P.WT[n]);
        mb.wfirst[n + 1] = mb.wfirst[n] + static_cast<int64_t>(P.K[n]) * P.Rn[n];
        WT[n] = P.WT[n];
      }
    }
    RT_TRY(launch_matmul_w_batch<T>(mb, s));
    int64_t D[RT_MAX_MODES];
    for (int p = 0; p < N; ++p) D[p] = P.K[p];
    int modes[RT_MAX_MODES];
    for (int p = 0; p < N; ++p) modes[p] = p;
    const T* X;
    RT_TRY(contract_chain<T>(P.Gt, D, N, modes, N, WT, P.Rn, P.Gtmp, P.X1, &X,
                             s));
    if (hipMemcpyAsync(Gout, X, P.core_out * sizeof(T), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
      return hip_fail(hipGetLastError(), "G copy");
  }
  RT_TRY(launch_norm2<T>(static_cast<const T*>(Gout), P.core_out, P.partial,
                         norm2_blocks(), P.scal + 1, P.iflags + 2, s));
  if (info) {
    // scal[0..1] -> normY2, normG2; iflags[0] nonfinite, iflags[1] rank
    if (hipMemcpyAsync(info, P.scal, 2 * sizeof(double), hipMemcpyDeviceToDevice,
                       s) != hipSuccess ||
        hipMemcpyAsync(reinterpret_cast<char*>(info) + 16, P.iflags,
                       2 * sizeof(int32_t), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
      return hip_fail(hipGetLastError(), "info copy");
  }
  return kOk;
}

// ------------------------------------------------------------------ ffcp

int validate_ffcp(const rt_ffcp_desc* d) {
  if (!d) {
    set_error("desc is NULL");
    return kErrInvalid;
  }
  if (d->N < 2 || d->N > RT_MAX_MODES) {
    set_error("N=%d outside 2..%d", d->N, RT_MAX_MODES);
    return kErrInvalid;
  }
  if (d->R < 1 || d->R > RT_MAX_SKETCH) {
    set_error("R=%d outside 1..%d", d->R, RT_MAX_SKETCH);
    return kErrInvalid;
  }
  if (d->update < 0 || d->update > 2) {
    set_error("unknown update rule %d", d->update);
    return kErrInvalid;
  }
  if (d->init < 0 || d->init > 3) {
    set_error("unknown init %d", d->init);
    return kErrInvalid;
  }
  if (d->max_it < 1) {
    set_error("max_it=%d < 1", d->max_it);
    return kErrInvalid;
  }
  if (!(d->tol >= 0.0) || !(d->l1 >= 0.0)) {
    set_error("tol and l1 must be >= 0");
    return kErrInvalid;
  }
  int64_t core = 1;
  for (int n = 0; n < d->N; ++n) {
    if (d->dims[n] < 1 || d->ranks[n] < 1 || d->ranks[n] > RT_MAX_SKETCH ||
        d->ranks[n] > d->dims[n]) {
      set_error("mode %d: I=%lld R_n=%d invalid", n, (long long)d->dims[n],
                d->ranks[n]);
      return kErrInvalid;
    }
    core *= d->ranks[n];
  }
  if (core > (int64_t(1) << 24)) {
    set_error("core too large for the FFCP kernel");
    return kErrUnsupported;
  }
  return kOk;
}

struct FfcpPlan {
  double* A[RT_MAX_MODES];
  double* V[RT_MAX_MODES];
  double* Gram[RT_MAX_MODES];
  double* U64[RT_MAX_MODES];
  double* G64;
  double* H;
  double* Qm;
  double* T;
  double* W1;
  double* W2;
  double* scal;
  double* part;
  unsigned* bar;
  double* nrm;
  double* Vinit[RT_MAX_MODES];
  double* Valt[RT_MAX_MODES];
  double* hgram[RT_MAX_MODES];
  size_t plan(const rt_ffcp_desc* d, void* ws) {
    Arena ar(ws);
    const int N = d->N, R = d->R;
    int64_t core = 1, Imax = 1;
    int Rmin = 1 << 30, Rmax = 0;
    for (int n = 0; n < N; ++n) {
      core *= d->ranks[n];
      Imax = d->dims[n] > Imax ? d->dims[n] : Imax;
      Rmin = d->ranks[n] < Rmin ? d->ranks[n] : Rmin;
      Rmax = d->ranks[n] > Rmax ? d->ranks[n] : Rmax;
    }
    // MTTKRP intermediates (rows padded to a multiple of 4 columns) and the
    // core-sized chain of the ||Yt||^2 computation
    int64_t wsize = core / Rmin * ((R + 3) / 4 * 4);
    if (wsize < core) wsize = core;
    for (int n = 0; n < N; ++n) {
      A[n] = ar.take<double>(d->dims[n] * R);
      V[n] = ar.take<double>(static_cast<int64_t>(d->ranks[n]) * R);
      Gram[n] = ar.take<double>(R * R);
      U64[n] = ar.take<double>(d->dims[n] * d->ranks[n]);
      Vinit[n] = ar.take<double>(static_cast<int64_t>(d->ranks[n]) * R);
      Valt[n] = ar.take<double>(static_cast<int64_t>(d->ranks[n]) * R);
      hgram[n] = ar.take<double>(static_cast<int64_t>(d->ranks[n]) * d->ranks[n]);
    }
    G64 = ar.take<double>(core);
    int64_t hs = static_cast<int64_t>(Rmax) * (R > Rmax ? R : Rmax);
    H = ar.take<double>(hs);
    // I_n x R lift (generic kernel) or the first MTTKRP step (compressed ALS)
    Qm = ar.take<double>(Imax * R > wsize ? Imax * R : wsize);
    T = ar.take<double>(R * R);
    W1 = ar.take<double>(wsize);
    W2 = ar.take<double>(wsize);
    scal = ar.take<double>(8 + RT_MAX_SKETCH);
    // per-workgroup partial sums of the multi-workgroup kernel: U_n^T A_n
    // with A_n^T A_n, U_n^T U_n, column norms
    int64_t nout = static_cast<int64_t>(Rmax) * R + static_cast<int64_t>(R) * R;
    if (static_cast<int64_t>(Rmax) * Rmax > nout) nout = static_cast<int64_t>(Rmax) * Rmax;
    part = ar.take<double>(ffcp_grid_part_doubles(nout));
    bar = ar.take<unsigned>(64);
    nrm = ar.take<double>(static_cast<int64_t>(N) * R);
    return ar.need;
  }
};

__global__ void hosvd_pad_kernel(const double* W, const float* pad, double* V,
                                 int Rn, int k, int R) {
  // V[j, r] = W[j, r] for r < k, pad[j, r-k] for r >= k
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= Rn * R) return;
  const int j = l / R, r = l % R;
  V[l] = (r < k) ? W[j * k + r] : static_cast<double>(pad[j * (R - k) + (r - k)]);
}

}  // namespace
}  // namespace rt

namespace rt {
namespace {

// ---------------------------------------------------- rt_ffcp_noalloc

// Scratch of rt_ffcp_noalloc: one copy per GPU, loaded with the code object
// and held until the process ends.  Host code never passes `scratch` itself
// to a kernel (on the host it is a stand-in, not a device address): it uses
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace
}  // namespace rt

static __device__ __align__(256) char scratch[rt::kNoallocScratchBytes];

namespace rt {
namespace {

// Device address of this device's `scratch`, looked up once per device with
// that device current.
int noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside 0..%d", dev, kMaxDevices - 1);
    return kErrNoDevice;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      set_error("hipGetSymbolAddress(scratch) returned NULL");
      return kErrHip;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return kOk;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_tucker_rand_workspace(const rt_tucker_desc* desc, size_t* bytes) {
  RT_TRY(validate_tucker(desc));
  if (!bytes) {
    set_error("bytes is NULL");
    return kErrInvalid;
  }
  if (desc->precision == RT_F64) {
    TuckerPlan<double> p;
    *bytes = p.plan(desc, nullptr);
  } else {
    TuckerPlan<float> p;
    *bytes = p.plan(desc, nullptr);
  }
  return kOk;
}

int rt_tucker_bf16_copy_elems(const rt_tucker_desc* desc, int64_t* elems) {
  RT_TRY(validate_tucker(desc));
  if (!elems) {
    set_error("elems is NULL");
    return kErrInvalid;
  }
  if (desc->precision != RT_BF16_MIXED || (desc->flags & RT_FLAG_BF16_INPUT)) {
    *elems = 0;
    return kOk;
  }
  int64_t e = bf16_copy_ld(desc->dims[desc->N - 1]);
  for (int p = 0; p < desc->N - 1; ++p) e *= desc->dims[p];
  *elems = e;
  return kOk;
}

int rt_tucker_rand(const rt_tucker_desc* desc, const void* Y,
                   const void* const* Omega, const void* const* Omega_t,
                   void* ws, size_t ws_bytes, void* const* U, void* G,
                   uint16_t* Ybf16, rt_tucker_info* info,
                   const rt_tucker_trace* trace, void* stream) {
  RT_TRY(validate_tucker(desc));
  RT_TRY(check_ptr(Y, "Y"));
  RT_TRY(check_ptr(ws, "ws"));
  RT_TRY(check_ptr(G, "G"));
  if (!Omega || !Omega_t || !U) {
    set_error("Omega, Omega_t and U arrays must not be NULL");
    return kErrInvalid;
  }
  for (int n = 0; n < desc->N; ++n) {
    RT_TRY(check_ptr(Omega[n], "Omega[n]"));
    RT_TRY(check_ptr(U[n], "U[n]"));
    for (int s = 0; s < desc->sweeps; ++s)
      RT_TRY(check_ptr(Omega_t[s * desc->N + n], "Omega_t[s*N+n]"));
  }
  const bool mixed = desc->precision == RT_BF16_MIXED;
  if (mixed && !(desc->flags & RT_FLAG_BF16_INPUT)) RT_TRY(check_ptr(Ybf16, "Ybf16"));
  if (info && !aligned16(info)) {
    set_error("info is not 16-byte aligned");
    return kErrInvalid;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (desc->precision == RT_F64)
    return tucker_run<double>(desc, Y, Omega, Omega_t, ws, ws_bytes, U, G,
                              Ybf16, info, trace, s);
  return tucker_run<float>(desc, Y, Omega, Omega_t, ws, ws_bytes, U, G, Ybf16,
                           info, trace, s);
}

int rt_ffcp_workspace(const rt_ffcp_desc* desc, size_t* bytes) {
  RT_TRY(validate_ffcp(desc));
  if (!bytes) {
    set_error("bytes is NULL");
    return kErrInvalid;
  }
  FfcpPlan p;
  *bytes = p.plan(desc, nullptr);
  return kOk;
}

int rt_ffcp(const rt_ffcp_desc* desc, const float* const* U, const float* G,
            const float* const* A_init, const float* const* pad, void* ws,
            size_t ws_bytes, float* const* A, float* lambda, double* fit_trace,
            rt_ffcp_info* info, void* stream) {
  RT_TRY(validate_ffcp(desc));
  RT_TRY(check_ptr(G, "G"));
  RT_TRY(check_ptr(ws, "ws"));
  RT_TRY(check_ptr(lambda, "lambda"));
  if (!U || !A) {
    set_error("U and A arrays must not be NULL");
    return kErrInvalid;
  }
  const int N = desc->N, R = desc->R;
  for (int n = 0; n < N; ++n) {
    RT_TRY(check_ptr(U[n], "U[n]"));
    RT_TRY(check_ptr(A[n], "A[n]"));
  }
  const bool coeff = desc->init == RT_INIT_COEFF || desc->init == RT_INIT_COEFF_GUARDED;
  const bool hosvd = desc->init == RT_INIT_HOSVD || desc->init == RT_INIT_COEFF_GUARDED;
  if (desc->init == RT_INIT_USER || coeff) {
    if (!A_init) {
      set_error("A_init is NULL with RT_INIT_USER / RT_INIT_COEFF");
      return kErrInvalid;
    }
    for (int n = 0; n < N; ++n) RT_TRY(check_ptr(A_init[n], "A_init[n]"));
  }
  if (hosvd) {
    for (int n = 0; n < N; ++n) {
      if (R > desc->ranks[n]) {
        if (!pad || !pad[n]) {
          set_error("HOSVD init with R > R_%d needs pad[%d]", n, n);
          return kErrInvalid;
        }
        RT_TRY(check_ptr(pad[n], "pad[n]"));
      }
    }
  }
  if ((info && !aligned16(info)) || (fit_trace && !aligned16(fit_trace))) {
    set_error("info / fit_trace not 16-byte aligned");
    return kErrInvalid;
  }
  FfcpPlan P;
  const size_t need = P.plan(desc, ws);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  FfcpArgs a{};
  a.N = N;
  a.R = R;
  a.update = desc->update;
  a.max_it = desc->max_it;
  a.tol = desc->tol;
  a.l1 = desc->l1;
  a.normY2 = (std::isnan(desc->normY2) || desc->normY2 < 0.0) ? -1.0 : desc->normY2;
  a.G = G;
  a.lambda = lambda;
  a.fit_trace = fit_trace;
  a.info = info;
  for (int n = 0; n < N; ++n) {
    a.I[n] = desc->dims[n];
    a.Rn[n] = desc->ranks[n];
    a.U[n] = U[n];
    a.A_out[n] = A[n];
    a.A[n] = P.A[n];
    a.V[n] = P.V[n];
    a.Gram[n] = P.Gram[n];
    a.U64[n] = P.U64[n];
    a.A_init[n] = desc->init == RT_INIT_USER ? A_init[n] : nullptr;
    a.V_init[n] = P.Vinit[n];
    a.V_alt[n] = desc->init == RT_INIT_COEFF_GUARDED ? P.Valt[n] : nullptr;
  }
  a.G64 = P.G64;
  a.H = P.H;
  a.Qm = P.Qm;
  a.T = P.T;
  a.W1 = P.W1;
  a.W2 = P.W2;
  a.scal = P.scal;
  a.part = P.part;
  a.bar = P.bar;
  a.nrm = P.nrm;
  if (coeff) {
    // the caller's coefficient matrices (FP32 R_n x R) as the FP64 start
    for (int n = 0; n < N; ++n)
      RT_TRY((launch_convert<float, double>(
          A_init[n], P.Vinit[n], static_cast<int64_t>(desc->ranks[n]) * R, s)));
  }
  if (hosvd) {
    // V_n = top-min(R, R_n) eigenvectors of G_(n) G_(n)^T, padded with the
    // caller's columns when R > R_n; the kernel then forms A_n = U_n V_n.
    // With the guarded start this is the alternative the kernel compares.
    double* const* dstV = desc->init == RT_INIT_COEFF_GUARDED ? P.Valt : P.Vinit;
    int64_t core = 1;
    for (int n = 0; n < N; ++n) core *= desc->ranks[n];
    // The Grams are formed one wavefront per entry, and the N eigenproblems
    // run as one batch. Each writes its R_n x k eigenvectors over its own
    // Gram: the eigensolver reads its whole input before writing.
    int64_t Apre = 1;
    EigBatch eb{};
    eb.nb = N;
    GramWavesBatch gb{};
    gb.nb = N;
    for (int n = 0; n < N; ++n) {
      const int Rn = desc->ranks[n];
      gb.S[n] = P.hgram[n];
      gb.A[n] = Apre;
      gb.I[n] = Rn;
      gb.C[n] = core / (Apre * Rn);
      gb.first[n + 1] = gb.first[n] + Rn * (Rn + 1) / 2;
      Apre *= Rn;
      eb.S[n] = P.hgram[n];
      eb.W[n] = P.hgram[n];
      eb.evals[n] = nullptr;
      eb.n[n] = Rn;
      eb.k[n] = R < Rn ? R : Rn;
    }
    RT_TRY(launch_gram_waves_batch<float>(G, gb, s));
    RT_TRY(launch_eig(eb, s));
    for (int n = 0; n < N; ++n) {
      const int Rn = desc->ranks[n];
      const int k = eb.k[n];
      hipLaunchKernelGGL(hosvd_pad_kernel, dim3((Rn * R + 255) / 256), dim3(256),
                         0, s, P.hgram[n], (k < R) ? pad[n] : nullptr, dstV[n], Rn,
                         k, R);
      RT_LAUNCH_CHECK("hosvd pad");
    }
  }
  ProfScope ps(kStageFfcp, s);
  if (ffcp_als_core_applicable(a)) {
    const int rc = launch_ffcp_als_core(a, s);
    if (rc != kErrUnsupported) return rc;
  }
  return launch_ffcp(a, s);
}

namespace {

// The FFCP stage of rt_ffcp_dense fits the Tucker format rt_tucker_rand
// returns: same order and sizes, FP32.
int validate_dense(const rt_tucker_desc* td, const rt_ffcp_desc* fd) {
  RT_TRY(validate_tucker(td));
  RT_TRY(validate_ffcp(fd));
  if (td->precision == RT_F64) {
    set_error("rt_ffcp_dense: FFCP reads an FP32 Tucker format (RT_F32 or "
              "RT_BF16_MIXED)");
    return kErrUnsupported;
  }
  if (fd->N != td->N) {
    set_error("rt_ffcp_dense: FFCP N=%d differs from the tensor's N=%d", fd->N, td->N);
    return kErrInvalid;
  }
  const bool trunc = !(td->flags & RT_FLAG_NO_TRUNCATE);
  for (int n = 0; n < td->N; ++n) {
    const int rn = trunc ? td->ranks[n] : td->ranks_tilde[n];
    if (fd->dims[n] != td->dims[n] || fd->ranks[n] != rn) {
      set_error("rt_ffcp_dense: mode %d of the FFCP description (I=%lld, R_n=%d) "
                "differs from the Tucker output (I=%lld, R_n=%d)",
                n, (long long)fd->dims[n], fd->ranks[n], (long long)td->dims[n], rn);
      return kErrInvalid;
    }
  }
  return kOk;
}

struct DensePlan {
  void* tws;
  size_t tbytes;
  float* U[RT_MAX_MODES];
  float* G;
  void* fws;
  size_t fbytes;
  size_t plan(const rt_tucker_desc* td, const rt_ffcp_desc* fd, void* ws) {
    Arena ar(ws);
    if (td->precision == RT_F64) {
      TuckerPlan<double> p;
      tbytes = p.plan(td, nullptr);
    } else {
      TuckerPlan<float> p;
      tbytes = p.plan(td, nullptr);
    }
    FfcpPlan fp;
    fbytes = fp.plan(fd, nullptr);
    tws = ar.take<char>(tbytes);
    int64_t core = 1;
    for (int n = 0; n < fd->N; ++n) {
      U[n] = ar.take<float>(fd->dims[n] * fd->ranks[n]);
      core *= fd->ranks[n];
    }
    G = ar.take<float>(core);
    fws = ar.take<char>(fbytes);
    return ar.need;
  }
};

}  // namespace

int rt_ffcp_dense_workspace(const rt_tucker_desc* tdesc, const rt_ffcp_desc* fdesc,
                            size_t* bytes) {
  RT_TRY(validate_dense(tdesc, fdesc));
  if (!bytes) {
    set_error("bytes is NULL");
    return kErrInvalid;
  }
  DensePlan p;
  *bytes = p.plan(tdesc, fdesc, nullptr);
  return kOk;
}

int rt_ffcp_dense(const rt_tucker_desc* tdesc, const rt_ffcp_desc* fdesc, const void* Y,
                  const void* const* Omega, const void* const* Omega_t, uint16_t* Ybf16,
                  const float* const* A_init, const float* const* pad, void* ws,
                  size_t ws_bytes, float* const* A, float* lambda, double* fit_trace,
                  rt_tucker_info* tinfo, rt_ffcp_info* finfo, void* stream) {
  RT_TRY(validate_dense(tdesc, fdesc));
  RT_TRY(check_ptr(ws, "ws"));
  DensePlan p;
  const size_t need = p.plan(tdesc, fdesc, nullptr);
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  p.plan(tdesc, fdesc, ws);
  // every argument of both stages is checked before the first launch: the
  // FFCP stage's pointers here, the Tucker stage's by rt_tucker_rand itself
  // (which enqueues nothing when it rejects an argument)
  RT_TRY(check_ptr(lambda, "lambda"));
  if (!A) {
    set_error("A array must not be NULL");
    return kErrInvalid;
  }
  const int N = fdesc->N, R = fdesc->R;
  for (int n = 0; n < N; ++n) RT_TRY(check_ptr(A[n], "A[n]"));
  const bool coeff = fdesc->init == RT_INIT_COEFF || fdesc->init == RT_INIT_COEFF_GUARDED;
  const bool hosvd = fdesc->init == RT_INIT_HOSVD || fdesc->init == RT_INIT_COEFF_GUARDED;
  if (fdesc->init == RT_INIT_USER || coeff) {
    if (!A_init) {
      set_error("A_init is NULL with RT_INIT_USER / RT_INIT_COEFF");
      return kErrInvalid;
    }
    for (int n = 0; n < N; ++n) RT_TRY(check_ptr(A_init[n], "A_init[n]"));
  }
  if (hosvd) {
    for (int n = 0; n < N; ++n) {
      if (R > fdesc->ranks[n]) {
        if (!pad || !pad[n]) {
          set_error("HOSVD init with R > R_%d needs pad[%d]", n, n);
          return kErrInvalid;
        }
        RT_TRY(check_ptr(pad[n], "pad[n]"));
      }
    }
  }
  if ((finfo && !aligned16(finfo)) || (fit_trace && !aligned16(fit_trace))) {
    set_error("info / fit_trace not 16-byte aligned");
    return kErrInvalid;
  }
  void* Uv[RT_MAX_MODES];
  const float* Uc[RT_MAX_MODES];
  for (int n = 0; n < N; ++n) {
    Uv[n] = p.U[n];
    Uc[n] = p.U[n];
  }
  RT_TRY(rt_tucker_rand(tdesc, Y, Omega, Omega_t, p.tws, p.tbytes, Uv, p.G, Ybf16, tinfo,
                        nullptr, stream));
  return rt_ffcp(fdesc, Uc, p.G, A_init, pad, p.fws, p.fbytes, A, lambda, fit_trace, finfo,
                 stream);
}

int rt_ffcp_noalloc(const rt_ffcp_desc* desc, const float* const* U, const float* G,
                    const float* const* A_init, const float* const* pad, float* const* A,
                    float* lambda, double* fit_trace, rt_ffcp_info* info, void* stream) {
  RT_TRY(validate_ffcp(desc));
  FfcpPlan P;
  const size_t need = P.plan(desc, nullptr);
  if (need > kNoallocScratchBytes) {
    set_error("rt_ffcp_noalloc: this problem needs %zu bytes of scratch, above the "
              "library's static %zu bytes (use rt_ffcp with a workspace)",
              need, kNoallocScratchBytes);
    return kErrUnsupported;
  }
  void* ws = nullptr;
  RT_TRY(noalloc_scratch(&ws));
  return rt_ffcp(desc, U, G, A_init, pad, ws, kNoallocScratchBytes, A, lambda, fit_trace,
                 info, stream);
}

int rt_ttm(int32_t dtype, int64_t A, int64_t I, int64_t C, int32_t K,
           const void* X, const void* M, void* out, void* stream) {
  if (A < 1 || I < 1 || C < 1 || K < 1 || K > RT_MAX_SKETCH) {
    set_error("rt_ttm: bad sizes");
    return kErrInvalid;
  }
  RT_TRY(check_ptr(X, "X"));
  RT_TRY(check_ptr(M, "M"));
  RT_TRY(check_ptr(out, "out"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == RT_F32)
    return launch_ttm<float>(static_cast<const float*>(X),
                             static_cast<const float*>(M),
                             static_cast<float*>(out), A, I, C, K, s);
  if (dtype == RT_F64)
    return launch_ttm<double>(static_cast<const double*>(X),
                              static_cast<const double*>(M),
                              static_cast<double*>(out), A, I, C, K, s);
  set_error("rt_ttm: dtype %d unsupported", dtype);
  return kErrInvalid;
}

int rt_stream_pass(int32_t dtype, int64_t A, int64_t I1, int64_t I2,
                   const void* Y, const void* B2, int32_t K2, const void* B1,
                   int32_t K1, void* TA, void* TB, double* norm_out, void* ws,
                   size_t ws_bytes, void* stream) {
  if (A < 1 || I1 < 1 || I2 < 1 || K2 < 1 || K2 > RT_MAX_SKETCH ||
      (TB && (K1 < 1 || K1 > RT_MAX_SKETCH))) {
    set_error("rt_stream_pass: bad sizes");
    return kErrInvalid;
  }
  RT_TRY(check_ptr(Y, "Y"));
  RT_TRY(check_ptr(B2, "B2"));
  RT_TRY(check_ptr(TA, "TA"));
  RT_TRY(check_ptr(ws, "ws"));
  if (TB) {
    RT_TRY(check_ptr(B1, "B1"));
    RT_TRY(check_ptr(TB, "TB"));
  }
  if (ws_bytes < 8192) {
    set_error("rt_stream_pass: workspace too small");
    return kErrWorkspace;
  }
  rt_tucker_desc d{};
  d.N = 3;
  d.sweeps = 1;
  d.precision = dtype;
  d.dims[0] = A;
  d.dims[1] = I1;
  d.dims[2] = I2;
  Arena ar(ws);
  double* nout = ar.take<double>(1);
  int32_t* flag = ar.take<int32_t>(4);
  void* sws = ar.take<char>(8192 - 512);
  StreamCtx sc = make_stream_ctx(&d, Y, nullptr, sws, 8192 - 512,
                                 norm_out ? norm_out : nout, flag);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == RT_F32) {
    if (TB)
      return stream_dual<float>(sc, 0, static_cast<const float*>(B2), K2,
                                static_cast<const float*>(B1), K1,
                                static_cast<float*>(TA), static_cast<float*>(TB), nullptr,
                                nullptr, s);
    return stream_single<float>(sc, 0, static_cast<const float*>(B2), K2, nullptr, 0,
                                static_cast<float*>(TA), nullptr, nullptr, s);
  }
  if (dtype == RT_F64) {
    if (TB)
      return stream_dual<double>(sc, 0, static_cast<const double*>(B2), K2,
                                 static_cast<const double*>(B1), K1,
                                 static_cast<double*>(TA), static_cast<double*>(TB),
                                 nullptr, nullptr, s);
    return stream_single<double>(sc, 0, static_cast<const double*>(B2), K2, nullptr, 0,
                                 static_cast<double*>(TA), nullptr, nullptr, s);
  }
  set_error("rt_stream_pass: dtype %d unsupported", dtype);
  return kErrInvalid;
}

int rt_cp_fit_workspace(const rt_ffcp_desc* desc, size_t* bytes) {
  if (!desc || !bytes || desc->N < 2 || desc->N > RT_MAX_MODES || desc->R < 1 ||
      desc->R > RT_MAX_SKETCH) {
    set_error("rt_cp_fit_workspace: bad arguments");
    return kErrInvalid;
  }
  int64_t total = 1, rpow = 1;
  for (int n = 0; n < desc->N; ++n) {
    if (desc->dims[n] < 1) {
      set_error("rt_cp_fit_workspace: dims[%d] < 1", n);
      return kErrInvalid;
    }
    total *= desc->dims[n];
    rpow *= desc->R;
    if (rpow > (int64_t(1) << 24)) {
      set_error("rt_cp_fit: R^N too large");
      return kErrUnsupported;
    }
  }
  const int64_t t1 = total / desc->dims[desc->N - 1] * desc->R;
  Arena ar(nullptr);
  ar.take<float>(t1);
  ar.take<float>(t1);
  ar.take<double>(norm2_blocks());
  ar.take<double>(8);
  ar.take<int32_t>(8);
  for (int n = 0; n < desc->N; ++n) ar.take<double>(desc->R * desc->R);
  *bytes = ar.need;
  return kOk;
}

int rt_cp_fit_dense(const rt_ffcp_desc* desc, const float* Y,
                    const float* const* A, const float* lambda, void* ws,
                    size_t ws_bytes, double* out3, void* stream) {
  size_t need = 0;
  RT_TRY(rt_cp_fit_workspace(desc, &need));
  RT_TRY(check_ptr(Y, "Y"));
  RT_TRY(check_ptr(ws, "ws"));
  RT_TRY(check_ptr(out3, "out3"));
  if (!A) {
    set_error("A is NULL");
    return kErrInvalid;
  }
  const int N = desc->N, R = desc->R;
  for (int n = 0; n < N; ++n) RT_TRY(check_ptr(A[n], "A[n]"));
  if (lambda) RT_TRY(check_ptr(lambda, "lambda"));
  if (ws_bytes < need) {
    set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
    return kErrWorkspace;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t total = 1;
  for (int n = 0; n < N; ++n) total *= desc->dims[n];
  const int64_t t1 = total / desc->dims[N - 1] * R;
  Arena ar(ws);
  float* b0 = ar.take<float>(t1);
  float* b1 = ar.take<float>(t1);
  double* partial = ar.take<double>(norm2_blocks());
  double* scal = ar.take<double>(8);
  int32_t* flags = ar.take<int32_t>(8);
  double* grams[RT_MAX_MODES];
  for (int n = 0; n < N; ++n) grams[n] = ar.take<double>(R * R);
  RT_TRY(launch_fill_i32(flags, 0, 8, s));
  RT_TRY(launch_norm2<float>(Y, total, partial, norm2_blocks(), scal + 0,
                             flags, s));
  // Y x_N A_N^T ... x_1 A_1^T  ->  R^N tensor; its diagonal gives <Y, Yhat>
  int64_t D[RT_MAX_MODES];
  for (int n = 0; n < N; ++n) D[n] = desc->dims[n];
  const float* src = Y;
  float* bufs[2] = {b0, b1};
  int cur = 0;
  for (int p = N - 1; p >= 0; --p) {
    int64_t Apre = 1, Cpost = 1;
    for (int q = 0; q < p; ++q) Apre *= D[q];
    for (int q = p + 1; q < N; ++q) Cpost *= D[q];
    RT_TRY(launch_ttm<float>(src, A[p], bufs[cur], Apre, D[p], Cpost, R, s));
    D[p] = R;
    src = bufs[cur];
    cur ^= 1;
  }
  for (int n = 0; n < N; ++n)
    RT_TRY(launch_gram_unfold<float>(A[n], grams[n], desc->dims[n], R, 1, s));
  return launch_cp_fit_final(src, N, R, lambda, grams, scal, out3, s);
}

const char* rt_status_string(int status) {
  switch (status) {
    case RT_OK: return "RT_OK";
    case RT_ERR_INVALID_ARG: return "RT_ERR_INVALID_ARG";
    case RT_ERR_UNSUPPORTED: return "RT_ERR_UNSUPPORTED";
    case RT_ERR_WORKSPACE: return "RT_ERR_WORKSPACE";
    case RT_ERR_NONFINITE: return "RT_ERR_NONFINITE";
    case RT_ERR_NUMERICAL: return "RT_ERR_NUMERICAL";
    case RT_ERR_HIP: return "RT_ERR_HIP";
    case RT_ERR_NO_DEVICE: return "RT_ERR_NO_DEVICE";
    default: return "unknown status";
  }
}

const char* rt_last_error(void) { return g_err; }

const char* rt_version(void) { return "rtucker 0.1 (gfx950)"; }

}  // extern "C"
