// Y-streaming passes of RandTucker2i (see stream.hpp).
//
// Y is viewed as A slabs M_a = Y[a, :, :] of size I1 x I2 (I1 = I_{N-1},
// I2 = I_N, row-major).  One pass over Y computes, for every slab,
//     P_a = M_a B2          (I1 x K2: the mode-N contraction, TA)
//     Q_a = B1^T M_a        (K1 x I2: the mode-(N-1) contraction, TB)
// so a single read of Y feeds every sketch of one Jacobi sweep (Algorithm 3,
// lines 3-6: X_n for n < N is reached from TA, X_N from TB); the core pass
// (Algorithm 3, line 8) computes P only.  These are the blocked products of
// eq. (22) restricted to one GPU: each workgroup owns whole slabs, and the
// partial products over column ranges are summed in a fixed order.
//
// Matrix cores: v_mfma_f32_32x32x2f32 (FP32 path).  A wavefront owns a
// 32-row chunk of a slab and a range of CT 32-column tiles:
//   P tile (32 rows x 32 of K2): A operand = M rows (lane (m, h) holds
//       M[r0+m][c0+16h+4u+e], loaded as float4), B operand = B2 rows held in
//       registers for the wave's whole column range;
//   Q tiles (32 of K1 x 32 cols): A operand = B1 rows of the chunk, B
//       operand = M[r0+2t+h][c0+m] (coalesced 128-byte row segments).
// The K index of each MFMA is a permutation of the contracted index, applied
// identically to both operands.  The same tile is read twice in two layouts;
// the second read hits the caches, so HBM sees one read of Y.
// ||Y||^2 (FP64) and a non-finite check ride along on the P-layout loads,
// which touch every element exactly once.
#include "stream.hpp"

#include "kernels.hpp"

namespace rt {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kMaxCT = 4;  // 32-column tiles per wave (register budget)

struct DualArgs {
  const float* Y;
  int64_t A;
  int I1, I2;
  const float* B2;
  int K2;
  const float* B1;
  int K1;
  float* TA;
  float* TB;
  int wps;          // wavefronts per slab (1, 2, 4 or 8)
  int red_offset;   // float offset of the P-reduction tiles in LDS
  double* norm_partial;  // per workgroup, or null
};

// Raw buffer resource over one slab, used for 32-bit loads: offsets >=
// `bytes` read as zero (hardware range check), which masks rows past the
// slab end; the row step of the Q layout goes in the scalar offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const float* base,
                                                            uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, bytes,
                                           0x00020000);
}

constexpr uint32_t kOob = 0x7ffffff0u;  // any offset past every slab

__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}

// DOQ = true: sweep pass (P and Q; B2 in LDS to leave registers to the Q
// accumulators).  DOQ = false: core pass (P only; B2 in registers).
template <int CT, bool DOQ>
__global__ __launch_bounds__(kThreads) void dual_f32_kernel(DualArgs p) {
  extern __shared__ float lds[];
  float* b2s = lds;                     // B2, I2 x K2 row-major (DOQ only)
  float* red = lds + p.red_offset;      // kWaves partial P tiles (32 x 32)
  __shared__ double nred[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 31, h = lane >> 5;
  const int wps = p.wps, G = kWaves / wps;
  const int g = wave / wps, sub = wave % wps;
  const int I1 = p.I1, I2 = p.I2, K1 = p.K1, K2 = p.K2;
  const int colbase = sub * CT * 32;
  int nct = (I2 - colbase + 31) / 32;
  nct = nct < 0 ? 0 : (nct > CT ? CT : nct);
  // Lanes with m >= K2 produce discarded P columns; clamp their B2 index.
  const int mB = m < K2 ? m : K2 - 1;
  float b2f[DOQ ? 1 : CT][16];
  if constexpr (DOQ) {
    for (int i = threadIdx.x; i < I2 * K2; i += kThreads) b2s[i] = p.B2[i];
    __syncthreads();
  } else {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = colbase + 32 * ct + 16 * h + 4 * (t >> 2) + (t & 3);
        b2f[ct][t] = (c < I2 && m < K2) ? p.B2[static_cast<int64_t>(c) * K2 + m] : 0.f;
      }
    }
  }
  double nacc = 0.0;
  const int64_t slab = static_cast<int64_t>(I1) * I2;
  const uint32_t slab_bytes = static_cast<uint32_t>(slab * 4);

  for (int64_t base = static_cast<int64_t>(blockIdx.x) * G; base < p.A;
       base += static_cast<int64_t>(gridDim.x) * G) {
    const int64_t a = base + g;
    const bool live = a < p.A;
    const __amdgpu_buffer_rsrc_t rs = slab_rsrc(p.Y + (live ? a : 0) * slab,
                                               live ? slab_bytes : 0u);
    v16f accq[DOQ ? CT : 1];
    if constexpr (DOQ) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) accq[ct] = v16f{};
    }
    for (int r0 = 0; r0 < I1; r0 += 32) {
      float b1v[16];
      if constexpr (DOQ) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int row = r0 + 2 * t + h;
          b1v[t] = (row < I1 && m < K1) ? p.B1[static_cast<int64_t>(row) * K1 + m] : 0.f;
        }
      }
      v16f accp = v16f{};
      // P layout: lane (m, h) reads M[r0 + m][c0 + 16h + 4u .. +3] (float4).
      const bool prow_ok = live && (r0 + m) < I1;
      const float* prow_ptr = p.Y + (live ? a : 0) * slab +
                              static_cast<int64_t>(prow_ok ? r0 + m : 0) * I2;
      // Q layout: lane (m, h) reads M[r0 + 2t + h][c0 + m]; the 2t part is a
      // wave-uniform scalar offset.
      const uint32_t qrow_off = static_cast<uint32_t>((r0 + h) * I2) * 4u;
      float4 pv[2][4];
      float qv[16];
      auto load_p = [&](int ct, int buf) {
        const int c0 = colbase + 32 * ct;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int col = c0 + 16 * h + 4 * u;
          pv[buf][u] = (prow_ok && col < I2) ? ld4(prow_ptr + col)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      };
      if (nct > 0) load_p(0, 0);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (ct < nct) {
          const int buf = ct & 1;
          const int c0 = colbase + 32 * ct;
          if (ct + 1 < nct) load_p(ct + 1, buf ^ 1);
          if constexpr (DOQ) {
            const int col = c0 + m;
            const uint32_t off = col < I2 ? qrow_off + 4u * col : kOob;
#pragma unroll
            for (int t = 0; t < 16; ++t)
              qv[t] = __builtin_bit_cast(
                  float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 8 * t * I2, 0));
          }
          float ss = 0.f;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float e4[4] = {pv[buf][u].x, pv[buf][u].y, pv[buf][u].z, pv[buf][u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float bv;
              if constexpr (DOQ) {
                int c = c0 + 16 * h + 4 * u + e;
                c = c < I2 ? c : I2 - 1;  // the matching Y value reads as 0
                bv = b2s[c * K2 + mB];
              } else {
                bv = b2f[ct][4 * u + e];
              }
              accp = __builtin_amdgcn_mfma_f32_32x32x2f32(e4[e], bv, accp, 0, 0, 0);
              ss += e4[e] * e4[e];
            }
          }
          if constexpr (DOQ) {
#pragma unroll
            for (int t = 0; t < 16; ++t)
              accq[ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(b1v[t], qv[t],
                                                              accq[ct], 0, 0, 0);
          }
          nacc += static_cast<double>(ss);
        }
      }
      // P: lane holds P[8(v/4) + 4h + v%4][m]
      if (wps == 1) {
        if (live) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int row = r0 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (row < I1 && m < K2)
              p.TA[(a * I1 + row) * K2 + m] = accp[v];
          }
        }
      } else {
        float* mine = red + wave * 1024;
#pragma unroll
        for (int v = 0; v < 16; ++v)
          mine[(8 * (v >> 2) + 4 * h + (v & 3)) * 32 + m] = accp[v];
        __syncthreads();
        const int rows_per = 32 / wps;
        for (int idx = lane; idx < rows_per * 32; idx += 64) {
          const int rl = sub * rows_per + idx / 32, n = idx % 32;
          float s = 0.f;
          for (int w = 0; w < wps; ++w) s += red[(g * wps + w) * 1024 + rl * 32 + n];
          const int row = r0 + rl;
          if (live && row < I1 && n < K2) p.TA[(a * I1 + row) * K2 + n] = s;
        }
        __syncthreads();
      }
    }
    if constexpr (DOQ) {
      if (live) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          if (ct < nct) {
            const int col = colbase + 32 * ct + m;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int j = 8 * (v >> 2) + 4 * h + (v & 3);
              if (j < K1 && col < I2) p.TB[(a * K1 + j) * I2 + col] = accq[ct][v];
            }
          }
        }
      }
    }
  }
  if (p.norm_partial) {
    double s = wave_sum(nacc);
    if (lane == 0) nred[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t += nred[w];
      p.norm_partial[blockIdx.x] = t;
    }
  }
}

constexpr size_t kLdsLimit = 160 * 1024;

size_t dual_lds_bytes(int I2, int K2, bool doQ) {
  const size_t b2 = doQ ? (static_cast<size_t>(I2) * K2 + 63) / 64 * 64 : 0;
  return (b2 + kWaves * 1024) * sizeof(float);
}

template <int CT, bool DOQ>
int launch_dual(const DualArgs& a, int grid, size_t lds, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(dual_f32_kernel<CT, DOQ>),
        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsLimit - 1024));
    if (e != hipSuccess) return hip_fail(e, "dual_f32 LDS attribute");
    attr_set = true;
  }
  hipLaunchKernelGGL((dual_f32_kernel<CT, DOQ>), dim3(grid), dim3(kThreads), lds,
                     s, a);
  return kOk;
}

template <bool DOQ>
int launch_dual_ct(int ct, const DualArgs& a, int grid, size_t lds, hipStream_t s) {
  switch (ct) {
    case 1: return launch_dual<1, DOQ>(a, grid, lds, s);
    case 2: return launch_dual<2, DOQ>(a, grid, lds, s);
    case 3: return launch_dual<3, DOQ>(a, grid, lds, s);
    default: return launch_dual<4, DOQ>(a, grid, lds, s);
  }
}

// Choose (waves per slab, tiles per wave) for a slab width; false if the
// MFMA kernel does not apply.
bool plan_dual(int I2, int K1, int K2, int* wps, int* ct) {
  if (K1 > 32 || K2 > 32 || K2 < 1 || (I2 & 3) != 0) return false;
  if (dual_lds_bytes(I2, K2, true) + 1024 > kLdsLimit) return false;
  const int tiles = (I2 + 31) / 32;
  for (int w = 1; w <= kWaves; w *= 2) {
    const int c = (tiles + w - 1) / w;
    if (c <= kMaxCT) {
      *wps = w;
      *ct = c;
      return true;
    }
  }
  return false;
}

int grid_for(int64_t A, int wps) {
  const int64_t groups = (A + (kWaves / wps) - 1) / (kWaves / wps);
  const int64_t cap = 1024;  // grid-stride beyond this many workgroups
  return static_cast<int>(groups < cap ? groups : cap);
}

int run_dual_f32(const StreamCtx& c, const float* Y, const float* B2, int K2,
                 const float* B1, int K1, float* TA, float* TB, bool doQ,
                 bool doNorm, hipStream_t s, bool* used) {
  int wps = 0, ct = 0;
  *used = false;
  if (!plan_dual(static_cast<int>(c.I2), K1, K2, &wps, &ct) || c.I1 > (1 << 30) ||
      c.I2 > (1 << 30))
    return kOk;
  DualArgs a{};
  a.Y = Y;
  a.A = c.A;
  a.I1 = static_cast<int>(c.I1);
  a.I2 = static_cast<int>(c.I2);
  a.B2 = B2;
  a.K2 = K2;
  a.B1 = B1;
  a.K1 = doQ ? K1 : 0;
  a.TA = TA;
  a.TB = TB;
  a.wps = wps;
  const int grid = grid_for(c.A, wps);
  a.norm_partial = doNorm ? c.norm_partial : nullptr;
  const size_t lds = dual_lds_bytes(a.I2, K2, doQ);
  a.red_offset = doQ ? static_cast<int>((static_cast<size_t>(a.I2) * K2 + 63) / 64 * 64) : 0;
  const int rc0 = doQ ? launch_dual_ct<true>(ct, a, grid, lds, s)
                      : launch_dual_ct<false>(ct, a, grid, lds, s);
  if (rc0 != kOk) return rc0;
  RT_LAUNCH_CHECK("dual_f32");
  if (doNorm) {
    int rc = launch_sum_partials(c.norm_partial, grid, c.norm_out, c.nonfinite, s);
    if (rc != kOk) return rc;
  }
  *used = true;
  return kOk;
}

}  // namespace

size_t stream_workspace_bytes(const rt_tucker_desc*) {
  return 1024 * sizeof(double) + 256;
}

StreamCtx make_stream_ctx(const rt_tucker_desc* d, const void* y,
                          uint16_t* ybf16, void* ws, size_t ws_bytes,
                          double* norm_out, int32_t* nonfinite) {
  StreamCtx c{};
  c.y = y;
  c.precision = d->precision;
  c.bf16_input = (d->flags & RT_FLAG_BF16_INPUT) != 0;
  c.ybf16 = c.bf16_input ? const_cast<uint16_t*>(static_cast<const uint16_t*>(y))
                         : ybf16;
  const int N = d->N;
  c.A = 1;
  for (int p = 0; p < N - 2; ++p) c.A *= d->dims[p];
  c.I1 = d->dims[N - 2];
  c.I2 = d->dims[N - 1];
  c.ws = ws;
  c.ws_bytes = ws_bytes;
  c.norm_partial = static_cast<double*>(ws);
  c.norm_out = norm_out;
  c.nonfinite = nonfinite;
  return c;
}

template <typename T>
int stream_dual(const StreamCtx& c, int sweep, const T* B2, int K2, const T* B1,
                int K1, T* TA, T* TB, hipStream_t s) {
  if (c.precision == RT_BF16_MIXED) {
    set_error("BF16 mixed precision is not available in this build");
    return kErrUnsupported;
  }
  const T* Y = static_cast<const T*>(c.y);
  const bool doNorm = sweep == 0;
  if constexpr (sizeof(T) == sizeof(float)) {
    bool used = false;
    int rc = run_dual_f32(c, Y, B2, K2, B1, K1, TA, TB, true, doNorm, s, &used);
    if (rc != kOk || used) return rc;
  }
  // generic path: two vector-ALU passes and a separate norm pass
  if (doNorm) {
    int rc = launch_norm2<T>(Y, c.A * c.I1 * c.I2, c.norm_partial, norm2_blocks(),
                             c.norm_out, c.nonfinite, s);
    if (rc != kOk) return rc;
  }
  int rc = launch_ttm<T>(Y, B2, TA, c.A * c.I1, c.I2, 1, K2, s);
  if (rc != kOk) return rc;
  return launch_ttm<T>(Y, B1, TB, c.A, c.I1, c.I2, K1, s);
}

template <typename T>
int stream_single(const StreamCtx& c, int, const T* B2, int K2, T* TA,
                  hipStream_t s) {
  if (c.precision == RT_BF16_MIXED) {
    set_error("BF16 mixed precision is not available in this build");
    return kErrUnsupported;
  }
  const T* Y = static_cast<const T*>(c.y);
  if constexpr (sizeof(T) == sizeof(float)) {
    bool used = false;
    int rc = run_dual_f32(c, Y, B2, K2, nullptr, 0, TA, nullptr, false, false, s,
                          &used);
    if (rc != kOk || used) return rc;
  }
  return launch_ttm<T>(Y, B2, TA, c.A * c.I1, c.I2, 1, K2, s);
}

template int stream_dual<float>(const StreamCtx&, int, const float*, int,
                                const float*, int, float*, float*, hipStream_t);
template int stream_dual<double>(const StreamCtx&, int, const double*, int,
                                 const double*, int, double*, double*,
                                 hipStream_t);
template int stream_single<float>(const StreamCtx&, int, const float*, int,
                                  float*, hipStream_t);
template int stream_single<double>(const StreamCtx&, int, const double*, int,
                                   double*, hipStream_t);

}  // namespace rt
