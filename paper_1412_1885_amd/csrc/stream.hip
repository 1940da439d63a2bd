// Y-streaming passes of RandTucker2i (see stream.hpp).
//
// Y is viewed as A slabs M_a = Y[a, :, :] of size I1 x I2 (I1 = I_{N-1},
// I2 = I_N, row-major).  One pass over Y computes, for every slab,
//     P_a = M_a B2          (I1 x K2: the mode-N contraction, TA)
//     Q_a = B1^T M_a        (K1 x I2: the mode-(N-1) contraction, TB)
// so a single read of Y feeds every sketch of one Jacobi sweep of
// Algorithm 3 (X_n for n < N is reached from TA, X_N from TB); the core pass
// (the core projection of Algorithm 3) computes P only.  These are the blocked products of
// eq. (22) restricted to one GPU: each workgroup owns whole slabs, and the
// partial products over column ranges are summed in a fixed order.
//
// Data path.  A wavefront owns a range of CT 32-column tiles of a slab and
// walks the slab in 32-row chunks.  Each 32 x 32 FP32 tile is read from HBM
// once with fully coalesced float4 loads (8 rows x 128 bytes per
// instruction, prefetched one tile ahead across chunks), written to a
// wave-private LDS tile whose 16-byte chunks are XOR-swizzled by row, and
// read back in the two operand layouts of v_mfma_f32_32x32x2f32:
//   P (32 rows x 32 of K2): A operand M[r0+m][c0+16h+4u+e] (b128 reads),
//       B operand B2[c0+16h+4u+e][m] (registers, or LDS in the sweep pass);
//   Q (32 of K1 x 32 cols): A operand B1[r0+2t+h][m], B operand
//       M[r0+2t+h][c0+m] (b32 reads).
// The K index of each MFMA is a permutation of the contracted index applied
// identically to both operands.  ||Y||^2 (FP64) and a non-finite check ride
// along on the staged values, which cover every element exactly once.
// TA and TB are written with non-temporal stores: they are read once, by
// a later kernel, and normal stores of them slowed the read stream.
#include "stream.hpp"

#include "kernels.hpp"
#include "profile.hpp"

namespace rt {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kMaxCT = 4;     // 32-column tiles per wave (register budget)
constexpr int kTile = 1024;   // floats per staged 32 x 32 tile

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
  int stage_offset; // float offset of the per-wave tiles in dynamic LDS
  double* norm_partial;  // per workgroup, or null
};

__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}

// Position of logical (row, 16-byte chunk) in a staged tile.
__device__ __forceinline__ int swz(int row, int chunk) {
  return row * 32 + 4 * (chunk ^ (row & 7));
}

// DOQ = true: sweep pass (P and Q; B2 in LDS to leave registers to the Q
// accumulators).  DOQ = false: core pass (P only; B2 in registers).
template <int CT, bool DOQ>
__global__ __launch_bounds__(kThreads) void dual_f32_kernel(DualArgs p) {
  extern __shared__ float lds[];
  float* b2s = lds;                                    // I2 x K2 (DOQ only)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* tile = lds + p.stage_offset + wave * kTile;   // this wave's tile
  float* stage = lds + p.stage_offset;                 // all tiles (reduction)
  __shared__ double nred[kWaves];
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
  // coalesced load mapping: lane -> (row 8u + lrow, 16-byte chunk lchunk)
  const int lrow = lane >> 3, lchunk = lane & 7;

  for (int64_t base = static_cast<int64_t>(blockIdx.x) * G; base < p.A;
       base += static_cast<int64_t>(gridDim.x) * G) {
    const int64_t a = base + g;
    const bool live = a < p.A;
    const float* Ysl = p.Y + (live ? a : 0) * slab;
    v16f accq[DOQ ? CT : 1];
    if constexpr (DOQ) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) accq[ct] = v16f{};
    }
    float4 gcur[4], gnext[4];
    auto load_tile = [&](int rr, int ct, float4(&dst)[4]) {
      const int col = colbase + 32 * ct + 4 * lchunk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = rr + 8 * u + lrow;
        dst[u] = (live && row < I1 && col < I2)
                     ? ld4(Ysl + static_cast<int64_t>(row) * I2 + col)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    if (nct > 0) load_tile(0, 0, gcur);
    for (int r0 = 0; r0 < I1; r0 += 32) {
      const int rn = r0 + 32;
      float b1v[16];
      if constexpr (DOQ) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int row = r0 + 2 * t + h;
          b1v[t] = (row < I1 && m < K1) ? p.B1[static_cast<int64_t>(row) * K1 + m] : 0.f;
        }
      }
      v16f accp = v16f{};
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (ct < nct) {
          const int c0 = colbase + 32 * ct;
          if (ct + 1 < nct) load_tile(r0, ct + 1, gnext);
          else if (rn < I1) load_tile(rn, 0, gnext);
          // stage the tile (wave-private; LDS accesses of a wave are ordered)
          // squares in FP64: FLT_MAX^2 is finite there, so only a NaN or
          // Inf in Y makes ||Y||^2 non-finite
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            *reinterpret_cast<float4*>(tile + swz(8 * u + lrow, lchunk)) = gcur[u];
            const double x = gcur[u].x, y = gcur[u].y, z = gcur[u].z, w = gcur[u].w;
            nacc += (x * x + y * y) + (z * z + w * w);
          }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float4 v = *reinterpret_cast<const float4*>(tile + swz(m, 4 * h + u));
            const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float bv;
              if constexpr (DOQ) {
                int c = c0 + 16 * h + 4 * u + e;
                c = c < I2 ? c : I2 - 1;  // the matching Y value is 0
                bv = b2s[c * K2 + mB];
              } else {
                bv = b2f[ct][4 * u + e];
              }
              accp = __builtin_amdgcn_mfma_f32_32x32x2f32(e4[e], bv, accp, 0, 0, 0);
            }
          }
          if constexpr (DOQ) {
#pragma unroll
            for (int t = 0; t < 16; ++t) {
              const int row = 2 * t + h;
              const float qv = tile[swz(row, m >> 2) + (m & 3)];
              accq[ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(b1v[t], qv, accq[ct],
                                                              0, 0, 0);
            }
          }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int u = 0; u < 4; ++u) gcur[u] = gnext[u];
        }
      }
      // P: lane holds P[8(v/4) + 4h + v%4][m]
      if (wps == 1) {
        if (live) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int row = r0 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (row < I1 && m < K2)
              __builtin_nontemporal_store(accp[v], p.TA + (a * I1 + row) * K2 + m);
          }
        }
      } else {
        // the staged tiles are consumed: reuse them for the reduction
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v)
          tile[(8 * (v >> 2) + 4 * h + (v & 3)) * 32 + m] = accp[v];
        __syncthreads();
        const int rows_per = 32 / wps;
        for (int idx = lane; idx < rows_per * 32; idx += 64) {
          const int rl = sub * rows_per + idx / 32, n = idx % 32;
          float s = 0.f;
          for (int w = 0; w < wps; ++w) s += stage[(g * wps + w) * kTile + rl * 32 + n];
          const int row = r0 + rl;
          if (live && row < I1 && n < K2)
            __builtin_nontemporal_store(s, p.TA + (a * I1 + row) * K2 + n);
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
              if (j < K1 && col < I2)
                __builtin_nontemporal_store(accq[ct][v], p.TB + (a * K1 + j) * I2 + col);
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

size_t b2_floats(int I2, int K2, bool doQ) {
  return doQ ? (static_cast<size_t>(I2) * K2 + 63) / 64 * 64 : 0;
}

size_t dual_lds_bytes(int I2, int K2, bool doQ) {
  return (b2_floats(I2, K2, doQ) + kWaves * kTile) * sizeof(float);
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
bool plan_dual(int I2, int K1, int K2, bool doQ, int* wps, int* ct) {
  if (K1 > 32 || K2 > 32 || K2 < 1 || (I2 & 3) != 0) return false;
  if (dual_lds_bytes(I2, K2, doQ) + 1024 > kLdsLimit) return false;
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
                 bool doNorm, int stage, hipStream_t s, bool* used) {
  int wps = 0, ct = 0;
  *used = false;
  if (!plan_dual(static_cast<int>(c.I2), doQ ? K1 : 0, K2, doQ, &wps, &ct) ||
      c.I1 > (1 << 30) || c.I2 > (1 << 30))
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
  a.stage_offset = static_cast<int>(b2_floats(a.I2, K2, doQ));
  const size_t lds = dual_lds_bytes(a.I2, K2, doQ);
  int rc0;
  {
    ProfScope ps(stage, s);
    rc0 = doQ ? launch_dual_ct<true>(ct, a, grid, lds, s)
              : launch_dual_ct<false>(ct, a, grid, lds, s);
  }
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

size_t stream_workspace_bytes(const rt_tucker_desc* d) {
  size_t b = 1024 * sizeof(double) + 256;
  if (d->precision == RT_BF16_MIXED) {
    int64_t A = 1;
    for (int p = 0; p < d->N - 2; ++p) A *= d->dims[p];
    b += bf16_stream_workspace_bytes(A, d->dims[d->N - 2], d->dims[d->N - 1]);
  }
  return b;
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
  c.ldy = c.bf16_input ? c.I2 : bf16_copy_ld(c.I2);
  c.ws = ws;
  c.ws_bytes = ws_bytes;
  c.norm_partial = static_cast<double*>(ws);
  c.norm_out = norm_out;
  c.nonfinite = nonfinite;
  return c;
}

template <typename T>
int stream_dual(const StreamCtx& c, int sweep, const T* B2, int K2, const T* B1,
                int K1, T* TA, T* TB, T* C, bool* c_done, hipStream_t s) {
  if (c_done) *c_done = false;
  if (c.precision == RT_BF16_MIXED) {
    if constexpr (sizeof(T) == sizeof(float))
      return bf16_stream_pass(c, sweep == 0, B2, K2, B1, K1, TA, TB, C, c_done,
                              sweep == 0 ? kStageFirstPass : kStageSweepPass, s);
    set_error("BF16 mixed precision computes in FP32");
    return kErrUnsupported;
  }
  const T* Y = static_cast<const T*>(c.y);
  const bool doNorm = sweep == 0;
  if constexpr (sizeof(T) == sizeof(float)) {
    bool used = false;
    int rc = run_dual_f32(c, Y, B2, K2, B1, K1, TA, TB, true, doNorm,
                          sweep == 0 ? kStageFirstPass : kStageSweepPass, s, &used);
    if (rc != kOk || used) return rc;
  }
  // generic path: two vector-ALU passes and a separate norm pass
  if (doNorm) {
    int rc = launch_norm2<T>(Y, c.A * c.I1 * c.I2, c.norm_partial, norm2_blocks(),
                             c.norm_out, c.nonfinite, s);
    if (rc != kOk) return rc;
  }
  ProfScope ps(sweep == 0 ? kStageFirstPass : kStageSweepPass, s);
  int rc = launch_ttm<T>(Y, B2, TA, c.A * c.I1, c.I2, 1, K2, s);
  if (rc != kOk) return rc;
  return launch_ttm<T>(Y, B1, TB, c.A, c.I1, c.I2, K1, s);
}

template <typename T>
int stream_single(const StreamCtx& c, int sweep, const T* B2, int K2, const T* B1, int K1,
                  T* TA, T* C, bool* c_done, hipStream_t s) {
  if (c_done) *c_done = false;
  if (c.precision == RT_BF16_MIXED) {
    if constexpr (sizeof(T) == sizeof(float))
      return bf16_stream_pass(c, sweep == 0, B2, K2, C ? B1 : nullptr, C ? K1 : 0, TA,
                              nullptr, C, c_done, kStageCorePass, s);
    set_error("BF16 mixed precision computes in FP32");
    return kErrUnsupported;
  }
  const T* Y = static_cast<const T*>(c.y);
  const bool doNorm = sweep == 0;
  if constexpr (sizeof(T) == sizeof(float)) {
    bool used = false;
    int rc = run_dual_f32(c, Y, B2, K2, nullptr, 0, TA, nullptr, false, doNorm,
                          kStageCorePass, s, &used);
    if (rc != kOk || used) return rc;
  }
  if (doNorm) {
    int rc = launch_norm2<T>(Y, c.A * c.I1 * c.I2, c.norm_partial, norm2_blocks(),
                             c.norm_out, c.nonfinite, s);
    if (rc != kOk) return rc;
  }
  ProfScope ps(kStageCorePass, s);
  return launch_ttm<T>(Y, B2, TA, c.A * c.I1, c.I2, 1, K2, s);
}

template int stream_dual<float>(const StreamCtx&, int, const float*, int, const float*, int,
                                float*, float*, float*, bool*, hipStream_t);
template int stream_dual<double>(const StreamCtx&, int, const double*, int, const double*,
                                 int, double*, double*, double*, bool*, hipStream_t);
template int stream_single<float>(const StreamCtx&, int, const float*, int, const float*, int,
                                  float*, float*, bool*, hipStream_t);
template int stream_single<double>(const StreamCtx&, int, const double*, int, const double*,
                                   int, double*, double*, bool*, hipStream_t);

}  // namespace rt
