// BF16 precision form of the Y-streaming passes (RT_BF16_MIXED).
//
// The sketches and the core projection of Algorithm 3 contract Y against
// thin factor matrices (the blocked products of eq. (22)).  In this form
// the tensor is stored once in BF16 and every pass after the
// first reads 2 bytes per element; the products run on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation, so at R~ <= 32 a pass is
// bound by HBM bandwidth, not by the matrix cores.
//
// Scaling.  Each slab a of the streaming view [A, I1, I2] carries a power of
// two 2^e_a; the stored value is bf16_rne(Y * 2^-e_a) and every product of
// the slab is multiplied by 2^e_a.  A power-of-two scale is exact, so it
// changes nothing while every value and product of the slab stays in the
// normal FP32 range: e_a = 0 unless the binary exponent of max|Y[a]| lies
// outside [-kScaleWindow, kScaleWindow], and then e_a is that exponent (the
// slab's largest entries land in [1, 2), its small ones out of the BF16
// subnormal range, its products and FP32 sums away from overflow).
//
// Passes.  The first pass of a call (FP32 input) reads Y once: a conversion
// kernel of many small workgroups (its HBM write stream overlaps its read
// stream only with that many requests in flight) writes the copy at scale
// 2^0 and per-block partials of max|Y| and ||Y||^2; a per-slab reduction
// sets e_a, and the rare slabs with e_a != 0 are converted again, scaled.
// Every contraction, of every sweep and of the core pass, reads the copy.
//
// Layout of the copy.  Rows of I2 values are stored at a stride rounded up
// to 64 values (128 bytes, one L2 line), the padding written as zeros, so
// every 64-column tile row is exactly one line.  With rows packed at 2*I2
// bytes (I2 = 1000: 2000 B) a tile row straddles two lines, each line is
// shared by two column tiles that a workgroup reads far apart in time, and
// the second read of the line misses L2: the contractions then fetched
// 1.3-1.9x the bytes of the copy.  A caller's own BF16 tensor
// (RT_FLAG_BF16_INPUT) is read with its packed stride.
//
// Data path (one workgroup of 8 wavefronts per slab).  Wave w owns the
// 32-row blocks w, w+8, w+16, w+24 (I1 <= 1024) and walks the slab in
// 64-column tiles, column tile by column tile (RBW steps per column tile:
// the number of row blocks a wave owns, rounded up to 1, 2 or 4).  Lane l
// loads, for each 16-column chunk q of the tile, the 8 values
// Y[r0 + l%32][c0 + 16q + 8(l/32) .. +7] (16 bytes of BF16): exactly the A
// operand of the 32x32x16 MFMA for TA = M B2 (K = columns).  For TB = B1^T M
// (K = rows) the B operand needs 8 consecutive rows of one column, so the
// wave also writes its tile transposed into a private LDS tile and reads it
// back with 16-byte loads.  TA accumulates in registers across the column
// tiles; TB's partial sums over each wave's rows are reduced across the 8
// waves in LDS, in a fixed order, once per column tile.
//
// Latency.  The vector-memory counter completes in issue order, so a wait
// for any load also waits for every load issued before it.  Tiles are
// loaded several steps ahead into a statically indexed ring of registers
// (three tiles ahead), B1^T sits in LDS for the whole
// slab and B2^T of the next column tile is loaded one column tile ahead,
// before that step's tile, so no wait inside the loop stalls on a tile
// that is not yet needed.  A workgroup holds about 246 VGPRs per lane and
// 130 KB of LDS, so a CU runs one (8 wavefronts): the tiles in flight,
// not the access pattern, bound a pass (3.7-4.2 TB/s at 1000^3).
#include <cfloat>
#include <utility>

#include "stream.hpp"

#include "kernels.hpp"
#include "profile.hpp"

namespace rt {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kBW = 8;                 // wavefronts per workgroup
constexpr int kBThreads = kBW * 64;
constexpr int kRBMax = 4;              // 32-row blocks per wave
constexpr int kCT = 64;                // columns per tile
constexpr int kYtStride = 40;          // halfwords per row of the transposed tile
constexpr int kMaxI1 = 32 * kBW * kRBMax;
constexpr int kWaveLds = 32 * kCT * 4; // per-wave LDS: transposed tile, then TB partial
constexpr int kB1Pad = 8;              // halfwords of padding per B1^T row in LDS
// Steps per loop trip: a multiple of the ring size and of two column tiles.
// The compiler's wait counts at the loop head are conservative (the first
// step of a trip waits for every tile in flight), so a longer trip pays
// that drain less often: 16 steps took the core pass from 0.50 to 0.47 ms.
constexpr int kUnroll = 16;
static_assert(kCT * kYtStride * 2 <= kWaveLds, "transposed tile fits the wave's region");
static_assert(2 * 32 * 32 * 4 <= kWaveLds, "two TA row blocks fit the wave's region");

struct BfArgs {
  const uint16_t* Y;      // BF16 bit patterns (the scaled copy or the caller's)
  const int32_t* exps;    // per-slab exponent
  int64_t A;
  int I1, I2;
  int ldy;                // row stride of Y in values (>= I2, multiple of 4)
  const uint16_t* B2t;    // [32][ldb2] BF16, zero beyond (K2, I2)
  int ldb2, K2;
  const uint16_t* B1t;    // [32][ldb1] BF16, zero beyond (K1, I1)
  int ldb1, K1;
  float* TA;              // [A, I1, K2]
  float* TB;              // [A, K1, I2]
};

__device__ __forceinline__ v8bf as_v8bf(uint4 u) { return __builtin_bit_cast(v8bf, u); }

__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  return static_cast<uint32_t>(f32_to_bf16_rne(lo)) |
         (static_cast<uint32_t>(f32_to_bf16_rne(hi)) << 16);
}

// The same two roundings with gfx950's packed conversion instruction
// (round to nearest even; equal to pack2 for every non-NaN input, checked
// on the device against it)
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2_hw(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{lo, hi}, v2bf));
}

// Operands of one 32 x 64 tile for one lane: 4 chunks of 8 BF16 values.
struct Tile {
  uint4 v[4];
};

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

constexpr int kOob = 0x7ffffff0;       // offset past every slab: loads return zero
constexpr int kCopyAlign = 64;         // row stride multiple of the BF16 copy (128 B)
constexpr int kScaleWindow = 100;      // |exponent of max|Y[a]|| up to which e_a = 0

// Buffer descriptor over one slab (byte range); loads past it return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0,
                                           static_cast<int>(bytes), 0x00020000);
}

// Loads the lane's part of the 32 x 64 tile at rows rb*32.. and columns
// c0..: buffer loads with a 32-bit offset into the slab; masked lanes (rows
// or columns past the slab, including whole tiles past the end) get an
// offset past the slab, so the hardware returns zeros without branches.
// HALF (row stride ldy % 8 == 4): rows start 8-byte aligned, two 8-byte
// loads per chunk, the second absent in the half chunk at a row's end.
template <bool HALF>
__device__ __forceinline__ void load_tile(__amdgpu_buffer_rsrc_t rs, const BfArgs& a,
                                          int rb, int lr, int c0, int g, Tile& t) {
  const int r = rb * 32 + lr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + 16 * q + 8 * g;
    const bool ok = r < a.I1 && c < a.I2;   // I2 % 4 == 0
    const bool full = ok && c + 8 <= a.I2;  // else only 4 of the 8 columns exist
    // (r * ldy + c) * 2 < slab bytes < 2^31 whenever ok; clamped otherwise
    const int off = ok ? ((ok ? r : 0) * a.ldy + (ok ? c : 0)) * 2 : kOob;
    if constexpr (!HALF) {
      const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      t.v[q] = make_uint4(v.x, v.y, v.z, v.w);
    } else {
      const v2u lo = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
      const v2u hi = __builtin_amdgcn_raw_buffer_load_b64(rs, full ? off + 8 : kOob, 0, 0);
      t.v[q] = make_uint4(lo.x, lo.y, hi.x, hi.y);
    }
  }
}

// f(std::integral_constant<int, u>) for u = 0 .. N-1, unrolled at compile time.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// B2^T operand of column tile ct for this lane (row lr of B2^T).
__device__ __forceinline__ void load_b2t(const uint16_t* B2t, int ldb2, int ct, int lr, int g,
                                         v8bf* b2) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    b2[q] = as_v8bf(*reinterpret_cast<const uint4*>(
        B2t + static_cast<int64_t>(lr) * ldb2 + ct * kCT + 16 * q + 8 * g));
}
__device__ __forceinline__ void load_b2(const BfArgs& a, int ct, int lr, int g, v8bf* b2) {
  load_b2t(a.B2t, a.ldb2, ct, lr, g, b2);
}

// RBW: steps per column tile (the row blocks a wave owns, rounded up to 1, 2
// or 4); with it every register array below is indexed statically.
template <bool DOQ, bool HALF, int RBW>
__global__ __launch_bounds__(kBThreads) void bf16_stream_kernel(BfArgs a) {
  extern __shared__ __align__(16) char smem[];
  constexpr int kSlots = 4;   // tiles in registers: the current one + three in flight
  static_assert((RBW == 1 || RBW == 2 || RBW == 4) && RBW <= kRBMax, "row blocks");
  static_assert(kUnroll % kSlots == 0 && kUnroll % (2 * RBW) == 0, "static indexing");
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int lr = lane & 31, g = lane >> 5;
  uint16_t* yt = reinterpret_cast<uint16_t*>(smem + w * kWaveLds);
  float* red = reinterpret_cast<float*>(smem);   // [kBW][32][kCT]: wave w's region
  uint16_t* b1s = reinterpret_cast<uint16_t*>(smem + kBW * kWaveLds);
  const int ldb1s = a.ldb1 + kB1Pad;
  const int nrb = (a.I1 + 31) / 32;
  const int nct = (a.I2 + kCT - 1) / kCT;
  // whole loop trips (kUnroll steps = 8 / RBW column tiles): the steps past
  // the last column tile read masked (zero) tiles, so the loop body has no
  // branches and every wait counts loads exactly
  const int nsteps = (nct * RBW + kUnroll - 1) / kUnroll * kUnroll;
  const int64_t slab_elems = static_cast<int64_t>(a.I1) * a.ldy;

  // one slab per workgroup: no outer loop, so nothing slab-invariant is kept
  // live across slabs
  const int64_t slab = blockIdx.x;
  const int e = a.exps[slab];
  const float up = ldexpf(1.0f, e);
  const int64_t base = slab * slab_elems;
  const __amdgpu_buffer_rsrc_t rs = slab_rsrc(a.Y + base, slab_elems * 2);

  // Prologue, in the order the loop's steady state has its loads in
  // flight: B2^T of the current column tile older than the tiles of the
  // ring.  The compiler's wait counts at the loop head hold for both the
  // entry and the back edge; with B2^T issued after the ring here, the
  // first step of every loop trip waited for all tiles in flight.
  if constexpr (DOQ) {
    // B1^T for the whole slab, rows padded against bank conflicts (its
    // loads complete here, before anything else is in flight)
    const int rowc = a.ldb1 / 8;
    for (int l = threadIdx.x; l < 32 * rowc; l += kBThreads) {
      const int k = l / rowc, cc = l - k * rowc;
      *reinterpret_cast<uint4*>(b1s + k * ldb1s + 8 * cc) =
          *reinterpret_cast<const uint4*>(a.B1t + static_cast<int64_t>(k) * a.ldb1 + 8 * cc);
    }
  }
  // B2^T of column tile ct in b2[ct % 2], loaded one column tile ahead
  v8bf b2[2][4];
  load_b2(a, 0, lr, g, b2[0]);
  __builtin_amdgcn_sched_barrier(0);   // issued before the ring's tiles
  // step s: column tile s / RBW, row block w + kBW (s % RBW)
  Tile ring[kSlots];
#pragma unroll
  for (int k = 0; k + 1 < kSlots; ++k)
    load_tile<HALF>(rs, a, w + kBW * (k % RBW), lr, (k / RBW) * kCT, g, ring[k]);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (DOQ) __syncthreads();   // B1^T visible to every wave

  v16f accA[RBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) accA[i][v] = 0.0f;
  v16f accB[2];

  for (int s0 = 0; s0 < nsteps; s0 += kUnroll) {
    static_for<kUnroll>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int s = s0 + u;
      {
        const int ct = s / RBW;
        constexpr int i = u % RBW;           // s0 is a multiple of 2 RBW
        constexpr int cb = (u / RBW) % 2;   // ct % 2
        const int rb = w + kBW * i;
        const int c0 = ct * kCT;
        if constexpr (i == 0) {
          // the next column tile's B2^T, issued before this step's tile
          load_b2(a, ct + 1 < nct ? ct + 1 : nct - 1, lr, g, b2[cb ^ 1]);
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 16; ++v) accB[h][v] = 0.0f;
        }
        {
          const int sp = s + kSlots - 1;   // past the end: masked, no traffic
          load_tile<HALF>(rs, a, w + kBW * (sp % RBW), lr, (sp / RBW) * kCT, g,
                          ring[(u + kSlots - 1) % kSlots]);
        }
        __builtin_amdgcn_sched_barrier(0);   // this step's loads are issued first
        const Tile& cur = ring[u % kSlots];
        // chunk by chunk: TA product, then the transposed copy
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint4 yv = cur.v[q];
          accA[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(yv), b2[cb][q],
                                                            accA[i], 0, 0, 0);
          if constexpr (DOQ) {
            // transposed copy: yt[col][row]
            const uint32_t wds[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const uint16_t hv = static_cast<uint16_t>(wds[j >> 1] >> (16 * (j & 1)));
              yt[(16 * q + 8 * g + j) * kYtStride + lr] = hv;
            }
          }
        }
        if constexpr (DOQ) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // rows past the slab hold zeros; their B1^T columns are read clamped
          const int rbc = rb < nrb ? rb : nrb - 1;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const v8bf b1 = as_v8bf(*reinterpret_cast<const uint4*>(
                b1s + lr * ldb1s + rbc * 32 + 16 * h + 8 * g));
#pragma unroll
            for (int sh = 0; sh < 2; ++sh) {
              const v8bf yc = as_v8bf(*reinterpret_cast<const uint4*>(
                  yt + (32 * sh + lr) * kYtStride + 16 * h + 8 * g));
              accB[sh] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, yc, accB[sh], 0, 0,
                                                                 0);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

          if constexpr (i == RBW - 1) {
            // TB partial of this wave (32 x 64) -> its own LDS region (the
            // transposed tile is no longer needed); fixed-order sum over waves
#pragma unroll
            for (int sh = 0; sh < 2; ++sh)
#pragma unroll
              for (int v = 0; v < 16; ++v) {
                const int m = 8 * (v / 4) + 4 * g + (v % 4);
                red[(w * 32 + m) * kCT + 32 * sh + lr] = accB[sh][v];
              }
            __syncthreads();
            // four consecutive columns per thread (I2 % 4 == 0, so a
            // group is wholly inside or outside the slab), non-temporal
            for (int l = threadIdx.x; l < 32 * kCT / 4; l += kBThreads) {
              const int m = l / (kCT / 4), n = 4 * (l % (kCT / 4));
              v4f sum = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int ww = 0; ww < kBW; ++ww)
                sum += *reinterpret_cast<const v4f*>(red + (ww * 32 + m) * kCT + n);
              if (m < a.K1 && c0 + n < a.I2)
                __builtin_nontemporal_store(
                    sum * up,
                    reinterpret_cast<v4f*>(a.TB + (slab * a.K1 + m) * a.I2 + c0 + n));
            }
            __syncthreads();
          }
        }
      }
      // keep the steps in program order: the scheduler must not move a
      // step's loads ahead, where they would reuse registers still in flight
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  // TA rows of this wave's blocks.  A row block of TA (32 rows of K2
  // values) is one contiguous span of the output; it goes through the
  // wave's LDS region (free after the last column tile) so that each store
  // instruction writes 64 consecutive values.  Scattered stores straight
  // from the MFMA layout (two partial rows per instruction) left the CU
  // idle for a long tail at the end of every slab.
  float* st = reinterpret_cast<float*>(smem + w * kWaveLds);
  const int K2 = a.K2;
#pragma unroll
  for (int i = 0; i < RBW; ++i) {
    const int rb = w + kBW * i;
    if (rb < nrb) {   // wave-uniform
      float* sb = st + (i & 1) * (32 * 32);
      if (lr < K2) {
#pragma unroll
        for (int v = 0; v < 16; ++v) sb[(8 * (v / 4) + 4 * g + (v % 4)) * K2 + lr] = accA[i][v] * up;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int rows = a.I1 - rb * 32 < 32 ? a.I1 - rb * 32 : 32;
      const int64_t o = (slab * a.I1 + rb * 32) * K2;
      const int cnt = rows * K2;
      float* dst = a.TA + o;
      // non-temporal: written once, read by a later kernel (normal stores
      // of the 120 MB of TA at 1000^3 cost about three times their share
      // of the pass's bytes)
      if (((o | cnt) & 3) == 0) {   // wave-uniform
        for (int l = 4 * lane; l < cnt; l += 256)
          __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(sb + l),
                                      reinterpret_cast<v4f*>(dst + l));
      } else {
        for (int l = lane; l < cnt; l += 64) __builtin_nontemporal_store(sb[l], dst + l);
      }
    }
  }
}

// Statistics of a caller's BF16 input (no scaling: e_a = 0): ||Y||^2
// partial sums per workgroup (FP64), slabs strided over the grid.  An FP32
// input's statistics come from its conversion.
__global__ __launch_bounds__(256) void bf16_input_stats_kernel(const uint16_t* Y, int64_t A,
                                                               int64_t slab, int32_t* exps,
                                                               double* partial) {
  __shared__ double ssum[4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double acc = 0.0;
  for (int64_t a = blockIdx.x; a < A; a += gridDim.x) {
    const uint16_t* p = Y + a * slab;
    double s = 0.0;
    for (int64_t l = t; l < slab; l += 256) {
      const float v = bf16_to_f32(p[l]);
      s += static_cast<double>(v) * v;
    }
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) ssum[wv] = s;
    __syncthreads();
    if (t == 0) {
      exps[a] = 0;
      acc += (ssum[0] + ssum[1]) + (ssum[2] + ssum[3]);
    }
  }
  if (t == 0) partial[blockIdx.x] = acc;
}

// The BF16 copy of an FP32 input at scale 2^0, in the one read of Y:
// Yb[a][r][c] = bf16_rne(Y[a][r][c]) for c < I2 and zero for I2 <= c < ldy,
// plus this block's max|Y| and sum of Y^2 (FP64; NaN once a value is not
// finite) in pmax / psum [A][gridDim.x].  Slab a is row blockIdx.y of the
// grid; each thread writes kCvtGroups groups of 4 consecutive copy
// values (8-byte stores of 16-byte loads), consecutive threads on
// consecutive groups of the padded slab, so every wavefront instruction
// moves one contiguous span except where it crosses a row end.  Many small workgroups keep enough
// loads and stores in flight to overlap the two streams.
// Two groups per thread (8 KB read, 4 KB written per workgroup): at
// 1000^3 this ran at 5.96 TB/s against 5.29 with four groups and 5.12 with
// one, measured on the same kernel body.
constexpr int kCvtThreads = 256, kCvtGroups = 2;

__device__ __forceinline__ float4 load_group(const float* src, uint32_t gi, uint32_t q,
                                             uint32_t ng, int I2) {
  const uint32_t r = gi / q, c = 4 * (gi - r * q);
  return gi < ng && c < static_cast<uint32_t>(I2)
             ? *reinterpret_cast<const float4*>(src + r * I2 + c)
             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ __launch_bounds__(kCvtThreads) void bf16_convert_kernel(const float* Y,
                                                                    uint16_t* Yb, int I1,
                                                                    int I2, int ldy, int nb,
                                                                    float* pmax,
                                                                    double* psum) {
  __shared__ float smax[kCvtThreads / 64];
  __shared__ double ssum[kCvtThreads / 64];
  // one-dimensional grid of A * nb blocks: block b of slab a is a * nb + b
  const int64_t a = blockIdx.x / static_cast<uint32_t>(nb);
  const uint32_t blk = blockIdx.x - static_cast<uint32_t>(a) * static_cast<uint32_t>(nb);
  // I1 * ldy < 2^30 (shape check), so 32-bit group and value indexes
  const uint32_t q = static_cast<uint32_t>(ldy) / 4;   // groups per copy row
  const uint32_t ng = static_cast<uint32_t>(I1) * q;   // groups per copy slab
  const float* src = Y + a * I1 * I2;
  uint2* dst = reinterpret_cast<uint2*>(Yb + a * I1 * ldy);
  const uint32_t g0 = blk * (kCvtThreads * kCvtGroups) + threadIdx.x;
  float4 v[kCvtGroups];
#pragma unroll
  for (int u = 0; u < kCvtGroups; ++u) v[u] = load_group(src, g0 + u * kCvtThreads, q, ng, I2);
  float mx = 0.0f;
  double sq = 0.0;
  bool finite = true;
#pragma unroll
  for (int u = 0; u < kCvtGroups; ++u) {
    const uint32_t gi = g0 + u * kCvtThreads;
    if (gi < ng)   // non-temporal: the copy is read again only by later passes
      __builtin_nontemporal_store(v2u{pack2(v[u].x, v[u].y), pack2(v[u].z, v[u].w)},
                                  reinterpret_cast<v2u*>(dst) + gi);
    const float ax = fabsf(v[u].x), ay = fabsf(v[u].y), az = fabsf(v[u].z), aw = fabsf(v[u].w);
    mx = fmaxf(mx, fmaxf(fmaxf(ax, ay), fmaxf(az, aw)));
    const double dx = v[u].x, dy = v[u].y, dz = v[u].z, dw = v[u].w;
    sq += (dx * dx + dy * dy) + (dz * dz + dw * dw);
    // NaN fails every comparison and Inf exceeds the largest finite float
    finite = finite && ax <= FLT_MAX && ay <= FLT_MAX && az <= FLT_MAX && aw <= FLT_MAX;
  }
  if (!finite) sq = __longlong_as_double(0x7ff8000000000000LL);
  sq = wave_sum(sq);
  mx = wave_max(mx);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    smax[wv] = mx;
    ssum[wv] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = smax[0];
    double t = ssum[0];
#pragma unroll
    for (int w = 1; w < kCvtThreads / 64; ++w) {
      m = fmaxf(m, smax[w]);
      t += ssum[w];
    }
    pmax[blockIdx.x] = m;   // [a][blk]
    psum[blockIdx.x] = t;
  }
}

// Per slab (one workgroup each): max|Y[a]| and ||Y[a]||^2 from the
// conversion blocks' partials in a fixed order, and e_a (0 inside the
// window; the exponent of the maximum, clamped so 2^-e stays finite,
// outside it).
__global__ __launch_bounds__(256) void slab_finish_kernel(const float* pmax,
                                                          const double* psum, int nb,
                                                          int32_t* exps, double* slab_sum) {
  __shared__ double red[4];
  __shared__ float rmax[4];
  const int64_t a = blockIdx.x;
  float m = 0.0f;
  double t = 0.0;
  for (int j = threadIdx.x; j < nb; j += 256) {
    m = fmaxf(m, pmax[a * nb + j]);
    t += psum[a * nb + j];
  }
  m = wave_max(m);
  t = wave_sum(t);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    rmax[wv] = m;
    red[wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float mm = fmaxf(fmaxf(rmax[0], rmax[1]), fmaxf(rmax[2], rmax[3]));
    int e = 0;
    if (mm > 0.0f && mm <= FLT_MAX) e = ilogbf(mm);
    e = e < -126 ? -126 : (e > 127 ? 127 : e);
    exps[a] = (e >= -kScaleWindow && e <= kScaleWindow) ? 0 : e;
    slab_sum[a] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// The slabs with e_a != 0 again, scaled: Yb = bf16_rne(Y * 2^-e_a) (one
// workgroup per slab; the others return at once).
__global__ __launch_bounds__(256) void bf16_rescale_kernel(const float* Y, uint16_t* Yb,
                                                           const int32_t* exps, int I1,
                                                           int I2, int ldy) {
  const int64_t a = blockIdx.x;
  const int e = exps[a];
  if (e == 0) return;
  const float down = ldexpf(1.0f, -e);
  const uint32_t q = static_cast<uint32_t>(ldy) / 4;
  const uint32_t ng = static_cast<uint32_t>(I1) * q;
  const float* src = Y + a * I1 * I2;
  uint2* dst = reinterpret_cast<uint2*>(Yb + a * I1 * ldy);
  for (uint32_t gi = threadIdx.x; gi < ng; gi += 256) {
    const float4 v = load_group(src, gi, q, ng, I2);
    dst[gi] = make_uint2(pack2(v.x * down, v.y * down), pack2(v.z * down, v.w * down));
  }
}

// Bt[k][c] = bf16_rne(B[c][k]) for k < K, c < I; zero in the padding
// (k < 32, c < ld).
__global__ void prep_bt_kernel(const float* B, int I, int K, uint16_t* Bt, int ld) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= 32 * ld) return;
  const int k = l / ld, c = l % ld;
  Bt[l] = (k < K && c < I) ? f32_to_bf16_rne(B[static_cast<int64_t>(c) * K + k]) : 0;
}

int stats_grid(int64_t A) { return static_cast<int>(A < 1024 ? A : 1024); }

template <bool DOQ, bool HALF, int RBW>
int launch_bf(const BfArgs& a, int grid, hipStream_t s) {
  auto k = bf16_stream_kernel<DOQ, HALF, RBW>;
  // per-wave regions (transposed tile / TB partial, then the TA staging),
  // plus B1^T for the dual pass
  const size_t lds = static_cast<size_t>(kBW) * kWaveLds +
                     (DOQ ? static_cast<size_t>(32) * (a.ldb1 + kB1Pad) * 2 : 0);
  {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return hip_fail(e, "bf16 stream LDS attribute");
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(kBThreads), lds, s, a);
  RT_LAUNCH_CHECK("bf16 stream");
  return kOk;
}

template <bool DOQ, bool HALF>
int launch_bf_rbw(const BfArgs& a, int grid, hipStream_t s) {
  // row-block steps per column tile: the blocks a wave owns, rounded up to 1, 2, 4
  const int nrb = (a.I1 + 31) / 32;
  const int per_wave = (nrb + kBW - 1) / kBW;
  if (per_wave <= 1) return launch_bf<DOQ, HALF, 1>(a, grid, s);
  if (per_wave <= 2) return launch_bf<DOQ, HALF, 2>(a, grid, s);
  return launch_bf<DOQ, HALF, 4>(a, grid, s);
}

template <bool DOQ>
int launch_bf_half(const BfArgs& a, int grid, hipStream_t s) {
  // rows that start 8-byte aligned (ldy % 8 == 4) take the half-chunk loads
  if ((a.ldy & 7) != 0) return launch_bf_rbw<DOQ, true>(a, grid, s);
  return launch_bf_rbw<DOQ, false>(a, grid, s);
}

// ---------------------------------------------------------------------------
// Column-split pass, for slabs of 7..16 column tiles (384 < I2 <= 1024).
//
// Wave w owns the column tiles w and w + 8 of the slab (CPW = 2; CPW = 1
// when the slab has at most 8) and walks its 32-row blocks from top to
// bottom, so the 8 waves read one row block, a contiguous span of the slab,
// at a time.  For each 32 x 64 tile:
//   TA partial += M_tile B2_tile       (K = the tile's columns; the wave's
//                                      B2^T operands stay in registers)
//   TB_j       += B1_block^T M_tile    (K = the block's rows, B operand read
//                                      transposed from the wave's row-major
//                                      copy of the tile in LDS)
// After its tiles of a row block a wave parks its TA partial in LDS; one
// barrier per row block, then the partials are summed over the 8 waves in a
// fixed order into the block's TA rows, which are stored and kept in LDS for
//   C += B1_block^T TA_block           (FP32 MFMA: the mode-(N-1) product of
//                                      TA inside the slab, K1 x K2 per slab)
// TB is complete in each wave at the end (its columns, every row).  Both
// passes of the method that need TA only through C (the core, and the
// sketches of modes < N-1) read 3.6 MB instead of 120 MB at 1000^3.
//
// FIRST: the tiles come from the FP32 tensor.  The pass writes the BF16 copy
// at scale 2^0 and the slab's max|Y| and ||Y||^2 (FP64, NaN if a value is
// not finite), and multiplies the BF16-rounded values, so one read of Y
// replaces the conversion pass and the first sweep's read of the copy.  The
// rare slabs whose exponent puts them outside the window are converted again
// afterwards and their products recomputed from the scaled copy
// (only_scaled).
struct CsArgs {
  const float* Yf;        // FIRST: FP32 tensor [A][I1][I2]
  uint16_t* Yb;           // BF16 copy [A][I1][ldy]: written (FIRST) or read
  const int32_t* exps;    // per-slab exponent (not FIRST)
  float* smax;            // FIRST: per-slab max|Y|
  double* ssum;           // FIRST: per-slab sum of squares
  int only_scaled;        // skip the slabs whose exponent is 0
  int I1, I2, ldy, nct;
  const uint16_t* B2t;    // [32][ldb2] BF16, zero beyond (K2, I2)
  int ldb2, K2;
  const uint16_t* B1t;    // [32][ldb1] BF16, zero beyond (K1, I1) (DOQ)
  int ldb1, K1;
  const float* B1;        // [I1][K1] FP32 (C)
  float* TA;              // [A][I1][K2] or null
  float* TB;              // [A][K1][I2] (DOQ)
  float* C;               // [A][K1][K2] or null
};

constexpr int kCsRed = kBW * 32 * 32;   // floats of one TA-partial buffer
constexpr int kYtBytes = kCT * kYtStride * 2;   // a wave's transposed tile
constexpr int kStPitch = 144;                   // bytes per row of a staged BF16 tile (padded)
constexpr int kStBytes = 32 * kStPitch;
static_assert(kYtBytes % 16 == 0 && kStPitch % 16 == 0, "16-byte LDS accesses");

// per-wave LDS of the column-split pass: one 32 x 64 BF16 tile, row-major
// (rows of kStPitch bytes).  FIRST stages the copy through it; TB reads it
// back transposed.
constexpr int cs_wave_bytes(bool first, bool doq) {
  return (first || doq) ? kStBytes : 0;
}

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));

// TB's B operand of the 32x32x16 BF16 product from the wave's row-major
// tile (rows = the K of the product): lane l = 16 G + i gets rows
// k0 + 8 (G / 2) + 0..7 of column n0 + 16 (G % 2) + i.  ds_read_b64_tr_b16
// hands lane j of a 16-lane group element j % 4 of the four halfwords that
// lanes 4 k + j / 4 address (k = 0..3); so each of the two loads points
// lane i at row (i / 4) of its 4-row half and columns 4 (i % 4) .. + 3, and
// lane i receives four consecutive rows of column i.
__device__ __forceinline__ v8bf tile_b_operand(const char* tile, int k0, int n0, int lane) {
  const int G = lane >> 4, i = lane & 15;
  const int row = k0 + 8 * (G >> 1) + (i >> 2);
  const int col = n0 + 16 * (G & 1) + 4 * (i & 3);
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_v4s*)(tile + row * kStPitch + 2 * col));
  const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_v4s*)(tile + (row + 4) * kStPitch + 2 * col));
  const v8s v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(v8bf, v);
}

template <bool F>
struct CsTile {
  v4u v[F ? 8 : 4];   // FP32: 2 x 4 values per 8-column chunk; BF16: 8 values
};

// Tile of step (row block t, column tile ct): lane (lr, g) takes row
// 32 t + lr and, for chunk q, columns 64 ct + 16 q + 8 g .. + 7.  Masked
// lanes (rows past the slab, tiles past the last) read past the buffer
// range and get zeros.
template <bool FIRST>
__device__ __forceinline__ void cs_load(__amdgpu_buffer_rsrc_t rs, const CsArgs& a, int t,
                                        int ct, int lr, int g, CsTile<FIRST>& T) {
  const int r = t * 32 + lr;
  const bool rok = r < a.I1 && ct < a.nct;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (FIRST) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = ct * kCT + 16 * q + 8 * g + 4 * h;
        const bool ok = rok && c < a.I2;   // I2 % 4 == 0: all four or none
        const int off = ok ? ((ok ? r : 0) * a.I2 + (ok ? c : 0)) * 4 : kOob;
        T.v[2 * q + h] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      }
    } else {
      const int c = ct * kCT + 16 * q + 8 * g;
      const bool ok = rok && c < a.I2;     // I2 % 8 == 0 or zero padding
      const int off = ok ? ((ok ? r : 0) * a.ldy + (ok ? c : 0)) * 2 : kOob;
      T.v[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    }
  }
}

template <bool FIRST, bool DOQ, int CPW>
__global__ __launch_bounds__(kBThreads) void bf16_cs_kernel(CsArgs a) {
  extern __shared__ __align__(16) char smem[];
  constexpr int kSlots = FIRST ? 2 : 4;   // tiles in registers (FP32 tiles are twice as big)
  constexpr int kTrip = 4;                // steps per loop trip
  constexpr int kRpt = kTrip / CPW;       // row blocks per trip (even)
  static_assert(kTrip % kSlots == 0 && kTrip % CPW == 0 && kRpt % 2 == 0, "static indexing");
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 31, g = lane >> 5;
  // LDS: per-wave regions (transposed tile for TB, staged copy tile), two
  // TA-partial buffers, two reduced TA blocks, statistics
  constexpr int kWave = cs_wave_bytes(FIRST, DOQ);
  char* stg = smem + w * kWave;   // the wave's row-major tile
  float* red = reinterpret_cast<float*>(smem + kBW * kWave);
  float* tab = red + 2 * kCsRed;
  double* sred = reinterpret_cast<double*>(tab + 2 * 1024);
  float* mred = reinterpret_cast<float*>(sred + kBW);

  const int64_t slab = blockIdx.x;
  int e = 0;
  if constexpr (!FIRST) {
    e = a.exps[slab];
    if (a.only_scaled && e == 0) return;   // workgroup-uniform
  }
  const float up = ldexpf(1.0f, e);
  const int nrb = (a.I1 + 31) / 32;
  const int nsteps = (nrb * CPW + kTrip - 1) / kTrip * kTrip;   // masked steps past the end
  const int64_t slab_b = static_cast<int64_t>(a.I1) * a.ldy;
  const __amdgpu_buffer_rsrc_t rs =
      FIRST ? slab_rsrc(a.Yf + slab * a.I1 * a.I2, static_cast<int64_t>(a.I1) * a.I2 * 4)
            : slab_rsrc(a.Yb + slab * slab_b, slab_b * 2);
  // C is made by the passes over the copy only (the FIRST pass has no
  // registers to spare for it)
  const bool wantC = !FIRST && a.C != nullptr, wantA = a.TA != nullptr;

  // operands that do not change along the slab, then the first row
  // block's, then the ring: the loop head's wait counts then hold for the
  // entry as for the back edge
  v8bf b2[CPW][4];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int ct = w + kBW * j < a.nct ? w + kBW * j : 0;   // masked tiles: any valid row
    load_b2t(a.B2t, a.ldb2, ct, lr, g, b2[j]);
  }
  // B1^T of row block t (TB's A operand), loaded one row block ahead, and
  // B1 rows of block t (C's A operand, rows 4w .. 4w+3), loaded at the
  // block's first step and used at the end of the next block: slot t % 2
  uint4 b1r[2][2];
  float b1c[2][2];
  auto load_b1t = [&](int t, int slot) __attribute__((always_inline)) {
    const int tc = t < nrb ? t : nrb - 1;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      b1r[slot][h] = *reinterpret_cast<const uint4*>(
          a.B1t + static_cast<int64_t>(lr) * a.ldb1 + tc * 32 + 16 * h + 8 * g);
  };
  auto load_b1c = [&](int t, int slot) __attribute__((always_inline)) {
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      const int row = t * 32 + 4 * w + 2 * t2 + g;
      const bool ok = wantC && row < a.I1 && lr < a.K1;
      b1c[slot][t2] = ok ? a.B1[static_cast<int64_t>(ok ? row : 0) * a.K1 + lr] : 0.0f;
    }
  };
  if constexpr (DOQ) load_b1t(0, 0);
  __builtin_amdgcn_sched_barrier(0);
  CsTile<FIRST> ring[kSlots];
#pragma unroll
  for (int k = 0; k + 1 < kSlots; ++k)
    cs_load<FIRST>(rs, a, k / CPW, w + kBW * (k % CPW), lr, g, ring[k]);
  __builtin_amdgcn_sched_barrier(0);

  v16f accA, accC;
  v16f accB[CPW][2];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    accA[v] = 0.0f;
    accC[v] = 0.0f;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      accB[j][0][v] = 0.0f;
      accB[j][1][v] = 0.0f;
    }
  }
  uint32_t mxb = 0;   // FIRST: the lane's largest |Y| bit pattern
  double sq = 0.0;

  // C += B1_block^T TA_block for row block t (rows 4w .. 4w+3 of the block)
  auto c_step = [&](int slot, int buf) __attribute__((always_inline)) {
    const float* tb = tab + buf * 1024;
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
      accC = __builtin_amdgcn_mfma_f32_32x32x2f32(b1c[slot][t2],
                                                  tb[(4 * w + 2 * t2 + g) * 32 + lr], accC,
                                                  0, 0, 0);
  };

  for (int s0 = 0; s0 < nsteps; s0 += kTrip) {
    static_for<kTrip>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      constexpr int j = u % CPW;              // column tile of the wave
      constexpr int tl = u / CPW;             // row block within the trip
      constexpr int par = tl % 2;             // parity of the row block
      const int t = s0 / CPW + tl;
      const int ct = w + kBW * j;
      if constexpr (j == 0) {
        if constexpr (DOQ) load_b1t(t + 1, par ^ 1);
        if constexpr (!FIRST) load_b1c(t, par);
      }
      {
        constexpr int up_ = u + kSlots - 1;   // step whose tile is loaded now
        const int sp = s0 + up_;
        cs_load<FIRST>(rs, a, sp / CPW, w + kBW * (up_ % CPW), lr, g,
                       ring[up_ % kSlots]);
      }
      __builtin_amdgcn_sched_barrier(0);
      CsTile<FIRST>& cur = ring[u % kSlots];
      uint4 yb[4];
      if constexpr (FIRST) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float x[8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            x[4 * h + 0] = __uint_as_float(cur.v[2 * q + h].x);
            x[4 * h + 1] = __uint_as_float(cur.v[2 * q + h].y);
            x[4 * h + 2] = __uint_as_float(cur.v[2 * q + h].z);
            x[4 * h + 3] = __uint_as_float(cur.v[2 * q + h].w);
          }
          yb[q] = make_uint4(pack2_hw(x[0], x[1]), pack2_hw(x[2], x[3]),
                             pack2_hw(x[4], x[5]), pack2_hw(x[6], x[7]));
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t ab = __float_as_uint(x[k]) & 0x7fffffffu;
            mxb = mxb > ab ? mxb : ab;
            sq = fma(static_cast<double>(x[k]), static_cast<double>(x[k]), sq);
          }
          // keep the statistics here: left alone, the compiler sinks them
          // to the end of the loop trip and keeps four tiles live for them
          asm volatile("" : "+v"(mxb), "+v"(sq));
        }
        // the copy (rows of the slab, every column of the tile: the
        // padding past I2 was loaded as zeros).  The tile goes through the
        // wave's LDS so that each store instruction writes 8 whole rows of
        // 128 bytes; stored from the MFMA layout (32 rows x 32 bytes per
        // instruction) the copy's writes ran at a third of the bandwidth.
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<uint4*>(stg + lr * kStPitch + 32 * q + 16 * g) = yb[q];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ct < a.nct) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rl = 8 * i + (lane >> 3), r = t * 32 + rl;
            const v4u v = *reinterpret_cast<const v4u*>(stg + rl * kStPitch + 16 * (lane & 7));
            if (r < a.I1)
              __builtin_nontemporal_store(
                  v, reinterpret_cast<v4u*>(a.Yb + slab * slab_b + static_cast<int64_t>(r) * a.ldy +
                                            ct * kCT + 8 * (lane & 7)));
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          yb[q] = make_uint4(cur.v[q].x, cur.v[q].y, cur.v[q].z, cur.v[q].w);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        accA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(yb[q]), b2[j][q], accA, 0, 0, 0);
      if constexpr (DOQ) {
        // TB += B1_block^T M_tile: the tile row-major in the wave's LDS
        // (FIRST staged it there for the copy already), read back transposed
        if constexpr (!FIRST) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *reinterpret_cast<uint4*>(stg + lr * kStPitch + 32 * q + 16 * g) = yb[q];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int sh = 0; sh < 2; ++sh) {
            const v8bf yc = tile_b_operand(stg, 16 * h, 32 * sh, lane);
            accB[j][sh] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_v8bf(b1r[par][h]), yc,
                                                                accB[j][sh], 0, 0, 0);
          }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if constexpr (j == CPW - 1) {
        // row block t done in this wave: park the TA partial, then sum the
        // 8 partials (fixed order) into the block's TA rows
        float* rp = red + par * kCsRed + w * 1024;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          rp[(8 * (v / 4) + 4 * g + (v % 4)) * 32 + lr] = accA[v];
          accA[v] = 0.0f;
        }
        __syncthreads();
        // the previous block's C product: its TA block was completed
        // before this barrier
        if constexpr (!FIRST)
          if (wantC && t >= 1) c_step(par ^ 1, par ^ 1);
        for (int o = threadIdx.x; o < 1024; o += kBThreads) {
          float sum = 0.0f;
#pragma unroll
          for (int ww = 0; ww < kBW; ++ww) sum += red[par * kCsRed + ww * 1024 + o];
          sum *= up;
          if (wantC) tab[par * 1024 + o] = sum;
          const int row = t * 32 + o / 32, k = o % 32;
          if (wantA && row < a.I1 && k < a.K2)
            __builtin_nontemporal_store(sum, a.TA + (slab * a.I1 + row) * a.K2 + k);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  // the last row block's C product, then C summed over the waves
  const int tlast = nsteps / CPW - 1;
  __syncthreads();
  if constexpr (!FIRST)
    if (wantC) c_step(tlast & 1, tlast & 1);
  if constexpr (FIRST) {
    // a pattern above FLT_MAX's is an Inf or a NaN
    if (mxb > 0x7f7fffffu) sq = __longlong_as_double(0x7ff8000000000000LL);
    sq = wave_sum(sq);
    const float mx = wave_max(__uint_as_float(mxb > 0x7f7fffffu ? 0x7f800000u : mxb));
    if (lane == 0) {
      sred[w] = sq;
      mred[w] = mx;
    }
  }
  if (!FIRST && wantC) {
    float* rp = red + w * 1024;   // every reduction of the loop has finished
#pragma unroll
    for (int v = 0; v < 16; ++v) rp[(8 * (v / 4) + 4 * g + (v % 4)) * 32 + lr] = accC[v];
  }
  __syncthreads();
  if (wantC) {
    for (int o = threadIdx.x; o < 1024; o += kBThreads) {
      const int k1 = o / 32, k2 = o % 32;
      float sum = 0.0f;
#pragma unroll
      for (int ww = 0; ww < kBW; ++ww) sum += red[ww * 1024 + o];
      if (k1 < a.K1 && k2 < a.K2)
        __builtin_nontemporal_store(sum, a.C + (slab * a.K1 + k1) * a.K2 + k2);
    }
  }
  if constexpr (FIRST) {
    if (threadIdx.x == 0) {
      float m = mred[0];
      double t = sred[0];
#pragma unroll
      for (int ww = 1; ww < kBW; ++ww) {
        m = fmaxf(m, mred[ww]);
        t += sred[ww];
      }
      a.smax[slab] = m;
      a.ssum[slab] = t;
    }
  }
  if constexpr (DOQ) {
    // TB: the slab's K1 x I2 block is one contiguous span of the output.
    // Staged through LDS 16 rows at a time (the TA-partial buffers are
    // free), then written with 16-byte stores in order.
    float* tbs = red;   // [16][1024]
    static_assert(2 * kCsRed >= 16 * 1024, "TB staging fits");
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      __syncthreads();   // the previous use of the buffers is over
#pragma unroll
      for (int j = 0; j < CPW; ++j) {
        const int ct = w + kBW * j;
        if (ct < a.nct) {
#pragma unroll
          for (int sh = 0; sh < 2; ++sh)
#pragma unroll
            for (int v = 8 * half; v < 8 * half + 8; ++v) {
              const int k1l = 8 * (v / 4) + 4 * g + (v % 4) - 16 * half;
              tbs[k1l * 1024 + ct * kCT + 32 * sh + lr] = accB[j][sh][v] * up;
            }
        }
      }
      __syncthreads();
      const int rows = a.K1 - 16 * half < 16 ? a.K1 - 16 * half : 16;
      if (rows > 0) {
        float* dst = a.TB + (slab * a.K1 + 16 * half) * a.I2;   // I2 % 4 == 0: aligned
        const int cnt = rows * a.I2;
        for (int o = 4 * threadIdx.x; o < cnt; o += 4 * kBThreads) {
          const int k1l = o / a.I2, col = o - k1l * a.I2;
          __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(tbs + k1l * 1024 + col),
                                      reinterpret_cast<v4f*>(dst + o));
        }
      }
    }
  }
}

// LDS of the column-split pass
size_t cs_lds_bytes(bool first, bool doq) {
  return static_cast<size_t>(kBW) * cs_wave_bytes(first, doq) +
         (2 * kCsRed + 2 * 1024) * sizeof(float) + kBW * (sizeof(double) + sizeof(float));
}

template <bool FIRST, bool DOQ, int CPW>
int launch_cs(const CsArgs& a, int64_t grid, hipStream_t s) {
  auto k = bf16_cs_kernel<FIRST, DOQ, CPW>;
  const size_t lds = cs_lds_bytes(FIRST, DOQ);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return hip_fail(e, "bf16 column-split LDS attribute");
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(grid)), dim3(kBThreads), lds, s, a);
  RT_LAUNCH_CHECK("bf16 column-split pass");
  return kOk;
}

template <bool FIRST, bool DOQ>
int launch_cs_cpw(const CsArgs& a, int64_t grid, hipStream_t s) {
  if (a.nct <= kBW) return launch_cs<FIRST, DOQ, 1>(a, grid, s);
  return launch_cs<FIRST, DOQ, 2>(a, grid, s);
}

int launch_cs_first(const CsArgs& a, bool doq, bool first, int64_t grid, hipStream_t s) {
  if (first) return doq ? launch_cs_cpw<true, true>(a, grid, s) : launch_cs_cpw<true, false>(a, grid, s);
  return doq ? launch_cs_cpw<false, true>(a, grid, s) : launch_cs_cpw<false, false>(a, grid, s);
}

}  // namespace

int64_t bf16_copy_ld(int64_t I2) { return (I2 + kCopyAlign - 1) / kCopyAlign * kCopyAlign; }

namespace {

// conversion blocks per slab
int64_t cvt_blocks(int64_t I1, int64_t I2) {
  const int64_t per_block = static_cast<int64_t>(kCvtThreads) * kCvtGroups * 4;
  return (I1 * bf16_copy_ld(I2) + per_block - 1) / per_block;
}

// Workspace of the BF16 passes (inside the streaming workspace), in order:
// slab exponents (int32, A), the two transposed BF16 factor copies, the
// conversion blocks' partial sums (FP64, A x nb), their maxima (FP32,
// A x nb) and the slab sums (FP64, A).
struct BfWs {
  int32_t* exps;
  uint16_t* B2t;
  uint16_t* B1t;
  double* psum;
  float* pmax;
  double* slab_sum;
  size_t bytes;
};

BfWs bf16_ws_layout(char* base, int64_t A, int64_t I1, int64_t I2) {
  const int64_t l1 = (I1 + 63) / 64 * 64, l2 = (I2 + 63) / 64 * 64;
  const int64_t nb = cvt_blocks(I1, I2);
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  BfWs w{};
  int64_t o = 0;
  w.exps = reinterpret_cast<int32_t*>(base + o);
  o += up(A * 4);
  w.B2t = reinterpret_cast<uint16_t*>(base + o);
  o += up(2 * 32 * l2);
  w.B1t = reinterpret_cast<uint16_t*>(base + o);
  o += up(2 * 32 * l1);
  w.psum = reinterpret_cast<double*>(base + o);
  o += up(A * nb * 8);
  w.pmax = reinterpret_cast<float*>(base + o);
  o += up(A * nb * 4);
  w.slab_sum = reinterpret_cast<double*>(base + o);
  o += up(A * 8);
  w.bytes = static_cast<size_t>(o);
  return w;
}

}  // namespace

size_t bf16_stream_workspace_bytes(int64_t A, int64_t I1, int64_t I2) {
  return bf16_ws_layout(nullptr, A, I1, I2).bytes + 512;
}

namespace {

// The column-split pass takes slabs of 7..16 column tiles whose rows start
// 16-byte aligned (the padded copy, or a caller's BF16 tensor with
// I2 % 8 == 0) and whose FP32 and BF16 slabs stay below the masked-load
// offset; it has no limit on the number of rows.
bool cs_ok(int64_t I1, int64_t I2, int64_t ldy) {
  const int64_t nct = (I2 + kCT - 1) / kCT;
  return nct >= 7 && nct <= 2 * kBW && ldy % 8 == 0 && I1 * ldy * 2 <= kOob - 64 &&
         I1 * I2 * 4 <= kOob - 64;
}

}  // namespace

int bf16_check_shape(int64_t A, int64_t I1, int64_t I2, int K1, int K2, bool bf16_input) {
  const int64_t ldy = bf16_input ? I2 : bf16_copy_ld(I2);
  const bool cs = cs_ok(I1, I2, ldy);
  // a slab of the padded copy must stay below the masked-load offset
  if ((I1 > kMaxI1 && !cs) || I2 % 4 != 0 || K1 > 32 || K2 > 32 ||
      I1 * bf16_copy_ld(I2) * 2 > kOob - 64) {
    set_error("BF16 streaming pass needs I_{N-1} <= %d (or 384 < I_N <= 1024), "
              "I_N %% 4 == 0, I_{N-1} I_N < 2^30 and sketch widths <= 32 "
              "(got %lld, %lld, %d, %d)",
              kMaxI1, (long long)I1, (long long)I2, K1, K2);
    return kErrUnsupported;
  }
  // one-dimensional grids: A slabs (streaming passes), A x blocks per slab
  // (conversion)
  if (A > 0x7fffffffLL || (!cs && A * cvt_blocks(I1, I2) > 0x7fffffffLL)) {
    set_error("BF16 conversion: %lld slabs of %lld x %lld exceed 2^31 - 1 blocks",
              (long long)A, (long long)I1, (long long)I2);
    return kErrUnsupported;
  }
  return kOk;
}

// One BF16 streaming pass: TA = Y x_N B2^T (when TA is given), TB = Y
// x_{N-1} B1^T (when TB is given) and C = TA x_{N-1} B1^T per slab (when C
// is given and the slab shape takes the column-split pass: *c_done tells;
// without TB such a pass does not write TA).
// first: the pass also takes the statistics and, for an FP32 input, makes
// the BF16 copy.
int bf16_stream_pass(const StreamCtx& c, bool first, const float* B2, int K2,
                     const float* B1, int K1, float* TA, float* TB, float* C, bool* c_done,
                     int stage, hipStream_t s) {
  RT_TRY(bf16_check_shape(c.A, c.I1, c.I2, B1 ? K1 : 0, K2, c.bf16_input));
  const bool cs = cs_ok(c.I1, c.I2, c.ldy);
  if (c_done) *c_done = false;
  if (!cs) C = nullptr;
  if (C && !TB) TA = nullptr;   // the core pass needs TA only through C
  if (!TA && !C) {
    set_error("BF16 streaming pass without an output");
    return kErrInvalid;
  }
  const int64_t l1 = (c.I1 + 63) / 64 * 64, l2 = (c.I2 + 63) / 64 * 64;
  char* base = static_cast<char*>(c.ws) + 1024 * sizeof(double) + 256;
  const BfWs w = bf16_ws_layout(base, c.A, c.I1, c.I2);
  int32_t* exps = w.exps;
  uint16_t* B2t = w.B2t;
  uint16_t* B1t = w.B1t;
  if (first && c.bf16_input) {
    const int g = stats_grid(c.A);
    ProfScope ps(kStageStats, s);
    hipLaunchKernelGGL(bf16_input_stats_kernel, dim3(g), dim3(256), 0, s, c.ybf16, c.A,
                       c.I1 * c.I2, exps, c.norm_partial);
    RT_LAUNCH_CHECK("slab stats");
    RT_TRY(launch_sum_partials(c.norm_partial, g, c.norm_out, c.nonfinite, s));
  }
  hipLaunchKernelGGL(prep_bt_kernel, dim3((32 * l2 + 255) / 256), dim3(256), 0, s, B2,
                     static_cast<int>(c.I2), K2, B2t, static_cast<int>(l2));
  RT_LAUNCH_CHECK("prep B2");
  if (TB) {
    hipLaunchKernelGGL(prep_bt_kernel, dim3((32 * l1 + 255) / 256), dim3(256), 0, s,
                       B1, static_cast<int>(c.I1), K1, B1t, static_cast<int>(l1));
    RT_LAUNCH_CHECK("prep B1");
  }

  if (cs) {
    CsArgs a{};
    a.Yf = static_cast<const float*>(c.y);
    a.Yb = c.ybf16;
    a.exps = exps;
    a.smax = w.pmax;    // one value per slab
    a.ssum = w.psum;
    a.I1 = static_cast<int>(c.I1);
    a.I2 = static_cast<int>(c.I2);
    a.ldy = static_cast<int>(c.ldy);
    a.nct = static_cast<int>((c.I2 + kCT - 1) / kCT);
    a.B2t = B2t;
    a.ldb2 = static_cast<int>(l2);
    a.K2 = K2;
    a.B1t = B1t;
    a.ldb1 = static_cast<int>(l1);
    a.K1 = B1 ? K1 : 0;
    a.B1 = B1;
    a.TA = TA;
    a.TB = TB;
    a.C = C;
    if (first && !c.bf16_input) {
      // one read of Y: the BF16 copy at scale 2^0, the statistics and the
      // products of the rounded values; then the slab exponents, and the
      // slabs that need a scale are converted again and recomputed.  This
      // pass makes no C (TA is written instead).
      if (!TA) {
        set_error("the first BF16 pass writes TA");
        return kErrInvalid;
      }
      C = nullptr;
      a.C = nullptr;
      {
        ProfScope ps(stage, s);
        RT_TRY(launch_cs_first(a, TB != nullptr, true, c.A, s));
      }
      ProfScope ps(kStageStats, s);
      hipLaunchKernelGGL(slab_finish_kernel, dim3(static_cast<unsigned>(c.A)), dim3(256), 0, s,
                         w.pmax, w.psum, 1, exps, w.slab_sum);
      RT_LAUNCH_CHECK("slab finish");
      hipLaunchKernelGGL(bf16_rescale_kernel, dim3(static_cast<unsigned>(c.A)), dim3(256), 0,
                         s, static_cast<const float*>(c.y), c.ybf16, exps,
                         static_cast<int>(c.I1), static_cast<int>(c.I2),
                         static_cast<int>(c.ldy));
      RT_LAUNCH_CHECK("bf16 rescale");
      a.only_scaled = 1;
      RT_TRY(launch_cs_first(a, TB != nullptr, false, c.A, s));
      RT_TRY(launch_sum_partials(w.slab_sum, static_cast<int>(c.A), c.norm_out, c.nonfinite,
                                 s));
    } else {
      ProfScope ps(stage, s);
      RT_TRY(launch_cs_first(a, TB != nullptr, false, c.A, s));
    }
    if (c_done) *c_done = C != nullptr;
    return kOk;
  }

  if (first && !c.bf16_input) {
    // the BF16 copy (padded rows) and the statistics in one read of Y, then
    // the slab exponents and the rare slabs that need a scale; every
    // contraction reads the copy
    const int64_t nb = cvt_blocks(c.I1, c.I2);   // A * nb < 2^31 (shape check)
    {
      ProfScope ps(kStageConvert, s);
      hipLaunchKernelGGL(bf16_convert_kernel, dim3(static_cast<unsigned>(c.A * nb)),
                         dim3(kCvtThreads), 0, s, static_cast<const float*>(c.y), c.ybf16,
                         static_cast<int>(c.I1), static_cast<int>(c.I2),
                         static_cast<int>(c.ldy), static_cast<int>(nb), w.pmax, w.psum);
      RT_LAUNCH_CHECK("bf16 convert");
    }
    ProfScope ps(kStageStats, s);
    hipLaunchKernelGGL(slab_finish_kernel, dim3(static_cast<unsigned>(c.A)), dim3(256), 0, s,
                       w.pmax, w.psum, static_cast<int>(nb), exps, w.slab_sum);
    RT_LAUNCH_CHECK("slab finish");
    hipLaunchKernelGGL(bf16_rescale_kernel, dim3(static_cast<unsigned>(c.A)), dim3(256), 0, s,
                       static_cast<const float*>(c.y), c.ybf16, exps,
                       static_cast<int>(c.I1), static_cast<int>(c.I2),
                       static_cast<int>(c.ldy));
    RT_LAUNCH_CHECK("bf16 rescale");
    RT_TRY(launch_sum_partials(w.slab_sum, static_cast<int>(c.A), c.norm_out, c.nonfinite, s));
  }
  BfArgs a{};
  a.Y = c.ybf16;
  a.exps = exps;
  a.A = c.A;
  a.I1 = static_cast<int>(c.I1);
  a.I2 = static_cast<int>(c.I2);
  a.ldy = static_cast<int>(c.ldy);
  a.B2t = B2t;
  a.ldb2 = static_cast<int>(l2);
  a.K2 = K2;
  a.B1t = B1t;
  a.ldb1 = static_cast<int>(l1);
  a.K1 = TB ? K1 : 0;
  a.TA = TA;
  a.TB = TB;
  const int grid = static_cast<int>(c.A);   // one workgroup per slab
  ProfScope ps(stage, s);
  if (TB) return launch_bf_half<true>(a, grid, s);
  return launch_bf_half<false>(a, grid, s);
}

}  // namespace rt
