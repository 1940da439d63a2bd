// Y-streaming passes (see stream.hpp).
#include "stream.hpp"

#include "kernels.hpp"

namespace rt {

size_t stream_workspace_bytes(const rt_tucker_desc*) { return 256; }

StreamCtx make_stream_ctx(const rt_tucker_desc* d, const void* y,
                          uint16_t* ybf16, void* ws, size_t ws_bytes) {
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
  return c;
}

template <typename T>
int stream_dual(const StreamCtx& c, int, const T* B2, int K2, const T* B1,
                int K1, T* TA, T* TB, hipStream_t s) {
  if (c.precision == RT_BF16_MIXED) {
    set_error("BF16 mixed precision is not available in this build");
    return kErrUnsupported;
  }
  const T* Y = static_cast<const T*>(c.y);
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
