// Standalone encode: materialise every computed coded block
// C_g = sum over s in N(g) of A_s (FP32, members in ascending order), the
// master-side encode of Sec. II with XOR read as a real sum.  HBM-streaming:
// each thread produces one float4 of one coded row.  The coded GEMM does not
// use this kernel (it sums the blocks while loading its A tiles); it exists
// for tests and to measure encode bandwidth on its own.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void encode_kernel(EncodeParams p) {
  const int64_t k4 = p.K / 4;
  const int64_t per_sym = p.Mb * k4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int si = blockIdx.y;
  if (e >= per_sym) return;
  const int64_t r = e / k4;
  const int64_t kc = (e - r * k4) * 4;
  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  v4f sum = {0.f, 0.f, 0.f, 0.f};
  for (int m = 0; m < deg; ++m) {
    const int64_t row = (int64_t)p.ids[id_off + m] * p.Mb + r;
    if (row < p.M) sum += *reinterpret_cast<const v4f*>(p.A + row * p.lda + kc);
  }
  *reinterpret_cast<v4f*>(p.out + ((int64_t)si * p.Mb + r) * p.K + kc) = sum;
}

}  // namespace

hipError_t launch_encode(const EncodeParams& p, hipStream_t stream) {
  const int64_t per_sym = p.Mb * (p.K / 4);
  if (p.n_sym == 0 || per_sym == 0) return hipSuccess;
  const int64_t bx = (per_sym + 255) / 256;
  if (bx > 0x7fffffff || p.n_sym > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(encode_kernel, dim3((unsigned)bx, (unsigned)p.n_sym), dim3(256), 0, stream,
                     p);
  return hipGetLastError();
}

}  // namespace bpx
