// Coded GEMM in FP32 on MFMA (v_mfma_f32_16x16x4_f32), encode fused into
// the A-operand load.
//
// One workgroup (4 waves, 2 x 2) computes a BM x BN tile of one coded
// product Y_g = C_g . B, with C_g = sum over the symbol's data blocks A_s
// (the master-side encode of Sec. II, with the XOR of Sec. III-A read as a
// real sum).  The coded block is never stored: each K-step loads the deg(g)
// A tiles, sums them in FP32 registers and stages the sum in LDS.
//
// LDS layout: As[m][k] and Bs[k][n] (both as in global memory, padded by 4
// floats).  The k index inside a 16-wide chunk is permuted so that lane
// group q = lane/16 owns k = 4q..4q+3: MFMA t of the chunk contracts
// k = 4q + t, so each lane fetches its A values with one 128-bit LDS read.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kPre = 4;  // data blocks of a symbol prefetched ahead of the MFMAs

template <int BM, int BN, int BK>
struct F32Tile {
  static constexpr int TM = BM / 2, TN = BN / 2;  // wave tile
  static constexpr int FM = TM / 16, FN = TN / 16;
  static constexpr int LDA_S = BK + 4;            // As row stride (floats)
  static constexpr int LDB_S = BN + 4;            // Bs row stride (floats)
  static constexpr int A_F4 = BM * BK / 4 / kThreads;  // float4 per thread
  static constexpr int B_F4 = BK * BN / 4 / kThreads;
  static constexpr int A_SIZE = BM * LDA_S;
  static constexpr int B_SIZE = BK * LDB_S;
  static_assert(A_F4 >= 1 && B_F4 >= 1, "tile too small for 256 threads");
};

__device__ __forceinline__ int xcd_remap(int lin, int total) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of tiles so that tiles sharing A and B panels share an
  // L2.
  if ((total & 7) != 0) return lin;
  return (lin & 7) * (total >> 3) + (lin >> 3);
}

template <int BM, int BN, int BK>
__global__ __launch_bounds__(kThreads, 2) void coded_gemm_f32_kernel(GemmParams p) {
  using T = F32Tile<BM, BN, BK>;
  __shared__ __attribute__((aligned(16))) float lds[2 * (T::A_SIZE + T::B_SIZE)];
  float* As0 = lds;
  float* Bs0 = lds + 2 * T::A_SIZE;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = lane >> 4, c16 = lane & 15;

  const int total = gridDim.x;
  const int lin = xcd_remap(blockIdx.x, total);
  const int per_sym = p.tiles_m * p.tiles_n;
  const int si = lin / per_sym;
  const int rem = lin - si * per_sym;
  const int mt = rem / p.tiles_n;
  const int nt = rem - mt * p.tiles_n;
  const int m0 = mt * BM, n0 = nt * BN;

  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;

  const int64_t K = p.K, N = p.N, Mb = p.Mb, M = p.M;

  // Per-thread A rows / k offsets, B k-rows / n offsets.
  int a_row[T::A_F4], a_kc[T::A_F4];
#pragma unroll
  for (int i = 0; i < T::A_F4; ++i) {
    const int f = tid + kThreads * i;
    a_row[i] = f / (BK / 4);
    a_kc[i] = (f % (BK / 4)) * 4;
  }
  int b_kr[T::B_F4], b_nc[T::B_F4];
#pragma unroll
  for (int i = 0; i < T::B_F4; ++i) {
    const int f = tid + kThreads * i;
    b_kr[i] = f / (BN / 4);
    b_nc[i] = (f % (BN / 4)) * 4;
  }

  // Row bases of the (first kPre) member blocks: -1 marks an invalid row.
  auto a_rowptr = [&](int member, int i) -> const float* {
    const int64_t s = ids[member];
    const int64_t rb = m0 + a_row[i];
    const int64_t grow = s * Mb + rb;
    if (rb >= Mb || grow >= M) return nullptr;
    return p.A + grow * p.lda;
  };

  v4f pre[kPre][T::A_F4];
  v4f bre[T::B_F4];

  auto load_a_pre = [&](int k0) {
#pragma unroll
    for (int mbr = 0; mbr < kPre; ++mbr) {
#pragma unroll
      for (int i = 0; i < T::A_F4; ++i) {
        v4f v = {0.f, 0.f, 0.f, 0.f};
        if (mbr < deg) {
          const float* r = a_rowptr(mbr, i);
          const int64_t kk = k0 + a_kc[i];
          if (r && kk < K) v = *reinterpret_cast<const v4f*>(r + kk);
        }
        pre[mbr][i] = v;
      }
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int i = 0; i < T::B_F4; ++i) {
      v4f v = {0.f, 0.f, 0.f, 0.f};
      const int64_t kk = k0 + b_kr[i];
      const int64_t nn = n0 + b_nc[i];
      if (kk < K) {
        const float* r = p.B + kk * p.ldb + nn;
        if (nn + 3 < N) {
          v = *reinterpret_cast<const v4f*>(r);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (nn + e < N) v[e] = r[e];
        }
      }
      bre[i] = v;
    }
  };
  auto store_tiles = [&](int buf, int k0) {
    float* As = As0 + buf * T::A_SIZE;
    float* Bs = Bs0 + buf * T::B_SIZE;
#pragma unroll
    for (int i = 0; i < T::A_F4; ++i) {
      v4f sum = pre[0][i];
#pragma unroll
      for (int mbr = 1; mbr < kPre; ++mbr) sum += pre[mbr][i];
      // members beyond the prefetch depth (high-degree symbols)
      for (int mbr = kPre; mbr < deg; ++mbr) {
        const float* r = a_rowptr(mbr, i);
        const int64_t kk = k0 + a_kc[i];
        if (r && kk < K) sum += *reinterpret_cast<const v4f*>(r + kk);
      }
      *reinterpret_cast<v4f*>(As + a_row[i] * T::LDA_S + a_kc[i]) = sum;
    }
#pragma unroll
    for (int i = 0; i < T::B_F4; ++i)
      *reinterpret_cast<v4f*>(Bs + b_kr[i] * T::LDB_S + b_nc[i]) = bre[i];
  };

  v4f acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (int)((K + BK - 1) / BK);
  load_a_pre(0);
  load_b(0);
  store_tiles(0, 0);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      load_a_pre((kt + 1) * BK);
      load_b((kt + 1) * BK);
    }
    const float* As = As0 + buf * T::A_SIZE;
    const float* Bs = Bs0 + buf * T::B_SIZE;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      v4f a[T::FM];
      v4f b[T::FN];
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
        a[i] = *reinterpret_cast<const v4f*>(As + (wm * T::TM + i * 16 + c16) * T::LDA_S + kk +
                                             4 * q);
#pragma unroll
      for (int j = 0; j < T::FN; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          b[j][t] = Bs[(kk + 4 * q + t) * T::LDB_S + wn * T::TN + j * 16 + c16];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
          for (int j = 0; j < T::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
    }
    if (more) store_tiles(buf ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  // Epilogue: lane holds rows 4q..4q+3 of column c16 of each 16x16 subtile.
  float* out;
  int64_t ldo, rows;
  if (dest >= 0) {
    out = p.Y + (int64_t)dest * Mb * N;
    ldo = N;
    rows = Mb;
  } else {
    const int64_t s = -1 - dest;
    out = p.C + s * Mb * p.ldc;
    ldo = p.ldc;
    rows = M - s * Mb < Mb ? M - s * Mb : Mb;
  }
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) {
      const int64_t col = n0 + wn * T::TN + j * 16 + c16;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * T::TM + i * 16 + 4 * q + r;
        if (row < rows) out[row * ldo + col] = acc[i][j][r];
      }
    }
}

struct TileEntry {
  TileShape shape;
  void (*kernel)(GemmParams);
};

const TileEntry kTiles[] = {
    {{128, 128, 32}, coded_gemm_f32_kernel<128, 128, 32>},
    {{64, 64, 32}, coded_gemm_f32_kernel<64, 64, 32>},
    {{128, 64, 32}, coded_gemm_f32_kernel<128, 64, 32>},
    {{64, 128, 32}, coded_gemm_f32_kernel<64, 128, 32>},
};

}  // namespace

int32_t gemm_tile_count() { return (int32_t)(sizeof(kTiles) / sizeof(kTiles[0])); }
TileShape gemm_tile_shape(int32_t t) { return kTiles[t].shape; }

hipError_t launch_coded_gemm(const GemmParams& p0, int32_t tile, hipStream_t stream) {
  GemmParams p = p0;
  const TileEntry& e = kTiles[tile];
  p.tiles_m = (int32_t)((p.Mb + e.shape.bm - 1) / e.shape.bm);
  p.tiles_n = (int32_t)((p.N + e.shape.bn - 1) / e.shape.bn);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(e.kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
