// Coded GEMM of the two-dimensional form in FP32 on MFMA (v_mfma_f32_16x16x4_f32).
//
// Sec. III-A, Examples 1 and 2: A is split into grid row blocks a_r (Mb rows)
// and B into grid column blocks b_c (Nb columns), and data block s = r * grid
// + c is the block product a_r b_c.  A coded symbol g sums the products of
// its data blocks:
//   * all of them share the B block c  -> (sum of their a_r) . b_c
//     (the encode is a sum of A blocks, staged while the A tile is loaded);
//   * all of them share the A block r  -> a_r . (sum of their b_c)
//     (the encode is a sum of B blocks, staged while the B tile is loaded);
//   * neither (the paper's gray cells) -> sum over members of a_r b_c, i.e.
//     the product of the K-concatenated [a_r1 | a_r2 | ...] and
//     [b_c1 ; b_c2 ; ...]: deg passes over K accumulating into one tile.
// A degree-1 symbol is the first case.  The products go to the Y slots
// (Mb x Nb) or, for degree-1 releasers, straight into their C block.
//
// One workgroup (4 waves, 2 x 2) computes a 64 x 128 output tile; its
// K-slices of 32 run over all passes, double-buffered in LDS with the next
// slice's loads in registers during the current slice's MFMAs.  LDS layout
// and fragment permutations are those of the row-block FP32 kernel: lane
// group q owns k = 4q .. 4q+3 of a 16-wide chunk (128-bit A fragment reads),
// and MFMA column c16 of subtile j is output column 4 c16 + j (128-bit B
// fragment reads, float4 epilogue stores).  Loads are raw buffer loads whose
// range check zeroes A rows past a block's last row and B rows past K; the
// last K-slice masks columns past K.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int BM = 64, BN = 128, BK = 32;
constexpr int TM = BM / 2, TN = BN / 2;  // wave tile 32 x 64
constexpr int FM = TM / 16, FN = TN / 16;
constexpr int LDA_S = BK + 4, LDB_S = BN + 4;
constexpr int A_SIZE = BM * LDA_S, B_SIZE = BK * LDB_S;
constexpr int A_F4 = BM * BK / 4 / kThreads;  // 2
constexpr int B_F4 = BK * BN / 4 / kThreads;  // 4
constexpr int kPre = 4;                       // summed blocks held in registers
constexpr int kRsrcWord3 = 0x00020000;        // gfx9 raw buffer, 32-bit elements

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0,
                                           (int)(bytes > 0 ? bytes : 0), kRsrcWord3);
}
__device__ __forceinline__ v4f bload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

__global__ __launch_bounds__(kThreads, 2) void coded_gemm_2d_kernel(GemmParams p) {
  __shared__ __attribute__((aligned(16))) float lds[2 * (A_SIZE + B_SIZE)];
  float* As0 = lds;
  float* Bs0 = lds + 2 * A_SIZE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = lane >> 4, c16 = lane & 15;

  const int per_sym = p.tiles_m * p.tiles_n;
  const int si = (int)blockIdx.x / per_sym;
  const int rem = (int)blockIdx.x - si * per_sym;
  const int mt = rem / p.tiles_n, nt = rem - mt * p.tiles_n;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;
  const int G = p.grid;
  const int64_t Mb = p.Mb, Nb = p.Nb, K = p.K, lda = p.lda, ldb = p.ldb;

  // kind: 0 = members share the B block (sum A), 1 = share the A block (sum
  // B), 2 = gray (one pass per member)
  int kind = 0;
  {
    const int r0 = ids[0] / G, c0 = ids[0] - (ids[0] / G) * G;
    bool same_r = true, same_c = true;
    for (int m = 1; m < deg; ++m) {
      const int r = ids[m] / G, c = ids[m] - r * G;
      same_r = same_r && r == r0;
      same_c = same_c && c == c0;
    }
    kind = same_c ? 0 : (same_r ? 1 : 2);
  }
  const int npass = kind == 2 ? deg : 1;
  const int nk = (int)((K + BK - 1) / BK);

  // thread's loads: A float4 f = tid + 256 i: row f / 8, k (f % 8) * 4;
  // B float4: k-row f / 32, columns (f % 32) * 4
  int a_row[A_F4], a_k[A_F4], b_k[B_F4], b_n[B_F4];
#pragma unroll
  for (int i = 0; i < A_F4; ++i) {
    const int f = tid + kThreads * i;
    a_row[i] = f >> 3;
    a_k[i] = (f & 7) * 4;
  }
#pragma unroll
  for (int i = 0; i < B_F4; ++i) {
    const int f = tid + kThreads * i;
    b_k[i] = f >> 5;
    b_n[i] = (f & 31) * 4;
  }

  v4f pa[kPre][A_F4], pb[kPre][B_F4];
  // Blocks of pass `pass`: the A blocks and B blocks whose sums feed it.
  auto n_a = [&]() __attribute__((always_inline)) { return kind == 0 ? deg : 1; };
  auto n_b = [&]() __attribute__((always_inline)) { return kind == 1 ? deg : 1; };
  auto a_blk = [&](int pass, int m) __attribute__((always_inline)) {
    const int s = ids[kind == 2 ? pass : (kind == 0 ? m : 0)];
    return s / G;
  };
  auto b_blk = [&](int pass, int m) __attribute__((always_inline)) {
    const int s = ids[kind == 2 ? pass : (kind == 1 ? m : 0)];
    return s - (s / G) * G;
  };
  // Resources end at the block's last element (row rows-1, column K-1 of A;
  // row K-1, column N-1 of B), so nothing past the operands is read.
  auto a_src = [&](int r, int64_t k0) __attribute__((always_inline)) {
    const int64_t rows = p.M - r * Mb < Mb ? p.M - r * Mb : Mb;
    return rsrc(p.A + r * Mb * lda + k0, rows > 0 ? ((rows - 1) * lda + K - k0) * 4 : 0);
  };
  auto b_src = [&](int c, int64_t k0) __attribute__((always_inline)) {
    return rsrc(p.B + k0 * ldb + c * Nb, ((K - 1 - k0) * ldb + p.N - c * Nb) * 4);
  };
  auto load = [&](int v) __attribute__((always_inline)) {
    const int pass = v / nk;
    const int64_t k0 = (int64_t)(v - pass * nk) * BK;
    const int na = n_a(), nb = n_b();
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      if (m < na) {
        const auto r = a_src(a_blk(pass, m), k0);
#pragma unroll
        for (int i = 0; i < A_F4; ++i) {
          v4f x = bload(r, (uint32_t)(((m0 + a_row[i]) * lda + a_k[i]) * 4));
          if (m0 + a_row[i] >= Mb || k0 + a_k[i] >= K) x = v4f{0.f, 0.f, 0.f, 0.f};
          pa[m][i] = x;
        }
      }
      if (m < nb) {
        const auto r = b_src(b_blk(pass, m), k0);
#pragma unroll
        for (int i = 0; i < B_F4; ++i)
          pb[m][i] = bload(r, (uint32_t)((b_k[i] * ldb + n0 + b_n[i]) * 4));
      }
    }
  };
  auto store = [&](int buf, int v) __attribute__((always_inline)) {
    const int pass = v / nk;
    const int64_t k0 = (int64_t)(v - pass * nk) * BK;
    const int na = n_a(), nb = n_b();
    float* As = As0 + buf * A_SIZE;
    float* Bs = Bs0 + buf * B_SIZE;
#pragma unroll
    for (int i = 0; i < A_F4; ++i) {
      v4f sum = pa[0][i];
#pragma unroll
      for (int m = 1; m < kPre; ++m)
        if (m < na) sum += pa[m][i];
      for (int m = kPre; m < na; ++m) {  // blocks beyond the prefetch depth
        v4f x = bload(a_src(a_blk(pass, m), k0), (uint32_t)(((m0 + a_row[i]) * lda + a_k[i]) * 4));
        if (m0 + a_row[i] >= Mb || k0 + a_k[i] >= K) x = v4f{0.f, 0.f, 0.f, 0.f};
        sum += x;
      }
      *reinterpret_cast<v4f*>(As + a_row[i] * LDA_S + a_k[i]) = sum;
    }
#pragma unroll
    for (int i = 0; i < B_F4; ++i) {
      v4f sum = pb[0][i];
#pragma unroll
      for (int m = 1; m < kPre; ++m)
        if (m < nb) sum += pb[m][i];
      for (int m = kPre; m < nb; ++m)
        sum += bload(b_src(b_blk(pass, m), k0), (uint32_t)((b_k[i] * ldb + n0 + b_n[i]) * 4));
      *reinterpret_cast<v4f*>(Bs + b_k[i] * LDB_S + b_n[i]) = sum;
    }
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](int buf) __attribute__((always_inline)) {
    const float* As = As0 + buf * A_SIZE;
    const float* Bs = Bs0 + buf * B_SIZE;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      v4f a[FM], b[FN / 4][4];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const v4f*>(As + (wm * TM + i * 16 + c16) * LDA_S + kk + 4 * q);
#pragma unroll
      for (int jg = 0; jg < FN / 4; ++jg)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          b[jg][t] = *reinterpret_cast<const v4f*>(Bs + (kk + 4 * q + t) * LDB_S + wn * TN +
                                                   jg * 64 + 4 * c16);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j / 4][t][j % 4],
                                                             acc[i][j], 0, 0, 0);
    }
  };

  const int nv = npass * nk;  // K-slices over all passes
  load(0);
  store(0, 0);
  __syncthreads();
  for (int v = 0; v < nv; ++v) {
    const bool more = v + 1 < nv;
    if (more) load(v + 1);
    compute(v & 1);
    if (more) store((v + 1) & 1, v + 1);
    __syncthreads();
  }

  float* out;
  int64_t ldo, rows, cols = Nb;
  if (dest >= 0) {
    out = p.Y + (int64_t)dest * Mb * Nb;
    ldo = Nb;
    rows = Mb;
  } else {
    const int s = -1 - dest;
    const int64_t br = s / G, bc = s - br * G;
    out = p.C + br * Mb * p.ldc + bc * Nb;
    ldo = p.ldc;
    rows = p.M - br * Mb < Mb ? p.M - br * Mb : Mb;
  }
  const bool vec_ok = (ldo & 3) == 0;
#pragma unroll
  for (int jg = 0; jg < FN / 4; ++jg) {
    const int64_t col = n0 + wn * TN + jg * 64 + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * TM + i * 16 + 4 * q + r;
        if (row >= rows) continue;
        float* dst = out + row * ldo + col;
        const v4f v = {acc[i][4 * jg + 0][r], acc[i][4 * jg + 1][r], acc[i][4 * jg + 2][r],
                       acc[i][4 * jg + 3][r]};
        if (col + 3 < cols && vec_ok) {
          *reinterpret_cast<v4f*>(dst) = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < cols) dst[e] = v[e];
        }
      }
  }
}

}  // namespace

hipError_t launch_coded_gemm_2d(const GemmParams& p0, hipStream_t stream) {
  GemmParams p = p0;
  // buffer ranges and offsets are 32-bit
  const int64_t lim = (int64_t)1 << 31;
  if ((p.Mb + BM) * p.lda * 4 >= lim || p.K * p.ldb * 4 >= lim) return hipErrorInvalidValue;
  p.tiles_m = (int32_t)((p.Mb + BM - 1) / BM);
  p.tiles_n = (int32_t)((p.Nb + BN - 1) / BN);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(coded_gemm_2d_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
