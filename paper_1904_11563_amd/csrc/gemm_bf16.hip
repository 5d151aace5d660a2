// Coded GEMM in BF16 and split-BF16x3 on MFMA (v_mfma_f32_16x16x32_bf16),
// FP32 accumulation, encode fused into the A-operand load.
//
// The coded block C_g = sum of its data blocks A_s (Sec. II, XOR read as a
// real sum) is summed in FP32 registers while the A tile is staged, then
// rounded to BF16 (round to nearest even): hi = bf16(x), lo = bf16(x - hi).
// B is split the same way once per call by split_b_kernel into transposed
// planes Bt_hi, Bt_lo (N x Kp, k contiguous, zero past K) in the workspace.
//   BF16:   Y += A_hi . B_hi
//   BF16x3: Y += A_lo . B_hi + A_hi . B_lo + A_hi . B_hi, the two small
//           products of each 32-wide k step accumulated first.
//
// MFMA operands: lane (q = lane/16, c = lane%16) supplies row c of A and
// column c of B, eight consecutive k values each (k = 8q .. 8q+7 of the
// step); the same k assignment on both sides makes the contraction exact
// whatever order the unit sums in.  In the per-symbol tiles output columns
// are interleaved as in the FP32 kernel (subtile j, column c -> 4c + j) for
// float4 stores; the flat tiles below keep them in order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef unsigned short us;

constexpr int kThreads = 256;
constexpr int kPre = 4;
constexpr int BK = 32;
constexpr int KS = BK + 8;  // LDS row stride in bf16 (80 bytes)

__device__ __forceinline__ v4bf to_bf16(v4f x) {
  v4bf r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r[e] = (__bf16)x[e];
  return r;
}
__device__ __forceinline__ v4f from_bf16(v4bf x) {
  v4f r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r[e] = (float)x[e];
  return r;
}

// ------------------------------------------------------------- B split ---
// Bt_hi[n][k] = bf16(B[k][n]); Bt_lo[n][k] = bf16(B[k][n] - Bt_hi[n][k]);
// k in [K, Kp) is zero.  64 x 64 tiles transposed through LDS.
//
// LDS rows of 64 floats, unpadded, with the columns of k-row r stored at
// n ^ tsw(r).  The staging writes are 128-bit (8 consecutive lanes per
// 32-bank pass on gfx950: 8 distinct 16-byte slots of one row) and the
// transposed reads 32-bit (32 lanes per 32-bank pass: lanes of one pass read
// column nl of rows 16 a + j for a = 0..3, which the swizzle spreads over
// four distinct 8-bank groups).  Rows padded to 65 floats left both sides
// with 2-way conflicts.
__device__ __forceinline__ int tsw(int r) { return ((r >> 4) & 3) << 3; }

// Needs B 16-byte aligned, ldb a multiple of 4 and Kp a multiple of 16 (the
// library's argument checks and plan shapes guarantee all three).
__device__ __forceinline__ void split_b_tile(const float* B, int64_t ldb, int64_t K, int64_t N,
                                             int64_t Kp, us* bt_hi, us* bt_lo, int64_t k0,
                                             int64_t n0, float* t) {
  const int tid = threadIdx.x;
  // read: thread owns float4 (row kr, columns nc .. nc+3), four rows apart
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int f = tid + 256 * i;
    const int kr = f >> 4, nc = (f & 15) * 4;
    const int64_t k = k0 + kr, n = n0 + nc;
    v4f v = {0.f, 0.f, 0.f, 0.f};
    if (k < K) {
      const float* src = B + k * ldb + n;
      if (n + 3 < N) {
        v = *reinterpret_cast<const v4f*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < N) v[e] = src[e];
      }
    }
    *reinterpret_cast<v4f*>(t + kr * 64 + (nc ^ tsw(kr))) = v;
  }
  __syncthreads();
  // write: thread owns output row n = tid / 4, k kq .. kq+15 (two 16-byte
  // pieces per plane)
  const int nl = tid >> 2, kq = (tid & 3) * 16;
  const int64_t n = n0 + nl, k = k0 + kq;
  if (n >= N || k >= Kp) return;
  unsigned hw[8], lw[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int r = kq + 2 * j;  // rows r, r + 1 share the swizzle
    const float x0 = t[r * 64 + (nl ^ tsw(r))], x1 = t[(r + 1) * 64 + (nl ^ tsw(r))];
    const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
    const __bf16 l0 = (__bf16)(x0 - (float)h0), l1 = (__bf16)(x1 - (float)h1);
    hw[j] = (unsigned)__builtin_bit_cast(us, h0) | ((unsigned)__builtin_bit_cast(us, h1) << 16);
    lw[j] = (unsigned)__builtin_bit_cast(us, l0) | ((unsigned)__builtin_bit_cast(us, l1) << 16);
  }
  uint4* hp = reinterpret_cast<uint4*>(bt_hi + n * Kp + k);
  hp[0] = uint4{hw[0], hw[1], hw[2], hw[3]};
  hp[1] = uint4{hw[4], hw[5], hw[6], hw[7]};
  if (bt_lo) {
    uint4* lp = reinterpret_cast<uint4*>(bt_lo + n * Kp + k);
    lp[0] = uint4{lw[0], lw[1], lw[2], lw[3]};
    lp[1] = uint4{lw[4], lw[5], lw[6], lw[7]};
  }
}

__global__ __launch_bounds__(256) void split_b_kernel(const float* B, int64_t ldb, int64_t K,
                                                      int64_t N, int64_t Kp, us* bt_hi, us* bt_lo) {
  __shared__ __attribute__((aligned(16))) float t[64 * 64];
  split_b_tile(B, ldb, K, N, Kp, bt_hi, bt_lo, (int64_t)blockIdx.y * 64,
               (int64_t)blockIdx.x * 64, t);
}

// -------------------------------------------------------------- GEMM ---
template <int BM, int BN>
struct Bf16Tile {
  static constexpr int TM = BM / 2, TN = BN / 2;
  static constexpr int FM = TM / 16, FN = TN / 16;
  static constexpr int A_F4 = BM * BK / 4 / kThreads;     // fp32 float4 per thread
  static constexpr int B_CH = BN * BK * 2 / 16 / kThreads;  // 16-byte chunks per plane
  static constexpr int A_PLANE = BM * KS;                   // bf16 elements
  static constexpr int B_PLANE = BN * KS;
  static_assert(A_F4 >= 1 && B_CH >= 1 && FN % 4 == 0, "tile shape");
};

__device__ __forceinline__ int xcd_remap(int lin, int total) {
  if ((total & 7) != 0) return lin;
  return (lin & 7) * (total >> 3) + (lin >> 3);
}

template <int BM, int BN, int SPLIT>
__device__ __forceinline__ void bf16_tile(const GemmParams& p, int si, int mt, int nt,
                                          us* lds) {
  using T = Bf16Tile<BM, BN>;
  constexpr int NPL = SPLIT == 3 ? 2 : 1;  // planes per operand
  constexpr int STAGE = NPL * (T::A_PLANE + T::B_PLANE);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = lane >> 4, c16 = lane & 15;
  const int m0 = mt * BM, n0 = nt * BN;

  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;
  const int64_t K = p.K, N = p.N, Mb = p.Mb, M = p.M, Kp = p.kp;

  int a_row[T::A_F4], a_kc[T::A_F4];
  uint32_t a_off[T::A_F4];
#pragma unroll
  for (int i = 0; i < T::A_F4; ++i) {
    const int f = tid + kThreads * i;
    a_row[i] = f / (BK / 4);
    a_kc[i] = (f % (BK / 4)) * 4;
    a_off[i] = (uint32_t)((m0 + a_row[i]) * (int)p.lda + a_kc[i]) * 4u;
  }
  // B chunks: chunk f -> row n = f / 4 of the tile, k offset (f % 4) * 8
  int b_n[T::B_CH], b_kc[T::B_CH];
#pragma unroll
  for (int i = 0; i < T::B_CH; ++i) {
    const int f = tid + kThreads * i;
    b_n[i] = f / 4;
    b_kc[i] = (f % 4) * 8;
  }
  const char* mbase[kPre];
#pragma unroll
  for (int m = 0; m < kPre; ++m)
    mbase[m] = reinterpret_cast<const char*>(p.A + (m < deg ? (int64_t)ids[m] * Mb * p.lda : 0));
  const int64_t s_last = deg > 0 ? ids[deg - 1] : 0;
  const bool rows_full = m0 + BM <= Mb && s_last * Mb + m0 + BM <= M;

  auto a_valid = [&](int member, int i) __attribute__((always_inline)) -> bool {
    const int64_t rb = m0 + a_row[i];
    return rb < Mb && (int64_t)ids[member] * Mb + rb < M;
  };

  v4f pre[kPre][T::A_F4];
  uint4 bre[NPL][T::B_CH];

  auto load = [&](int k0) __attribute__((always_inline)) {
    if (rows_full && k0 + BK <= K) {
#pragma unroll
      for (int mbr = 0; mbr < kPre; ++mbr)
        if (mbr < deg) {
#pragma unroll
          for (int i = 0; i < T::A_F4; ++i)
            pre[mbr][i] = *reinterpret_cast<const v4f*>(mbase[mbr] + a_off[i] + k0 * 4u);
        }
    } else {
#pragma unroll
      for (int mbr = 0; mbr < kPre; ++mbr)
        if (mbr < deg) {
#pragma unroll
          for (int i = 0; i < T::A_F4; ++i) {
            v4f v = {0.f, 0.f, 0.f, 0.f};
            if (a_valid(mbr, i) && k0 + a_kc[i] < K)
              v = *reinterpret_cast<const v4f*>(mbase[mbr] + a_off[i] + k0 * 4u);
            pre[mbr][i] = v;
          }
        }
    }
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
      const us* bt = pl == 0 ? p.bt_hi : p.bt_lo;
#pragma unroll
      for (int i = 0; i < T::B_CH; ++i) {
        const int64_t n = n0 + b_n[i];
        uint4 v = {0u, 0u, 0u, 0u};
        if (n < N) v = *reinterpret_cast<const uint4*>(bt + n * Kp + k0 + b_kc[i]);
        bre[pl][i] = v;
      }
    }
  };
  auto store = [&](int buf, int k0) __attribute__((always_inline)) {
    us* st = lds + buf * STAGE;
    us* As_hi = st;
    us* As_lo = st + T::A_PLANE;
    us* Bs = st + NPL * T::A_PLANE;
#pragma unroll
    for (int i = 0; i < T::A_F4; ++i) {
      v4f sum = pre[0][i];
#pragma unroll
      for (int mbr = 1; mbr < kPre; ++mbr)
        if (mbr < deg) sum += pre[mbr][i];
      for (int mbr = kPre; mbr < deg; ++mbr) {
        if (a_valid(mbr, i) && k0 + a_kc[i] < K)
          sum += *reinterpret_cast<const v4f*>(p.A + (int64_t)ids[mbr] * Mb * p.lda +
                                               a_off[i] / 4u + k0);
      }
      const v4bf hi = to_bf16(sum);
      *reinterpret_cast<v4bf*>(As_hi + a_row[i] * KS + a_kc[i]) = hi;
      if (SPLIT == 3)
        *reinterpret_cast<v4bf*>(As_lo + a_row[i] * KS + a_kc[i]) = to_bf16(sum - from_bf16(hi));
    }
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
      for (int i = 0; i < T::B_CH; ++i)
        *reinterpret_cast<uint4*>(Bs + pl * T::B_PLANE + b_n[i] * KS + b_kc[i]) = bre[pl][i];
  };

  v4f acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](int buf) __attribute__((always_inline)) {
    const us* st = lds + buf * STAGE;
    const us* As_hi = st;
    const us* As_lo = st + T::A_PLANE;
    const us* Bs_hi = st + NPL * T::A_PLANE;
    const us* Bs_lo = Bs_hi + T::B_PLANE;
    v8bf ah[T::FM], al[T::FM], bh[T::FN], bl[T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i) {
      const int r = wm * T::TM + i * 16 + c16;
      ah[i] = *reinterpret_cast<const v8bf*>(As_hi + r * KS + 8 * q);
      if (SPLIT == 3) al[i] = *reinterpret_cast<const v8bf*>(As_lo + r * KS + 8 * q);
    }
#pragma unroll
    for (int j = 0; j < T::FN; ++j) {
      const int n = wn * T::TN + (j / 4) * 64 + 4 * c16 + (j % 4);
      bh[j] = *reinterpret_cast<const v8bf*>(Bs_hi + n * KS + 8 * q);
      if (SPLIT == 3) bl[j] = *reinterpret_cast<const v8bf*>(Bs_lo + n * KS + 8 * q);
    }
    if (SPLIT == 3) {
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
  };

  const int nk = (int)((K + BK - 1) / BK);
  load(0);
  store(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const bool more = kt + 1 < nk;
    if (more) load((kt + 1) * BK);
    compute(kt & 1);
    if (more) store((kt + 1) & 1, (kt + 1) * BK);
    __syncthreads();
  }

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
  const bool vec_ok = (ldo & 3) == 0;
#pragma unroll
  for (int jg = 0; jg < T::FN / 4; ++jg) {
    const int64_t col = n0 + wn * T::TN + jg * 64 + 4 * c16;
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * T::TM + i * 16 + 4 * q + r;
        if (row >= rows) continue;
        float* dst = out + row * ldo + col;
        const v4f v = {acc[i][4 * jg + 0][r], acc[i][4 * jg + 1][r], acc[i][4 * jg + 2][r],
                       acc[i][4 * jg + 3][r]};
        if (col + 3 < N && vec_ok) {
          *reinterpret_cast<v4f*>(dst) = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < N) dst[e] = v[e];
        }
      }
  }
}

// ------------------------------------------------------------ flat tile --
// The computed symbols' coded blocks, stacked, are one R x K matrix
// (R = n_sym * Mb) whose row gr belongs to symbol gr / Mb; one R x N x K
// product covers them all, so 128-row tiles span symbol boundaries and
// small blocks waste no rows.  Each thread looks up the symbol and member
// rows of the two A rows it stages; the encode sums the members in FP32 and
// splits the sum into BF16 hi / lo while staging.  8 waves (2 x 4) of
// 64 x 64, K-stages of 32, LDS double buffer: during the current stage's
// MFMAs the next stage's A loads land in registers and its B loads go
// straight to LDS.  Rows past a product's end come back as zeros from the
// buffer resource's range check.
// Needs K a multiple of 32.  Output columns are not interleaved here (B is
// stored n-major, and interleaved columns would read rows four apart, which
// no row swizzle spreads over the banks).
namespace flat {
constexpr int BM = 128, BN = 256, NT = 512;
constexpr int TM = 64, TN = 64, FM = 4, FN = 4;  // wave tile (2 x 4 waves)
constexpr int FKS = BK;  // LDS row: 32 bf16 = four 16-byte granules, no padding
// Granule g of row r sits in slot g ^ ((r >> 1) & 2).  gfx950 serves a
// 128-bit LDS read to 16 lanes at a time over 64 banks, the 16 being the
// lanes that agree in lane bit 5 and in the parity of lane bits 2..4, and a
// 128-bit write to 8 consecutive lanes over 32 banks.  A fragment read
// (lane 16 q + c: row c, granule q) then puts each such group of 16 on
// distinct bank quads, and a B store (4 lanes per row) each group of 8; the
// swizzle g ^ ((r >> 2) & 3) left two lanes on a quad in every read.
__device__ __forceinline__ int swz(int row, int granule) {
  return row * FKS + ((granule ^ ((row >> 1) & 2)) << 3);
}
constexpr int A_PLANE = BM * FKS, B_PLANE = BN * FKS;
constexpr int UA = BM * BK / 4 / NT;        // float4 of A per thread per member (2)
constexpr int UB = BN * BK * 2 / 16 / NT;   // 16-byte B chunks per thread per plane (2)
constexpr int kRsrcWord3 = 0x00020000;      // gfx9 raw buffer, 32-bit elements

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           (int)(bytes > 0 ? bytes : 0), kRsrcWord3);
}
__device__ __forceinline__ v4f bload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

// A's two stages in one array; B's stages in one array each, since they are
// filled by direct loads to LDS, and the compiler then sees that the stage
// being filled is not the one being read (no wait on those loads there).
template <int SPLIT>
constexpr int a_elems() {
  return 2 * (SPLIT == 3 ? 2 : 1) * A_PLANE;
}
template <int SPLIT>
constexpr int b_elems() {
  return (SPLIT == 3 ? 2 : 1) * B_PLANE;
}
typedef __attribute__((address_space(3))) void* lds_addr;
}  // namespace flat

// The grouped kernel reaches a product's tables and outputs through
// pointers read from its descriptor, which the compiler would access with
// flat instructions; those also count on the LDS counter, so the next
// tile's first LDS wait would wait for this tile's output stores.  They
// are device memory: read and written as global.
__device__ __forceinline__ int32_t gld(const int32_t* ptr) {
  return *(const __attribute__((address_space(1))) int32_t*)ptr;
}
__device__ __forceinline__ void gst(float* ptr, float v) {
  *(__attribute__((address_space(1))) float*)ptr = v;
}

template <int SPLIT>
__device__ __forceinline__ void bf16_flat_tile(const GemmParams& p, int mt, int nt, us* lds_a,
                                               us* lds_b0, us* lds_b1) {
  using namespace flat;
  constexpr int NPL = SPLIT == 3 ? 2 : 1;
  constexpr int A_STAGE = NPL * A_PLANE;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int64_t Mb = p.Mb, M = p.M, N = p.N, K = p.K, Kp = p.kp, lda = p.lda;
  const int64_t R = (int64_t)p.n_sym * Mb;

  // A: rows ar + 64 u of the tile, k ak .. ak+3 of the stage.  The rows of
  // one wave can belong to symbols of different degrees.  The wave loads
  // member m of its rows if any of them has one (a uniform branch, bit m of
  // need), and a row without it gets the offset M lda, past the resource's
  // range for every stage, whose load returns zeros: no per-lane branches.
  const int ar = tid >> 3, ak = (tid & 7) * 4;
  const uint32_t absent = (uint32_t)(M * lda * 4);
  uint32_t off[UA][kPre];
  int deg_u[UA], idoff_u[UA], lr_u[UA];
#pragma unroll
  for (int u = 0; u < UA; ++u) {
    const int64_t gr = m0 + ar + 64 * u;
    int deg = 0, id_off = 0;
    int64_t lr = 0;
    if (gr < R) {
      const int64_t si = gr / Mb;
      lr = gr - si * Mb;
      id_off = gld(p.syms + 4 * si + 0);
      deg = gld(p.syms + 4 * si + 1);
    }
    deg_u[u] = deg;
    idoff_u[u] = id_off;
    lr_u[u] = (int)lr;
#pragma unroll
    for (int m = 0; m < kPre; ++m)
      off[u][m] = m < deg ? (uint32_t)((((int64_t)gld(p.ids + id_off + m) * Mb + lr) * lda + ak) * 4)
                          : absent;
  }
  // B is staged by direct loads to LDS: one instruction of a wave fills 64
  // consecutive 16-byte LDS slots, lane l the slot base + 16 l, from the
  // lane's own global address.  Instruction c of wave w fills tile rows
  // 16 (w + 8 c) + l / 4, slot l % 4, which holds granule
  // (l % 4) ^ ((l >> 3) & 2) of that row (the swizzle above, the base row
  // being a multiple of 16).  Rows past N are out of the resource's range;
  // they only feed output columns that are never stored.
  uint32_t boff[UB];
  {
    const int gb = (lane & 3) ^ ((lane >> 3) & 2);
#pragma unroll
    for (int c = 0; c < UB; ++c)
      boff[c] = (uint32_t)(((16 * (wave + 8 * c) + (lane >> 2)) * Kp + gb * 8) * 2);
  }
  static_assert(UB * 8 * 16 == BN, "B staging covers the tile");

  int dmax = 0;
#pragma unroll
  for (int u = 0; u < UA; ++u) dmax = deg_u[u] > dmax ? deg_u[u] : dmax;
  uint32_t need = 1;  // member 0 is always loaded (zeros for rows past the end)
#pragma unroll
  for (int m = 1; m < kPre; ++m)
    if (__builtin_amdgcn_ballot_w64(m < dmax) != 0) need |= 1u << m;

  // a member the wave skips keeps these zeros for the whole tile
  v4f preA[kPre][UA];
#pragma unroll
  for (int m = 0; m < kPre; ++m)
#pragma unroll
    for (int u = 0; u < UA; ++u) preA[m][u] = v4f{0.f, 0.f, 0.f, 0.f};
  auto dma_b = [&](us* bst, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
      const auto rb = rsrc((pl == 0 ? p.bt_hi : p.bt_lo) + n0 * Kp + k0, ((N - n0) * Kp - k0) * 2);
#pragma unroll
      for (int c = 0; c < UB; ++c)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rb, (lds_addr)(bst + pl * B_PLANE + 16 * (wave + 8 * c) * FKS), 16, boff[c], 0, 0, 0);
    }
  };
  auto load = [&](v4f (&pre)[kPre][UA], int k0) __attribute__((always_inline)) {
    const auto ra = rsrc(p.A + k0, (M * lda - k0) * 4);
#pragma unroll
    for (int u = 0; u < UA; ++u)
#pragma unroll
      for (int m = 0; m < kPre; ++m)
        if ((need >> m) & 1) pre[m][u] = bload(ra, off[u][m]);
  };
  auto store = [&](v4f (&pre)[kPre][UA], us* st, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      v4f sum = pre[0][u];
#pragma unroll
      for (int m = 1; m < kPre; ++m) sum += pre[m][u];
      for (int m = kPre; m < deg_u[u]; ++m) {  // members beyond the prefetch depth
        const int64_t row = (int64_t)gld(p.ids + idoff_u[u] + m) * Mb + lr_u[u];
        if (row < M)
          sum += *(const __attribute__((address_space(1))) v4f*)(p.A + row * lda + k0 + ak);
      }
      const v4bf hi = to_bf16(sum);
      const int ao = swz(ar + 64 * u, ak >> 3) + (ak & 7);
      *reinterpret_cast<v4bf*>(st + ao) = hi;
      if (SPLIT == 3) *reinterpret_cast<v4bf*>(st + A_PLANE + ao) = to_bf16(sum - from_bf16(hi));
    }
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](const us* st, const us* Bs) __attribute__((always_inline)) {
    v8bf ah[FM], al[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = wm * TM + i * 16 + c16;
      ah[i] = *reinterpret_cast<const v8bf*>(st + swz(r, q));
      if (SPLIT == 3) al[i] = *reinterpret_cast<const v8bf*>(st + A_PLANE + swz(r, q));
    }
    // one output column group at a time keeps two B fragments live; MFMA
    // column c16 of subtile j is output column 16 j + c16, so the 16 lanes
    // of a k group read 16 consecutive B rows
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = wn * TN + 16 * j + c16;
      const v8bf bh = *reinterpret_cast<const v8bf*>(Bs + swz(n, q));
      if (SPLIT == 3) {
        const v8bf bl = *reinterpret_cast<const v8bf*>(Bs + B_PLANE + swz(n, q));
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
    }
  };

  // Stage kt sits in A stage kt & 1 and B array kt & 1.  The next stage's
  // A loads are issued before its B loads, so the A store waits on the A
  // loads only; each stage ends with all of this wave's loads done and a
  // barrier, so every wave's part of the next stage is in LDS before any
  // wave reads it, and a stage is refilled only after that barrier.
  auto step = [&](int kt, us* a_cur, us* a_nxt, const us* b_cur, us* b_nxt, int nk)
                  __attribute__((always_inline)) {
    const bool more = kt + 1 < nk;
    if (more) {
      load(preA, (kt + 1) * BK);
      dma_b(b_nxt, (kt + 1) * BK);
    }
    compute(a_cur, b_cur);
    if (more) store(preA, a_nxt, (kt + 1) * BK);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  const int nk = (int)(K / BK);
  load(preA, 0);
  dma_b(lds_b0, 0);
  store(preA, lds_a, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    step(kt, lds_a, lds_a + A_STAGE, lds_b0, lds_b1, nk);
    if (kt + 1 < nk) step(kt + 1, lds_a + A_STAGE, lds_a, lds_b1, lds_b0, nk);
  }

  // epilogue: lane holds rows 4q .. 4q+3 of column 16 j + c16 of each subtile
  const int64_t col0 = n0 + wn * TN + c16;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gr = m0 + wm * TM + i * 16 + 4 * q + r;
      if (gr >= R) continue;
      const int64_t si = gr / Mb;
      const int64_t lr = gr - si * Mb;
      const int dest = gld(p.syms + 4 * si + 2);
      float* dst;
      if (dest >= 0) {
        dst = p.Y + ((int64_t)dest * Mb + lr) * N + col0;
      } else {
        const int64_t row = (-1 - (int64_t)dest) * Mb + lr;
        if (row >= M) continue;
        dst = p.C + row * p.ldc + col0;
      }
#pragma unroll
      for (int j = 0; j < FN; ++j)
        if (col0 + 16 * j < N) gst(dst + 16 * j, acc[i][j][r]);
    }
}

template <int SPLIT>
__global__ __launch_bounds__(flat::NT, 1) void coded_gemm_bf16_flat_kernel(GemmParams p) {
  __shared__ __attribute__((aligned(16))) us lds_a[flat::a_elems<SPLIT>()];
  __shared__ __attribute__((aligned(16))) us lds_b0[flat::b_elems<SPLIT>()];
  __shared__ __attribute__((aligned(16))) us lds_b1[flat::b_elems<SPLIT>()];
  // Each XCD takes a contiguous range of tile indices, and consecutive
  // indices walk down groups of 8 row panels, column panel by column panel,
  // so the tiles an XCD runs together share their A rows and B columns in
  // its L2.
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  constexpr int kRowGroup = 8;
  const int per_group = kRowGroup * p.tiles_n;
  const int first = L / per_group * kRowGroup;
  const int rows = p.tiles_m - first < kRowGroup ? p.tiles_m - first : kRowGroup;
  const int r = L - (first / kRowGroup) * per_group;
  bf16_flat_tile<SPLIT>(p, first + r % rows, r / rows, lds_a, lds_b0, lds_b1);
}

// Persistent grouped form of the flat tile (GroupTile.lin = mt * tiles_n + nt).
template <int SPLIT>
__global__ __launch_bounds__(flat::NT, 1) void gemm_bf16_flat_grouped_kernel(
    const GroupDesc* __restrict__ d, const GroupTile* __restrict__ tiles, int32_t n_tiles) {
  __shared__ __attribute__((aligned(16))) us lds_a[flat::a_elems<SPLIT>()];
  __shared__ __attribute__((aligned(16))) us lds_b0[flat::b_elems<SPLIT>()];
  __shared__ __attribute__((aligned(16))) us lds_b1[flat::b_elems<SPLIT>()];
  // Each XCD takes a contiguous run of every grid-sized slice of the list,
  // so the tiles of one product (adjacent in the list) share an L2.
  const int slot = xcd_remap(blockIdx.x, gridDim.x);
  for (int t = slot; t < n_tiles; t += gridDim.x) {
    // uniform by construction; readfirstlane lets the compiler keep the
    // descriptor in scalar registers (copied, not re-read after stores)
    const int prod = __builtin_amdgcn_readfirstlane(tiles[t].prod);
    const int lin = __builtin_amdgcn_readfirstlane(tiles[t].lin);
    const GemmParams p = d[prod].g;
    const int mt = lin / p.tiles_n;
    bf16_flat_tile<SPLIT>(p, mt, lin - mt * p.tiles_n, lds_a, lds_b0, lds_b1);
  }
}

template <int BM, int BN, int SPLIT>
constexpr int bf16_lds_elems() {
  using T = Bf16Tile<BM, BN>;
  return 2 * (SPLIT == 3 ? 2 : 1) * (T::A_PLANE + T::B_PLANE);
}

template <int BM, int BN, int SPLIT, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void coded_gemm_bf16_kernel(GemmParams p) {
  __shared__ __attribute__((aligned(16))) us lds[bf16_lds_elems<BM, BN, SPLIT>()];
  // Row panels of all symbols in one sequence (every symbol multiplies the
  // same B), walked in groups of 8, column panel by column panel, as in the
  // flat kernel.
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  constexpr int kRowGroup = 8;
  const int panels = p.n_sym * p.tiles_m;
  const int per_group = kRowGroup * p.tiles_n;
  const int first = L / per_group * kRowGroup;
  const int rows = panels - first < kRowGroup ? panels - first : kRowGroup;
  const int r = L - (first / kRowGroup) * per_group;
  const int rp = first + r % rows;
  const int si = rp / p.tiles_m;
  bf16_tile<BM, BN, SPLIT>(p, si, rp - si * p.tiles_m, r / rows, lds);
}

// Grouped split-B: a flat range of 64 x 64 transpose blocks over products
// (bmap gives each block's product); float4 reads along n, 16-byte writes of
// eight bf16 along k.
__global__ __launch_bounds__(256) void split_b_grouped_kernel(const GroupDesc* d,
                                                              const int64_t* bstart,
                                                              const int32_t* bmap) {
  __shared__ __attribute__((aligned(16))) float t[64 * 64];
  const int64_t b = blockIdx.x;
  const int lo = bmap[b];
  const GroupDesc& g = d[lo];
  const int64_t r = b - bstart[lo];
  split_b_tile(g.g.B, g.g.ldb, g.g.K, g.g.N, g.g.kp, const_cast<us*>(g.g.bt_hi),
               const_cast<us*>(g.g.bt_lo), (r / g.b_tn) * 64, (r % g.b_tn) * 64, t);
}

// Persistent grouped GEMM: workgroup w takes tiles w, w + grid, w + 2 grid, ...
// of a list already ordered longest-K first.
template <int BM, int BN, int SPLIT>
__global__ __launch_bounds__(kThreads) void gemm_bf16_grouped_kernel(const GroupDesc* d,
                                                                     const GroupTile* tiles,
                                                                     int32_t n_tiles) {
  __shared__ __attribute__((aligned(16))) us lds[bf16_lds_elems<BM, BN, SPLIT>()];
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const GroupTile gt = tiles[t];
    const GemmParams& p = d[gt.prod].g;
    const int per_sym = p.tiles_m * p.tiles_n;
    const int si = gt.lin / per_sym;
    const int rem = gt.lin - si * per_sym;
    const int mt = rem / p.tiles_n;
    const int nt = rem - mt * p.tiles_n;
    bf16_tile<BM, BN, SPLIT>(p, si, mt, nt, lds);
  }
}

struct Bf16Entry {
  TileShape shape;
  void (*k1)(GemmParams);
  void (*k3)(GemmParams);
};
constexpr int32_t kBf16Flat = 4;

const Bf16Entry kBf16Tiles[] = {
    {{128, 128, 32}, coded_gemm_bf16_kernel<128, 128, 1, 2>, coded_gemm_bf16_kernel<128, 128, 3, 2>},
    {{64, 128, 32}, coded_gemm_bf16_kernel<64, 128, 1, 2>, coded_gemm_bf16_kernel<64, 128, 3, 2>},
    {{128, 256, 32}, coded_gemm_bf16_kernel<128, 256, 1, 1>, coded_gemm_bf16_kernel<128, 256, 3, 1>},
    {{64, 256, 32}, coded_gemm_bf16_kernel<64, 256, 1, 1>, coded_gemm_bf16_kernel<64, 256, 3, 1>},
    // flat rows over all symbols (tiles_m counts 128-row tiles of n_sym * Mb)
    {{128, 256, 32}, coded_gemm_bf16_flat_kernel<1>, coded_gemm_bf16_flat_kernel<3>},
};

}  // namespace

int32_t bf16_tile_count() { return (int32_t)(sizeof(kBf16Tiles) / sizeof(kBf16Tiles[0])); }
TileShape bf16_tile_shape(int32_t t) { return kBf16Tiles[t].shape; }
bool bf16_tile_is_flat(int32_t t) { return t == kBf16Flat; }

bool bf16_flat_ok(const GemmParams& p) {
  const int64_t lim = (int64_t)1 << 31;
  return p.K % 32 == 0 && p.kp == p.K && (p.M + p.Mb) * p.lda * 4 < lim &&
         p.N * p.kp * 2 < lim && (int64_t)p.n_sym * p.Mb < lim;
}

hipError_t launch_split_b(const float* B, int64_t ldb, int64_t K, int64_t N, int64_t Kp,
                          void* bt_hi, void* bt_lo, hipStream_t stream) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((Kp + 63) / 64));
  hipLaunchKernelGGL(split_b_kernel, grid, dim3(256), 0, stream, B, ldb, K, N, Kp,
                     static_cast<us*>(bt_hi), static_cast<us*>(bt_lo));
  return hipGetLastError();
}

hipError_t launch_split_b_grouped(const GroupDesc* d, const int64_t* bstart, const int32_t* bmap,
                                  int64_t total_blocks, hipStream_t stream) {
  if (total_blocks == 0) return hipSuccess;
  if (total_blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_b_grouped_kernel, dim3((unsigned)total_blocks), dim3(256), 0, stream,
                     d, bstart, bmap);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_grouped(const GroupDesc* d, const GroupTile* tiles, int32_t n_tiles,
                                    int32_t tile, int32_t split, int32_t grid,
                                    hipStream_t stream) {
  if (n_tiles == 0) return hipSuccess;
  if (tile == kBf16Flat) {
    if (split == 3)
      hipLaunchKernelGGL(gemm_bf16_flat_grouped_kernel<3>, dim3((unsigned)grid), dim3(flat::NT),
                         0, stream, d, tiles, n_tiles);
    else
      hipLaunchKernelGGL(gemm_bf16_flat_grouped_kernel<1>, dim3((unsigned)grid), dim3(flat::NT),
                         0, stream, d, tiles, n_tiles);
    return hipGetLastError();
  }
  void (*k)(const GroupDesc*, const GroupTile*, int32_t) = nullptr;
  switch (tile * 4 + split) {
    case 0 * 4 + 1: k = gemm_bf16_grouped_kernel<128, 128, 1>; break;
    case 0 * 4 + 3: k = gemm_bf16_grouped_kernel<128, 128, 3>; break;
    case 1 * 4 + 1: k = gemm_bf16_grouped_kernel<64, 128, 1>; break;
    case 1 * 4 + 3: k = gemm_bf16_grouped_kernel<64, 128, 3>; break;
    case 2 * 4 + 1: k = gemm_bf16_grouped_kernel<128, 256, 1>; break;
    case 2 * 4 + 3: k = gemm_bf16_grouped_kernel<128, 256, 3>; break;
    case 3 * 4 + 1: k = gemm_bf16_grouped_kernel<64, 256, 1>; break;
    case 3 * 4 + 3: k = gemm_bf16_grouped_kernel<64, 256, 3>; break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), 0, stream, d, tiles, n_tiles);
  return hipGetLastError();
}

hipError_t launch_coded_gemm_bf16(const GemmParams& p0, int32_t tile, hipStream_t stream) {
  GemmParams p = p0;
  if (tile == kBf16Flat) {
    if (bf16_flat_ok(p)) {
      p.tiles_m = (int32_t)(((int64_t)p.n_sym * p.Mb + flat::BM - 1) / flat::BM);
      p.tiles_n = (int32_t)((p.N + flat::BN - 1) / flat::BN);
      const int64_t blocks = (int64_t)p.tiles_m * p.tiles_n;
      if (blocks == 0) return hipSuccess;
      if (blocks > 0x7fffffff) return hipErrorInvalidValue;
      hipLaunchKernelGGL(p.prec == BPX_PREC_BF16X3 ? coded_gemm_bf16_flat_kernel<3>
                                                   : coded_gemm_bf16_flat_kernel<1>,
                         dim3((unsigned)blocks), dim3(flat::NT), 0, stream, p);
      return hipGetLastError();
    }
    tile = 1;  // K not a multiple of 32, or offsets past 31 bits
  }
  const Bf16Entry& e = kBf16Tiles[tile];
  p.tiles_m = (int32_t)((p.Mb + e.shape.bm - 1) / e.shape.bm);
  p.tiles_n = (int32_t)((p.N + e.shape.bn - 1) / e.shape.bn);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(p.prec == BPX_PREC_BF16X3 ? e.k3 : e.k1, dim3((unsigned)blocks),
                     dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
