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

// ------------------------------------------------------------ wide tile --
// The same products on 256 x 256 tiles (8 waves, 4 x 2, of 64 x 128), the
// tiling of the row-block FP32 kernel: K-slices of 32 in two 16-wide halves,
// each half's loads in registers during the other half's MFMAs, LDS double
// buffer with unpadded rows (A: 32 floats, 16-byte granule g of row r at
// slot g ^ ((r >> 1) & 7); B: 256 floats), on which gfx950's 128-bit LDS
// accesses are free of bank conflicts.  Per half-slice a thread stages two
// float4 of A and two of B, so one prefetch array holds the members of
// whichever operand the symbol sums (A blocks when they share a B block, B
// blocks when they share an A block, the pass's single member for gray
// symbols) and one more register set the other operand.  Needs full blocks:
// Mb and Nb multiples of 256, M = grid Mb, N = grid Nb, K a multiple of 32.
namespace w2d {
constexpr int BM = 256, BN = 256, BK = 32, WM = 4, WN = 2, NT = 64 * WM * WN;
constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 16, FN = TN / 16;
constexpr int U = (BM / 2) * BK / 4 / NT;  // float4 per thread per half, A and B alike (2)
constexpr int RA = NT / 8, RB = NT / 64;   // row step of a thread's A / B float4
constexpr int A_SIZE = BM * BK, B_SIZE = BK * BN;
static_assert(U == 2 && (BK / 2) * BN / 4 / NT == U && FN % 4 == 0 && RA % 16 == 0, "tile split");
__device__ __forceinline__ int a_slot(int row, int granule) { return granule ^ ((row >> 1) & 7); }
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_all(const float* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, -1, kRsrcWord3);
}
__device__ __forceinline__ v4f bload_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(v4f,
                            __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
}  // namespace w2d

__global__ __launch_bounds__(w2d::NT, 1) void coded_gemm_2d_wide_kernel(GemmParams p) {
  // local names shadow the 64 x 128 kernel's constants of the same names
  constexpr int BM = w2d::BM, BN = w2d::BN, BK = w2d::BK, WN = w2d::WN;
  constexpr int TM = w2d::TM, TN = w2d::TN, FM = w2d::FM, FN = w2d::FN, U = w2d::U;
  constexpr int RA = w2d::RA, RB = w2d::RB, A_SIZE = w2d::A_SIZE, B_SIZE = w2d::B_SIZE;
  using w2d::a_slot;
  using w2d::bload_s;
  using w2d::rsrc_all;
  __shared__ __attribute__((aligned(16))) float lds[2 * (A_SIZE + B_SIZE)];
  float* As0 = lds;
  float* Bs0 = lds + 2 * A_SIZE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int q = lane >> 4, c16 = lane & 15;

  // Tiles symbol-major in table order (the planner lists the symbols by
  // decreasing passes) with no XCD remapping: workgroups are dealt to the
  // XCDs round-robin, so every XCD gets its share of the longest tiles
  // first.  (Contiguous XCD ranges put all the gray symbols' tiles on a
  // few XCDs and left the others idle: 37.9 ms against 23.1 ms.)
  // Within a symbol, the tile dealt to XCD x as its u-th is the
  // (x per/8 + u)-th of the symbol's tiles in row-pair order (two row panels
  // at a time, walking the columns), so an XCD's tiles of a symbol form a
  // compact 2 x (per/16) block sharing A and B panels in its L2.
  const int per_sym = p.tiles_m * p.tiles_n;
  const int si = (int)blockIdx.x / per_sym;
  int rem = (int)blockIdx.x - si * per_sym;
  if ((per_sym & 7) == 0) rem = (rem & 7) * (per_sym >> 3) + (rem >> 3);
  int mt, nt;
  {
    const int pg = 2 * p.tiles_n;  // tiles per row pair
    const int g = rem / pg, first = 2 * g;
    const int gsz = p.tiles_m - first < 2 ? p.tiles_m - first : 2;
    const int r = rem - g * pg;
    mt = first + r % gsz;
    nt = r / gsz;
  }
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;
  const int G = p.grid;
  const int64_t Mb = p.Mb, Nb = p.Nb, lda = p.lda, ldb = p.ldb;

  // kind: 0 = members share the B block (sum A), 1 = share the A block (sum
  // B), 2 = gray (one pass per member)
  int kind;
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
  const int nk = (int)(p.K / BK);
  const int npre = kind == 2 ? 1 : deg;  // members of the summed operand

  // Half h of a slice: A rows 128 h + ar + RA u, k ak .. ak+3; B k-rows
  // 16 h + br + RB u, columns bc .. bc+3 (u < U).
  const int ar = tid >> 3, ak = (tid & 7) * 4;
  const int br = tid >> 6, bc = (tid & 63) * 4;
  const uint32_t a_off = (uint32_t)(((m0 + ar) * lda + ak) * 4);
  const uint32_t b_off = (uint32_t)((br * ldb + n0 + bc) * 4);
  const uint32_t a_row4 = (uint32_t)(lda * 4), b_row4 = (uint32_t)(ldb * 4);
  // Block bases: data block s is A row block s / G times B column block
  // s % G.  The summed operand's members (kinds 0 and 1) and the other
  // operand are fixed for the symbol; a gray symbol's pass takes both from
  // its own member.
  auto a_blk = [&](int s) __attribute__((always_inline)) -> const float* {
    return p.A + (int64_t)(s / G) * Mb * lda;
  };
  auto b_blk = [&](int s) __attribute__((always_inline)) -> const float* {
    return p.B + (int64_t)(s - (s / G) * G) * Nb;
  };
  const float* pbase[kPre];
#pragma unroll
  for (int m = 0; m < kPre; ++m) {
    const int s = ids[m < deg ? m : 0];
    pbase[m] = kind == 1 ? b_blk(s) : a_blk(s);
  }
  const float* sbase = kind == 1 ? a_blk(ids[0]) : b_blk(ids[0]);
  auto a_of = [&](int pass, int m) __attribute__((always_inline)) -> const float* {
    return kind == 2 ? a_blk(ids[pass]) : (kind == 0 ? (m < kPre ? pbase[m] : a_blk(ids[m])) : sbase);
  };
  auto b_of = [&](int pass, int m) __attribute__((always_inline)) -> const float* {
    return kind == 2 ? b_blk(ids[pass]) : (kind == 1 ? (m < kPre ? pbase[m] : b_blk(ids[m])) : sbase);
  };

  v4f pre[kPre][U];  // the summed operand's members (A for kinds 0 and 2, B for kind 1)
  v4f sgl[U];        // the other operand
  auto load_half = [&](int h, int v) __attribute__((always_inline)) {
    const int pass = v / nk;
    const int64_t k0 = (int64_t)(v - pass * nk) * BK;
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      if (m < npre) {
        if (kind == 1) {
          const auto r = rsrc_all(b_of(pass, m) + k0 * ldb);
#pragma unroll
          for (int u = 0; u < U; ++u) pre[m][u] = bload_s(r, b_off, (16 * h + RB * u) * b_row4);
        } else {
          const auto r = rsrc_all(a_of(pass, m) + k0);
#pragma unroll
          for (int u = 0; u < U; ++u) pre[m][u] = bload_s(r, a_off, (128 * h + RA * u) * a_row4);
        }
      }
    }
    if (kind == 1) {
      const auto r = rsrc_all(a_of(pass, 0) + k0);
#pragma unroll
      for (int u = 0; u < U; ++u) sgl[u] = bload_s(r, a_off, (128 * h + RA * u) * a_row4);
    } else {
      const auto r = rsrc_all(b_of(pass, 0) + k0 * ldb);
#pragma unroll
      for (int u = 0; u < U; ++u) sgl[u] = bload_s(r, b_off, (16 * h + RB * u) * b_row4);
    }
  };
  auto store_half = [&](int h, int buf, int v) __attribute__((always_inline)) {
    const int pass = v / nk;
    const int64_t k0 = (int64_t)(v - pass * nk) * BK;
    // rows ar + 128 h + RA u share the swizzle of row ar (RA is a multiple of 16)
    float* As = As0 + buf * A_SIZE + ar * BK + 4 * a_slot(ar, ak >> 2);
    float* Bs = Bs0 + buf * B_SIZE + br * BN + bc;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v4f sum = pre[0][u];
#pragma unroll
      for (int m = 1; m < kPre; ++m)
        if (m < npre) sum += pre[m][u];
      for (int m = kPre; m < npre; ++m) {  // members beyond the prefetch depth
        if (kind == 1)
          sum += bload_s(rsrc_all(b_of(pass, m) + k0 * ldb), b_off, (16 * h + RB * u) * b_row4);
        else
          sum += bload_s(rsrc_all(a_of(pass, m) + k0), a_off, (128 * h + RA * u) * a_row4);
      }
      const v4f av = kind == 1 ? sgl[u] : sum;
      const v4f bv = kind == 1 ? sum : sgl[u];
      *reinterpret_cast<v4f*>(As + (128 * h + RA * u) * BK) = av;
      *reinterpret_cast<v4f*>(Bs + (16 * h + RB * u) * BN) = bv;
    }
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute_chunk = [&](const float* As, const float* Bs, int kk) __attribute__((always_inline)) {
    v4f a[FM];
    v4f b[FN / 4][4];
    const float* Aw = As + (wm * TM + c16) * BK + 4 * a_slot(c16, (kk >> 2) + q);
    const float* Bw = Bs + (kk + 4 * q) * BN + wn * TN + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const v4f*>(Aw + i * 16 * BK);
#pragma unroll
    for (int jg = 0; jg < FN / 4; ++jg)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        b[jg][t] = *reinterpret_cast<const v4f*>(Bw + t * BN + jg * 64);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j / 4][t][j % 4],
                                                           acc[i][j], 0, 0, 0);
  };

  const int nv = npass * nk;  // K-slices over all passes
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    load_half(h, 0);
    store_half(h, 0, 0);
  }
  __syncthreads();
  for (int v = 0; v + 1 < nv; ++v) {
    const int buf = v & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      load_half(h, v + 1);
      compute_chunk(As0 + buf * A_SIZE, Bs0 + buf * B_SIZE, h * 16);
      store_half(h, buf ^ 1, v + 1);
    }
    __syncthreads();
  }
  {
    const int buf = (nv - 1) & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) compute_chunk(As0 + buf * A_SIZE, Bs0 + buf * B_SIZE, h * 16);
  }

  float* out;
  int64_t ldo;
  if (dest >= 0) {
    out = p.Y + (int64_t)dest * Mb * Nb;
    ldo = Nb;
  } else {
    const int s = -1 - dest;
    const int64_t bro = s / G, bco = s - bro * G;
    out = p.C + bro * Mb * p.ldc + bco * Nb;
    ldo = p.ldc;
  }
#pragma unroll
  for (int jg = 0; jg < FN / 4; ++jg) {
    const int64_t col = n0 + wn * TN + jg * 64 + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * TM + i * 16 + 4 * q + r;
        const v4f v = {acc[i][4 * jg + 0][r], acc[i][4 * jg + 1][r], acc[i][4 * jg + 2][r],
                       acc[i][4 * jg + 3][r]};
        *reinterpret_cast<v4f*>(out + row * ldo + col) = v;
      }
  }
}

}  // namespace

hipError_t launch_coded_gemm_2d(const GemmParams& p0, int32_t tile, hipStream_t stream) {
  GemmParams p = p0;
  // buffer ranges and offsets are 32-bit
  const int64_t lim = (int64_t)1 << 31;
  if ((p.Mb + BM) * p.lda * 4 >= lim || p.K * p.ldb * 4 >= lim) return hipErrorInvalidValue;
  // 256 x 256 tiles where every block is full and the shapes divide
  const bool wide = tile >= 4 && p.Mb % 256 == 0 && p.Nb % 256 == 0 && p.K % 32 == 0 &&
                    p.M == (int64_t)p.grid * p.Mb && p.N == (int64_t)p.grid * p.Nb &&
                    p.ldc % 4 == 0 && p.Nb % 4 == 0;
  if (wide) {
    p.tiles_m = (int32_t)(p.Mb / 256);
    p.tiles_n = (int32_t)(p.Nb / 256);
    const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(coded_gemm_2d_wide_kernel, dim3((unsigned)blocks), dim3(w2d::NT), 0,
                       stream, p);
    return hipGetLastError();
  }
  p.tiles_m = (int32_t)((p.Mb + BM - 1) / BM);
  p.tiles_n = (int32_t)((p.Nb + BN - 1) / BN);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(coded_gemm_2d_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
