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
// floats).  Two index permutations make every LDS fragment read 128 bits
// wide: (1) inside a 16-wide k chunk, lane group q = lane/16 owns
// k = 4q..4q+3 and MFMA t of the chunk contracts k = 4q + t, so a lane reads
// its four A values along k at once; (2) the wave's N range is split so that
// MFMA column c16 of subtile j is output column 4*c16 + j, so a lane reads
// the B values of its four subtiles along n at once, and in the epilogue it
// owns four adjacent output columns (one float4 store per row).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

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
  static_assert(FN % 4 == 0, "wave N tile must hold 4 interleaved 16-column subtiles");
};

__device__ __forceinline__ int xcd_remap(int lin, int total) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of tile indices so that tiles sharing A and B panels
  // share an L2.
  if ((total & 7) != 0) return lin;
  return (lin & 7) * (total >> 3) + (lin >> 3);
}

// Tile index -> (row panel, column panel), row panels taken in groups of gm:
// consecutive tiles walk down gm row panels before moving to the next column
// panel, so the tiles one XCD runs together share A and B K-slices in L2.
// Row panel = symbol * tiles_m + m-tile.
__device__ __forceinline__ void tile_coords(int L, int rows, int cols, int gm, int* row,
                                            int* col) {
  if (gm <= 1) {
    *row = L / cols;
    *col = L - *row * cols;
    return;
  }
  const int per_group = gm * cols;
  const int g = L / per_group;
  const int first = g * gm;
  const int gsz = rows - first < gm ? rows - first : gm;
  const int r = L - g * per_group;
  *row = first + r % gsz;
  *col = r / gsz;
}

template <int BM, int BN, int BK, int OCC>
__global__ __launch_bounds__(kThreads, OCC) void coded_gemm_f32_kernel(GemmParams p) {
  using T = F32Tile<BM, BN, BK>;
  __shared__ __attribute__((aligned(16))) float lds[2 * (T::A_SIZE + T::B_SIZE)];
  float* As0 = lds;
  float* Bs0 = lds + 2 * T::A_SIZE;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = lane >> 4, c16 = lane & 15;

  int rp, nt, si, m0, n0;
  if (p.wide_rem) {
    // sub-tile of a 256 x 256 tile left over from the wide launch
    constexpr int SN = 256 / BN, PER = (256 / BM) * SN;
    const int sub = blockIdx.x % PER;
    tile_coords(p.wide_lin0 + (int)blockIdx.x / PER, p.n_sym * p.tiles_m, p.tiles_n, p.group_m,
                &rp, &nt);
    si = rp / p.tiles_m;
    m0 = (rp - si * p.tiles_m) * 256 + (sub / SN) * BM;
    n0 = nt * 256 + (sub % SN) * BN;
  } else {
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    tile_coords(lin, p.n_sym * p.tiles_m, p.tiles_n, p.group_m, &rp, &nt);
    si = rp / p.tiles_m;
    m0 = (rp - si * p.tiles_m) * BM;
    n0 = nt * BN;
  }

  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;

  const int64_t K = p.K, N = p.N, Mb = p.Mb, M = p.M;

  // The next K-slice is staged in two halves, one per 16-wide k chunk of the
  // current slice: half h covers A rows [h*BM/2, (h+1)*BM/2) and B k-rows
  // [h*BK/2, (h+1)*BK/2).  Its global loads are issued before chunk h's MFMAs
  // and summed / stored to the other LDS buffer after them, which keeps only
  // half a slice of prefetch in registers.
  constexpr int AH = T::A_F4 / 2, BH = T::B_F4 / 2;
  static_assert(BK == 32 && AH >= 1 && BH >= 1, "two 16-wide chunks per slice");
  // Per-thread, member-independent byte offsets (32-bit: the host
  // guarantees a block of A and a K-slice of B fit in 2^30 floats).
  int a_row[T::A_F4], a_kc[T::A_F4];
  uint32_t a_off[T::A_F4];
#pragma unroll
  for (int i = 0; i < T::A_F4; ++i) {
    const int f = tid + kThreads * i;
    a_row[i] = f / (BK / 4);
    a_kc[i] = (f % (BK / 4)) * 4;
    a_off[i] = (uint32_t)((m0 + a_row[i]) * (int)p.lda + a_kc[i]) * 4u;
  }
  int b_kr[T::B_F4], b_nc[T::B_F4];
  uint32_t b_off[T::B_F4];
#pragma unroll
  for (int i = 0; i < T::B_F4; ++i) {
    const int f = tid + kThreads * i;
    b_kr[i] = f / (BN / 4);
    b_nc[i] = (f % (BN / 4)) * 4;
    b_off[i] = (uint32_t)(b_kr[i] * (int)p.ldb + n0 + b_nc[i]) * 4u;
  }
  // Member block bases (uniform).  A tile is "interior" when every member's
  // rows m0 .. m0+BM-1 and the columns n0 .. n0+BN-1 exist.
  const char* mbase[kPre];
#pragma unroll
  for (int m = 0; m < kPre; ++m)
    mbase[m] = reinterpret_cast<const char*>(p.A + (m < deg ? (int64_t)ids[m] * Mb * p.lda : 0));
  const int64_t s_last = deg > 0 ? ids[deg - 1] : 0;  // ids ascending
  const bool interior =
      m0 + BM <= Mb && s_last * Mb + m0 + BM <= M && n0 + BN <= N;

  auto a_valid = [&](int member, int i) __attribute__((always_inline)) -> bool {
    const int64_t rb = m0 + a_row[i];
    return rb < Mb && (int64_t)ids[member] * Mb + rb < M;
  };
  auto ld4 = [](const char* base, uint32_t off) __attribute__((always_inline)) -> v4f {
    return *reinterpret_cast<const v4f*>(base + off);
  };

  v4f pre[kPre][AH];
  v4f bre[BH];

  // Unpredicated loads of half h of the slice at k0 (interior tiles, full
  // slices).  Members past deg are not loaded and not summed.
  auto load_half_full = [&](int h, int k0) __attribute__((always_inline)) {
    const uint32_t kb4 = (uint32_t)k0 * 4u;
#pragma unroll
    for (int mbr = 0; mbr < kPre; ++mbr)
      if (mbr < deg) {
#pragma unroll
        for (int u = 0; u < AH; ++u) pre[mbr][u] = ld4(mbase[mbr], a_off[h * AH + u] + kb4);
      }
    const char* Bk = reinterpret_cast<const char*>(p.B + (int64_t)k0 * p.ldb);
#pragma unroll
    for (int u = 0; u < BH; ++u) bre[u] = ld4(Bk, b_off[h * BH + u]);
  };
  // Predicated loads (edge tiles, ragged last slice).
  auto load_half_edge = [&](int h, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int mbr = 0; mbr < kPre; ++mbr)
      if (mbr < deg) {
#pragma unroll
        for (int u = 0; u < AH; ++u) {
          const int i = h * AH + u;
          v4f v = {0.f, 0.f, 0.f, 0.f};
          if (a_valid(mbr, i) && k0 + a_kc[i] < K) v = ld4(mbase[mbr], a_off[i] + k0 * 4u);
          pre[mbr][u] = v;
        }
      }
    const float* Bk = p.B + (int64_t)k0 * p.ldb;
#pragma unroll
    for (int u = 0; u < BH; ++u) {
      const int i = h * BH + u;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      const int64_t nn = n0 + b_nc[i];
      if (k0 + b_kr[i] < K) {
        const float* r = Bk + b_off[i] / 4u;
        if (nn + 3 < N) {
          v = *reinterpret_cast<const v4f*>(r);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (nn + e < N) v[e] = r[e];
        }
      }
      bre[u] = v;
    }
  };
  auto store_half = [&](int h, int buf, int k0) __attribute__((always_inline)) {
    float* As = As0 + buf * T::A_SIZE;
    float* Bs = Bs0 + buf * T::B_SIZE;
#pragma unroll
    for (int u = 0; u < AH; ++u) {
      const int i = h * AH + u;
      v4f sum = pre[0][u];
#pragma unroll
      for (int mbr = 1; mbr < kPre; ++mbr)
        if (mbr < deg) sum += pre[mbr][u];
      // members beyond the prefetch depth (high-degree symbols)
      for (int mbr = kPre; mbr < deg; ++mbr) {
        if (a_valid(mbr, i) && k0 + a_kc[i] < K)
          sum += *reinterpret_cast<const v4f*>(p.A + (int64_t)ids[mbr] * Mb * p.lda +
                                               a_off[i] / 4u + k0);
      }
      *reinterpret_cast<v4f*>(As + a_row[i] * T::LDA_S + a_kc[i]) = sum;
    }
#pragma unroll
    for (int u = 0; u < BH; ++u) {
      const int i = h * BH + u;
      *reinterpret_cast<v4f*>(Bs + b_kr[i] * T::LDB_S + b_nc[i]) = bre[u];
    }
  };

  v4f acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute_chunk = [&](const float* As, const float* Bs, int kk) __attribute__((always_inline)) {
    v4f a[T::FM];
    v4f b[T::FN / 4][4];
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
      a[i] = *reinterpret_cast<const v4f*>(As + (wm * T::TM + i * 16 + c16) * T::LDA_S + kk +
                                           4 * q);
#pragma unroll
    for (int jg = 0; jg < T::FN / 4; ++jg)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        b[jg][t] = *reinterpret_cast<const v4f*>(Bs + (kk + 4 * q + t) * T::LDB_S + wn * T::TN +
                                                 jg * 64 + 4 * c16);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j / 4][t][j % 4],
                                                           acc[i][j], 0, 0, 0);
  };

  // One K-slice: compute slice kt from LDS, staging slice kt+1 (if any) into
  // the other buffer with full or predicated loads.
  auto slice = [&](int kt, bool more, auto full) __attribute__((always_inline)) {
    const int buf = kt & 1;
    const int kn = (kt + 1) * BK;
    const float* As = As0 + buf * T::A_SIZE;
    const float* Bs = Bs0 + buf * T::B_SIZE;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (more) {
        if constexpr (decltype(full)::value)
          load_half_full(h, kn);
        else
          load_half_edge(h, kn);
      }
      compute_chunk(As, Bs, h * 16);
      if (more) store_half(h, buf ^ 1, kn);
    }
    __syncthreads();
  };
  using Full = std::integral_constant<bool, true>;
  using Edge = std::integral_constant<bool, false>;

  const int nk = (int)((K + BK - 1) / BK);
  const int nk_full = (int)(K / BK);
  if (interior && nk_full >= 1) {
    load_half_full(0, 0);
    store_half(0, 0, 0);
    load_half_full(1, 0);
    store_half(1, 0, 0);
  } else {
    load_half_edge(0, 0);
    store_half(0, 0, 0);
    load_half_edge(1, 0);
    store_half(1, 0, 0);
  }
  __syncthreads();
  int kt = 0;
  if (interior) {
    // steady state: slice kt+1 is a full slice
    for (; kt + 1 < nk_full; ++kt) slice(kt, true, Full{});
  }
  for (; kt < nk; ++kt) slice(kt, kt + 1 < nk, Edge{});

  // Epilogue: for subtile (i, j) the lane holds rows 4q..4q+3; subtiles
  // j = 4*jg .. 4*jg+3 are the adjacent columns 64*jg + 4*c16 + 0..3.
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

// ------------------------------------------------------------ wide tile --
// 256 x 256 x 32 tile for shapes whose every tile is interior (Mb and N
// multiples of 256, K of 32, every data block full).  WM x WN waves each own
// a (256/WM) x (256/WN) wave tile whose accumulators live in the AGPR half
// of the register file, so that a K-slice is many MFMAs per wave between
// barriers.  Global loads are raw buffer loads: the per-thread offset is one
// 32-bit register each for A and B, the member block and the slice are in
// the (scalar) buffer resource and the row group in the scalar offset.  The
// loads and sums of members past deg are skipped by uniform branches (an
// empty buffer resource would return zeros without touching memory, but its
// loads still cost address-unit cycles: measured 7 % slower).
namespace wide {
constexpr int BM = 256, BN = 256, BK = 32;
// LDS rows are unpadded.  gfx950 serves a 128-bit LDS read to 16 lanes at a
// time over 64 banks, the 16 being the lanes that agree in lane bit 5 and in
// the parity of lane bits 2..4 (a write: 8 consecutive lanes over 32
// banks).  B fragment reads (lane 16 q + c: k-row 4 q + t, columns 4 c ..)
// are then conflict-free when k-rows four apart are 256-byte aligned, which
// unpadded 256-float rows are; A fragment reads (lane 16 q + c: row c,
// 16-byte granule g0 + q) need the granules of row r swizzled to slot
// g ^ ((r >> 1) & 7).  Padded rows (36 and 260 floats) left every fragment
// read with 2-way conflicts.
constexpr int LDA_S = BK, LDB_S = BN;
constexpr int A_SIZE = BM * LDA_S, B_SIZE = BK * LDB_S;
__device__ __forceinline__ int a_slot(int row, int granule) {
  return granule ^ ((row >> 1) & 7);
}
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer, 32-bit elements

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, bytes, kRsrcWord3);
}
__device__ __forceinline__ v4f bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(v4f,
                            __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
}  // namespace wide

template <int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, 1) void coded_gemm_f32_wide_kernel(GemmParams p) {
  using namespace wide;
  constexpr int NT = 64 * WM * WN;               // threads
  constexpr int TM = BM / WM, TN = BN / WN;      // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;      // 16 x 16 subtiles per wave
  constexpr int U = (BM / 2) * BK / 4 / NT;      // float4 per thread per half slice
  constexpr int RA = NT / 8, RB = NT / 64;       // row step of a thread's A / B loads
  static_assert(U >= 1 && FN % 4 == 0 && (BK / 2) * BN / 4 / NT == U, "tile split");
  static_assert(TM % 16 == 0 && RA % 16 == 0, "A rows of a fragment / a thread keep one swizzle");
  __shared__ __attribute__((aligned(16))) float lds[2 * (A_SIZE + B_SIZE)];
  float* As0 = lds;
  float* Bs0 = lds + 2 * A_SIZE;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int q = lane >> 4, c16 = lane & 15;

  const int nk_all = (int)(p.K / BK);
  int lin, kt0 = 0, kt1 = nk_all;
  if (p.wide_split) {  // piece b % P of tile wide_lin0 + b / P
    const int P = p.wide_split, piece = (int)blockIdx.x % P;
    lin = p.wide_lin0 + (int)blockIdx.x / P;
    kt0 = piece * nk_all / P;
    kt1 = (piece + 1) * nk_all / P;
  } else {
    lin = xcd_remap(blockIdx.x, gridDim.x);
  }
  int rp, nt;
  tile_coords(lin, p.n_sym * p.tiles_m, p.tiles_n, p.group_m, &rp, &nt);
  const int si = rp / p.tiles_m;
  const int mt = rp - si * p.tiles_m;
  const int m0 = mt * BM, n0 = nt * BN;

  const int id_off = p.syms[4 * si + 0];
  const int deg = p.syms[4 * si + 1];
  const int dest = p.syms[4 * si + 2];
  const int32_t* ids = p.ids + id_off;
  const int64_t lda = p.lda, ldb = p.ldb;

  // Half h of a slice: A rows 128 h + ar + RA u, k ak .. ak+3; B k-rows
  // 16 h + br + RB u, columns bc .. bc+3 (u < U).
  const int ar = tid >> 3, ak = (tid & 7) * 4;
  const int br = tid >> 6, bc = (tid & 63) * 4;
  const uint32_t a_off = (uint32_t)(((int64_t)(m0 + ar) * lda + ak) * 4);
  const uint32_t b_off = (uint32_t)(((int64_t)br * ldb + bc) * 4);
  const uint32_t a_row4 = (uint32_t)(lda * 4), b_row4 = (uint32_t)(ldb * 4);
  const int64_t blk = p.Mb * lda;  // floats per data block
  const int id0 = ids[0];
  const int id1 = deg > 1 ? ids[1] : 0;
  const int id2 = deg > 2 ? ids[2] : 0;
  const int id3 = deg > 3 ? ids[3] : 0;
  static_assert(kPre == 4, "member ids are held in four scalars");

  v4f pre[kPre][U];
  v4f bre[U];
  auto load_half = [&](int h, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      const int id = m == 0 ? id0 : m == 1 ? id1 : m == 2 ? id2 : id3;
      if (m < deg) {
        const auto r = rsrc(p.A + id * blk + k0, -1);
#pragma unroll
        for (int u = 0; u < U; ++u) pre[m][u] = bload(r, a_off, (128 * h + RA * u) * a_row4);
      }
    }
    const auto rb = rsrc(p.B + (int64_t)k0 * ldb + n0, -1);
#pragma unroll
    for (int u = 0; u < U; ++u) bre[u] = bload(rb, b_off, (16 * h + RB * u) * b_row4);
  };
  auto store_half = [&](int h, int buf, int k0) __attribute__((always_inline)) {
    // rows ar + 128 h + RA u share the swizzle of row ar (RA is a multiple of 16)
    float* As = As0 + buf * A_SIZE + ar * LDA_S + 4 * a_slot(ar, ak >> 2);
    float* Bs = Bs0 + buf * B_SIZE + br * LDB_S + bc;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v4f sum = pre[0][u];
#pragma unroll
      for (int m = 1; m < kPre; ++m)
        if (m < deg) sum += pre[m][u];
      if (deg > kPre) {  // members beyond the prefetch depth
        for (int m = kPre; m < deg; ++m)
          sum += bload(rsrc(p.A + ids[m] * blk + k0, -1), a_off, (128 * h + RA * u) * a_row4);
      }
      *reinterpret_cast<v4f*>(As + (128 * h + RA * u) * LDA_S) = sum;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      *reinterpret_cast<v4f*>(Bs + (16 * h + RB * u) * LDB_S) = bre[u];
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto compute_chunk = [&](const float* As, const float* Bs, int kk) __attribute__((always_inline)) {
    v4f a[FM];
    v4f b[FN / 4][4];
    const float* Aw = As + (wm * TM + c16) * LDA_S + 4 * a_slot(c16, (kk >> 2) + q);
    const float* Bw = Bs + (kk + 4 * q) * LDB_S + wn * TN + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const v4f*>(Aw + i * 16 * LDA_S);
#pragma unroll
    for (int jg = 0; jg < FN / 4; ++jg)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        b[jg][t] = *reinterpret_cast<const v4f*>(Bw + t * LDB_S + jg * 64);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j / 4][t][j % 4],
                                                           acc[i][j], 0, 0, 0);
  };

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    load_half(h, kt0 * BK);
    store_half(h, 0, kt0 * BK);
  }
  __syncthreads();
  for (int kt = kt0; kt + 1 < kt1; ++kt) {
    const int buf = (kt - kt0) & 1;
    const int kn = (kt + 1) * BK;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      load_half(h, kn);
      compute_chunk(As0 + buf * A_SIZE, Bs0 + buf * B_SIZE, h * 16);
      store_half(h, buf ^ 1, kn);
    }
    __syncthreads();
  }
  {
    const int buf = (kt1 - 1 - kt0) & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) compute_chunk(As0 + buf * A_SIZE, Bs0 + buf * B_SIZE, h * 16);
  }

  float* out;
  int64_t ldo;
  int64_t r0 = m0, c0 = n0;  // tile origin in out
  if (p.wide_split) {        // partial tile, 256 x 256 row-major
    out = p.part + (int64_t)blockIdx.x * BM * BN;
    ldo = BN;
    r0 = 0;
    c0 = 0;
  } else if (dest >= 0) {
    out = p.Y + (int64_t)dest * p.Mb * p.N;
    ldo = p.N;
  } else {
    out = p.C + (int64_t)(-1 - dest) * p.Mb * p.ldc;
    ldo = p.ldc;
  }
#pragma unroll
  for (int jg = 0; jg < FN / 4; ++jg) {
    const int64_t col = c0 + wn * TN + jg * 64 + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * TM + i * 16 + 4 * q + r;
        const v4f v = {acc[i][4 * jg + 0][r], acc[i][4 * jg + 1][r], acc[i][4 * jg + 2][r],
                       acc[i][4 * jg + 3][r]};
        *reinterpret_cast<v4f*>(out + row * ldo + col) = v;
      }
  }
}

// Sums the P partial tiles of each split tile in piece order (fixed, so
// results do not depend on scheduling) and writes the tile's output.
// grid: tiles x 64 blocks of 256 threads, one float4 per thread.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmParams p) {
  const int t = blockIdx.x >> 6;
  const int e = ((blockIdx.x & 63) << 8) + threadIdx.x;  // float4 index in the tile
  const int row = e >> 6, col = (e & 63) * 4;
  const int P = p.wide_split;
  const float* src = p.part + (int64_t)t * P * 65536 + row * 256 + col;
  v4f sum = *reinterpret_cast<const v4f*>(src);
  for (int k = 1; k < P; ++k) sum += *reinterpret_cast<const v4f*>(src + (int64_t)k * 65536);
  int rp, nt;
  tile_coords(p.wide_lin0 + t, p.n_sym * p.tiles_m, p.tiles_n, p.group_m, &rp, &nt);
  const int si = rp / p.tiles_m;
  const int64_t m = (int64_t)(rp - si * p.tiles_m) * 256 + row, n = (int64_t)nt * 256 + col;
  const int dest = p.syms[4 * si + 2];
  float* out = dest >= 0 ? p.Y + ((int64_t)dest * p.Mb + m) * p.N + n
                         : p.C + ((int64_t)(-1 - dest) * p.Mb + m) * p.ldc + n;
  *reinterpret_cast<v4f*>(out) = sum;
}

struct TileEntry {
  TileShape shape;
  void (*kernel)(GemmParams);
  unsigned threads;
};

const TileEntry kTiles[] = {
    {{128, 128, 32}, coded_gemm_f32_kernel<128, 128, 32, 2>, kThreads},
    {{64, 128, 32}, coded_gemm_f32_kernel<64, 128, 32, 2>, kThreads},
    {{128, 256, 32}, coded_gemm_f32_kernel<128, 256, 32, 1>, kThreads},
    {{256, 128, 32}, coded_gemm_f32_kernel<256, 128, 32, 1>, kThreads},
    // interior shapes only:
    {{256, 256, 32}, coded_gemm_f32_wide_kernel<2, 2>, 256},
    {{256, 256, 32}, coded_gemm_f32_wide_kernel<2, 4>, 512},
    {{256, 256, 32}, coded_gemm_f32_wide_kernel<4, 2>, 512},
};

constexpr int32_t kWideTile = 4;

}  // namespace

int32_t gemm_tile_count() { return (int32_t)(sizeof(kTiles) / sizeof(kTiles[0])); }
TileShape gemm_tile_shape(int32_t t) { return kTiles[t].shape; }

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

hipError_t launch_coded_gemm(const GemmParams& p0, int32_t tile, hipStream_t stream) {
  GemmParams p = p0;
  p.wide_rem = 0;
  p.wide_lin0 = 0;
  p.wide_split = 0;
  if (tile >= kWideTile) {
    // The wide tile has no edge path: shapes with a partial tile, a partial
    // data block or a ragged last K-slice take the 64 x 128 tile.
    const bool fits = p.Mb % 256 == 0 && p.N % 256 == 0 && p.K % 32 == 0 &&
                      p.M % p.Mb == 0 && p.ldc % 4 == 0;
    const int64_t T = fits ? (int64_t)p.n_sym * (p.Mb / 256) * (p.N / 256) : 0;
    const int64_t S = device_cu_count();  // one 256 x 256 workgroup per CU
    // Full rounds of 256 x 256 tiles run wide; a last round under 90 % full
    // runs as 64 x 128 sub-tiles (eight per tile, several per CU), which
    // keeps every CU busy to the end.  Both kernels sum in the same order,
    // so the split does not change results.
    const int64_t rem = T % S;
    const int64_t wide_tiles = rem * 10 < S * 9 ? T - rem : T;
    if (T == 0 || T > 0x7fffffff / 8) {
      tile = 1;
    } else {
      const TileEntry& e = kTiles[tile];
      p.tiles_m = (int32_t)(p.Mb / 256);
      p.tiles_n = (int32_t)(p.N / 256);
      if (wide_tiles > 0) {
        hipLaunchKernelGGL(e.kernel, dim3((unsigned)wide_tiles), dim3(e.threads), 0, stream, p);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
      }
      if (wide_tiles == T) return hipSuccess;
      // Last round: split each remaining tile's K range into P pieces (2 to
      // 4, each at least 8 slices), P chosen to minimise the rounds of
      // pieces in units of a wide round, ceil(R P / S) / P; used when that
      // is at most 0.8 of a round (64 x 128 sub-tiles of a 3/4-full round
      // measured 0.86) and the workspace holds partial tiles.  The pieces
      // run in chunks of as many tiles as the partial buffer holds, each
      // chunk followed by its reduction; otherwise 64 x 128 sub-tiles.
      const int64_t R = T - wide_tiles;
      int64_t P = 1;
      double best = 1e30;
      for (int64_t q = 2; q <= 4; ++q) {
        if ((p.K / 32) / q < 8 || !p.part || q > p.part_tiles) break;
        const double cost = (double)((R * q + S - 1) / S) / (double)q;
        if (cost < best - 1e-9) {
          best = cost;
          P = q;
        }
      }
      if (P >= 2 && best <= 0.8) {
        const int64_t chunk = p.part_tiles / P;  // tiles whose pieces fit the buffer
        p.wide_split = (int32_t)P;
        for (int64_t t0 = wide_tiles; t0 < T; t0 += chunk) {
          const int64_t r = std::min<int64_t>(chunk, T - t0);
          p.wide_lin0 = (int32_t)t0;
          hipLaunchKernelGGL(e.kernel, dim3((unsigned)(r * P)), dim3(e.threads), 0, stream, p);
          hipError_t err = hipGetLastError();
          if (err != hipSuccess) return err;
          hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)(r * 64)), dim3(256), 0,
                             stream, p);
          err = hipGetLastError();
          if (err != hipSuccess) return err;
        }
        return hipSuccess;
      }
      const TileEntry& s = kTiles[1];
      p.wide_rem = 1;
      p.wide_lin0 = (int32_t)wide_tiles;
      const int64_t per = (256 / s.shape.bm) * (256 / s.shape.bn);
      hipLaunchKernelGGL(s.kernel, dim3((unsigned)((T - wide_tiles) * per)), dim3(s.threads), 0,
                         stream, p);
      return hipGetLastError();
    }
  }
  const TileEntry& e = kTiles[tile];
  p.tiles_m = (int32_t)((p.Mb + e.shape.bm - 1) / e.shape.bm);
  p.tiles_n = (int32_t)((p.N + e.shape.bn - 1) / e.shape.bn);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(e.kernel, dim3((unsigned)blocks), dim3(e.threads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
