// FP8-e4m3 coded products with one power-of-two scale per 128 x 128 block.
//
// quant_a_kernel  - the encode for FP8: per computed symbol g and 128 x 128
//                   tile of its coded block C_g = sum of its data blocks A_s
//                   (Sec. II, XOR read as a real sum), sum the members in
//                   FP32 (ascending), take the tile's amax, scale s = the
//                   smallest power of two with amax <= 448 s (1 when
//                   amax = 0, at least 2^-122) and store
//                   q = e4m3(clamp(x / s, +-448)) (round to nearest even).
//                   FP8x2 also stores the residual term
//                   q2 = e4m3(clamp((x / s - q) * 16, +-448)), so that
//                   x ~ s (q + q2 / 16).  x / s is exact.
// quant_b_kernel  - the same for B, written transposed (N x Kp, k
//                   contiguous) so that both MFMA operands read k runs.
// coded_gemm_fp8  - Y_g = sum over 128-wide k chunks of sA sB (qA . qB) on
//                   v_mfma_scale_f32_16x16x128_f8f6f4, whose E8M0 scale
//                   operands carry sA and sB (and the residual plane's
//                   extra 2^-4), so that every chunk accumulates straight
//                   into the MFMA accumulators with no vector arithmetic.
//
// The encode cannot be folded into the GEMM prologue here: a tile's scale
// needs the amax of the whole 128 x 128 coded tile, and every N-tile of the
// GEMM would repeat the FP32 reads and the reduction; one streaming pass
// that writes 1-byte codes is cheaper.
//
// Workspace layout (bytes, each part 256-aligned, see bpx_plan::fp8_layout):
//   Y slots | Aq [n_sym][Mbp][Kp] | Aq2 (FP8x2) | sA [n_sym][Mbp/128][Kp/128]
//   | Bq [Np][Kp] | sB [Kp/128][Np/128]
// with Mbp = Mb rounded up to 128, Kp = K rounded up to 128, Np = N rounded
// up to 128; padding rows/columns are zero codes.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));

constexpr float kE4M3Max = 448.f;

// The smallest power of two s with amax <= 448 s, at least 2^-122 (so that
// s / 16 is a normal power of two too); 1 for amax = 0.  With amax =
// (1 + f 2^-23) 2^(b - 127): 448 = 1.75 2^8, so s = 2^(b - 135) when
// f <= 0.75 2^23, else 2^(b - 134).  Exact integer work, no rounding.
constexpr int kMinScaleExp = -122;
__device__ __forceinline__ float pow2_scale(float amax) {
  if (!(amax > 0.f)) return 1.f;
  const unsigned bits = __float_as_uint(amax);
  const int b = (int)((bits >> 23) & 0xffu);
  int e = b - ((bits & 0x7fffffu) <= 0x600000u ? 135 : 134);
  e = e < kMinScaleExp ? kMinScaleExp : e;
  return __uint_as_float((unsigned)(e + 127) << 23);
}
// Scales are read through the constant address space (scalar loads).
typedef __attribute__((address_space(4))) float cfloat;
// E8M0 byte of a power-of-two scale: its biased exponent.
__device__ __forceinline__ int e8m0(float s) { return (int)((__float_as_uint(s) >> 23) & 0xffu); }

__device__ __forceinline__ float clamp448(float v) {
  return v > kE4M3Max ? kE4M3Max : (v < -kE4M3Max ? -kE4M3Max : v);
}

// Four e4m3 codes of four floats, packed little-endian into one int.
__device__ __forceinline__ int pack_e4m3(v4f v) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp448(v[0]), clamp448(v[1]), 0, false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(clamp448(v[2]), clamp448(v[3]), w, true);
}
__device__ __forceinline__ v4f unpack_e4m3(int w) {
  return v4f{__builtin_amdgcn_cvt_f32_fp8(w, 0), __builtin_amdgcn_cvt_f32_fp8(w, 1),
             __builtin_amdgcn_cvt_f32_fp8(w, 2), __builtin_amdgcn_cvt_f32_fp8(w, 3)};
}

__device__ __forceinline__ float block_amax(float m, float* red) {
  // wave reduction then across the 4 waves of the block
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  return m;
}

// grid: (Kp/128, Mbp/128, n_sym), 256 threads; thread t owns float4 chunks
// f = t + 256 i (i < 16): row f / 32, k offset (f % 32) * 4 of the tile.
// Members are summed one at a time, ascending, each member's 16 loads
// issued together: the member's rows of the tile are a raw buffer whose
// range ends at its last row that exists (rows past Mb or M read zero),
// and chunks past K are sent out of range.
__device__ __forceinline__ v4f qload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}
__global__ __launch_bounds__(256) void quant_a_kernel(Fp8Params p) {
  __shared__ float red[4];
  const int kb = blockIdx.x, rb = blockIdx.y, si = blockIdx.z;
  const int id_off = __builtin_amdgcn_readfirstlane(p.syms[4 * si + 0]);
  const int deg = __builtin_amdgcn_readfirstlane(p.syms[4 * si + 1]);
  const int32_t* ids = p.ids + id_off;
  const int64_t k0 = (int64_t)kb * 128, r0 = (int64_t)rb * 128;
  uint32_t off[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int64_t lr = f / 32, kk = (f % 32) * 4;
    off[i] = k0 + kk < p.K ? (uint32_t)((lr * p.lda + kk) * 4) : 0x80000000u;
  }
  v4f x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int m = 0; m < deg; ++m) {
    const int64_t first = (int64_t)__builtin_amdgcn_readfirstlane(ids[m]) * p.Mb + r0;
    int64_t rows = p.Mb - r0 < p.M - first ? p.Mb - r0 : p.M - first;
    rows = rows < 0 ? 0 : (rows > 128 ? 128 : rows);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.A + first * p.lda + k0), (short)0, (int)(rows * p.lda * 4),
        0x00020000);
    v4f v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = qload(rs, off[i]);
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] += v[i];
  }
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const v4f s = x[i];
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(s[0]), fabsf(s[1])), fmaxf(fabsf(s[2]), fabsf(s[3]))));
  }
  amax = block_amax(amax, red);
  const float sc = pow2_scale(amax);
  const int64_t sym_bytes = p.Mbp * p.Kp;
  unsigned char* q = p.aq + (int64_t)si * sym_bytes;
  unsigned char* q2 = p.aq2 ? p.aq2 + (int64_t)si * sym_bytes : nullptr;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int64_t r = r0 + f / 32, k = k0 + (f % 32) * 4;
    const v4f v = x[i] / sc;
    const int w = pack_e4m3(v);
    *reinterpret_cast<int*>(q + r * p.Kp + k) = w;
    if (q2) *reinterpret_cast<int*>(q2 + r * p.Kp + k) = pack_e4m3((v - unpack_e4m3(w)) * 16.f);
  }
  if (threadIdx.x == 0) p.sa[((int64_t)si * (p.Mbp / 128) + rb) * (p.Kp / 128) + kb] = sc;
}

// grid: (Np/128, Kp/128), 256 threads.  Reads a 128 (k) x 128 (n) block of B
// coalesced along n, writes codes transposed through LDS.
__global__ __launch_bounds__(256) void quant_b_kernel(Fp8Params p) {
  __shared__ float red[4];
  __shared__ unsigned char t[128][132];
  const int nb = blockIdx.x, kb = blockIdx.y;
  const int64_t n0 = (int64_t)nb * 128, k0 = (int64_t)kb * 128;
  v4f x[16];
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int64_t k = k0 + f / 32, n = n0 + (f % 32) * 4;
    v4f s = {0.f, 0.f, 0.f, 0.f};
    if (k < p.K) {
      const float* src = p.B + k * p.ldb + n;
      if (n + 3 < p.N) {
        s = *reinterpret_cast<const v4f*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < p.N) s[e] = src[e];
      }
    }
    x[i] = s;
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(s[0]), fabsf(s[1])), fmaxf(fabsf(s[2]), fabsf(s[3]))));
  }
  amax = block_amax(amax, red);
  const float sc = pow2_scale(amax);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int kl = f / 32, nl = (f % 32) * 4;
    const int w = pack_e4m3(x[i] / sc);
#pragma unroll
    for (int e = 0; e < 4; ++e) t[nl + e][kl] = (unsigned char)((w >> (8 * e)) & 0xff);
  }
  __syncthreads();
  // 128 rows (n) of 128 code bytes: thread writes 16-byte pieces
  for (int f = threadIdx.x; f < 128 * 8; f += 256) {
    const int nl = f / 8, kc = (f % 8) * 16;
    uint4 v;
    v.x = *reinterpret_cast<const unsigned*>(&t[nl][kc + 0]);
    v.y = *reinterpret_cast<const unsigned*>(&t[nl][kc + 4]);
    v.z = *reinterpret_cast<const unsigned*>(&t[nl][kc + 8]);
    v.w = *reinterpret_cast<const unsigned*>(&t[nl][kc + 12]);
    *reinterpret_cast<uint4*>(p.bq + (n0 + nl) * p.Kp + k0 + kc) = v;
  }
  if (threadIdx.x == 0) p.sb[(int64_t)kb * (p.Np / 128) + nb] = sc;
}

// ----------------------------------------------------------------- GEMM --
constexpr int kThreads = 256;
constexpr int CK = 128;       // k chunk = scale block
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// LDS layout of a staged chunk: rows of 128 bytes (one k chunk of codes),
// unpadded; the 16-byte granule g of row r sits at granule slot
// g ^ ((r >> 1) & 5) of the row.  gfx950 serves a 128-bit LDS write to 8
// lanes at a time over 32 banks (the staging stores: one row's 8 granules
// per 8 lanes, distinct slots in any row) and a 128-bit read to 16 lanes at
// a time over 64 banks, the 16 being the lanes that agree in lane bit 5 and
// in the parity of lane bits 2..4.  For the MFMA fragment reads (lane
// 16 q + c of a k group reads row c, granule 2 q or 2 q + 1) this swizzle
// puts each such group on 16 distinct bank quads; padded rows of 144 bytes
// left two lanes on a quad (2-way conflicts on every fragment read).
__device__ __forceinline__ int lds_off(int row, int granule) {
  return row * CK + ((granule ^ ((row >> 1) & 5)) << 4);
}

// LDS row of B row n.  The MFMA's lane c16 of output block j takes the
// interleaved column 4 c16 + j of a 64-column group (so that the epilogue
// writes four adjacent columns); stored at row 16 (n % 4) + (n % 64) / 4 of
// its group, column 4 c16 + j is read from row 16 j + c16: 16 consecutive
// rows per fragment, the shape the swizzle above is made for.
__device__ __forceinline__ int b_slot(int n) {
  return (n & ~63) | ((n & 3) << 4) | ((n & 63) >> 2);
}

// One lane's 32-byte MFMA operand (granules 2 q, 2 q + 1 of a row): two
// 16-byte reads at the swizzled granule offsets x0 and x0 ^ 16.
__device__ __forceinline__ v8i frag(const unsigned char* row, int x0) {
  const v4u lo = *reinterpret_cast<const v4u*>(row + x0);
  const v4u hi = *reinterpret_cast<const v4u*>(row + (x0 ^ 16));
  return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
             (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
}

__device__ __forceinline__ int xcd_remap(int lin, int total) {
  if ((total & 7) != 0) return lin;
  return (lin & 7) * (total >> 3) + (lin >> 3);
}

template <int X2>
__global__ __launch_bounds__(kThreads, 1) void coded_gemm_fp8_kernel(Fp8Params p) {
  constexpr int BM = 128, BN = 128, TM = 64, TN = 64, FM = 4, FN = 4;
  constexpr int NA = X2 ? 2 : 1;                  // A planes
  constexpr int STAGE = (NA * BM + BN) * CK;       // bytes per stage
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int q = lane >> 4, c16 = lane & 15;

  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int per_sym = p.tiles_m * p.tiles_n;
  const int si = lin / per_sym;
  const int rem = lin - si * per_sym;
  const int mt = rem / p.tiles_n;
  const int nt = rem - mt * p.tiles_n;
  const int m0 = mt * BM, n0 = nt * BN;
  const int dest = p.syms[4 * si + 2];

  const int64_t sym_bytes = p.Mbp * p.Kp;
  const unsigned char* Aq = p.aq + (int64_t)si * sym_bytes + (int64_t)m0 * p.Kp;
  const unsigned char* Aq2 = X2 ? p.aq2 + (int64_t)si * sym_bytes + (int64_t)m0 * p.Kp : nullptr;
  const unsigned char* Bq = p.bq + (int64_t)n0 * p.Kp;
  const cfloat* sa = (const cfloat*)p.sa + ((int64_t)si * (p.Mbp / 128) + mt) * (p.Kp / 128);
  const cfloat* sb = (const cfloat*)p.sb + nt;
  const int64_t np128 = p.Np / 128;

  // 16-byte pieces: row f / 8, byte offset (f % 8) * 16; 4 per thread per plane
  uint4 ra[NA][4], rbv[4];
  auto load = [&](int c) __attribute__((always_inline)) {
    const int64_t kc = (int64_t)c * CK;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + kThreads * i;
      const int64_t off = (int64_t)(f / 8) * p.Kp + kc + (f % 8) * 16;
      ra[0][i] = *reinterpret_cast<const uint4*>(Aq + off);
      if (X2) ra[NA - 1][i] = *reinterpret_cast<const uint4*>(Aq2 + off);
      rbv[i] = *reinterpret_cast<const uint4*>(Bq + off);
    }
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
    unsigned char* st = lds + buf * STAGE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + kThreads * i;
      const int o = lds_off(f / 8, f % 8);
#pragma unroll
      for (int a = 0; a < NA; ++a) *reinterpret_cast<uint4*>(st + a * BM * CK + o) = ra[a][i];
      *reinterpret_cast<uint4*>(st + NA * BM * CK + lds_off(b_slot(f / 8), f % 8)) = rbv[i];
    }
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nc = (int)(p.Kp / CK);
  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    const bool more = c + 1 < nc;
    if (more) load(c + 1);
    const unsigned char* st = lds + (c & 1) * STAGE;
    const int x0 = lds_off(c16, 2 * q) - c16 * CK;  // rows below are c16 mod 16
    v8i a[NA][FM], b[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int pl = 0; pl < NA; ++pl)
        a[pl][i] = frag(st + (pl * BM + wm * TM + i * 16 + c16) * CK, x0);
#pragma unroll
    for (int j = 0; j < FN; ++j)  // output column wn TN + 4 c16 + j, at row 16 j + c16
      b[j] = frag(st + (NA * BM + wn * TN + 16 * j + c16) * CK, x0);
    // the chunk's scales as E8M0 bytes (uniform: scalar loads)
    const int ea = __builtin_amdgcn_readfirstlane(e8m0(sa[c]));
    const int eb = __builtin_amdgcn_readfirstlane(e8m0(sb[(int64_t)c * np128]));
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if (X2)  // the residual plane carries a factor 16: scale 2^-4 more
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[1][i], b[j], acc[i][j], 0,
                                                                        0, 0, ea - 4, 0, eb);
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[0][i], b[j], acc[i][j], 0,
                                                                      0, 0, ea, 0, eb);
      }
    if (more) store((c + 1) & 1);
    __syncthreads();
  }

  float* out;
  int64_t ldo, rows;
  const int64_t Mb = p.Mb, N = p.N, M = p.M;
  if (dest >= 0) {
    out = p.Y + (int64_t)dest * Mb * N;
    ldo = N;
    rows = Mb;
  } else {
    const int64_t sb_ = -1 - dest;
    out = p.C + sb_ * Mb * p.ldc;
    ldo = p.ldc;
    rows = M - sb_ * Mb < Mb ? M - sb_ * Mb : Mb;
  }
  const bool vec_ok = (ldo & 3) == 0;
  const int64_t col = n0 + wn * TN + 4 * c16;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m0 + wm * TM + i * 16 + 4 * q + r;
      if (row >= rows) continue;
      float* dst = out + row * ldo + col;
      const v4f v = {acc[i][0][r], acc[i][1][r], acc[i][2][r], acc[i][3][r]};
      if (col + 3 < N && vec_ok) {
        *reinterpret_cast<v4f*>(dst) = v;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < N) dst[e] = v[e];
      }
    }
}

// ----------------------------------------------------------- wide tile --
// The coded blocks' codes are one matrix of R = n_sym * Mbp rows (Mbp a
// multiple of 128), so the products of all symbols form one R x Np x Kp
// GEMM whose 128-row blocks each belong to one symbol.  Tiles of BM x 256
// (BM = 128: a 256-row tile with FP32 accumulators does not fit the
// registers), 8 waves of (BM / WM) x (256 / WN), each wave inside one 128 x 128
// scale block, so a chunk's scales sA and sB are one E8M0 byte each per
// wave; the MFMA applies them (and the residual plane's extra 2^-4) exactly
// and both planes accumulate straight into the accumulators.  Global loads
// are raw buffer loads (scalar resource per plane and chunk, one 32-bit
// per-thread offset).
namespace wide8 {
constexpr int BN = 256;
constexpr int NT = 512;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer, 32-bit elements

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const unsigned char* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(base), (short)0, -1,
                                           kRsrcWord3);
}
typedef __attribute__((address_space(3))) void* lds_addr;
__device__ __forceinline__ lds_addr lds_ptr(unsigned char* p) { return (lds_addr)p; }
}  // namespace wide8

// Tile order of the wide kernel: each XCD takes a contiguous range of tile
// indices (xcd_remap), and consecutive indices walk down gm row panels
// before the next column panel, so the 32 tiles an XCD runs at once cover
// gm row panels x 32 / gm column panels and share their A and B chunks in
// that XCD's L2 (one row panel across all column panels would stream all
// of B through it for every row panel).
__device__ __forceinline__ void grouped_tile(int L, int rows, int cols, int gm, int* row,
                                             int* col) {
  const int per_group = gm * cols;
  const int g = L / per_group;
  const int first = g * gm;
  const int gsz = rows - first < gm ? rows - first : gm;
  const int r = L - g * per_group;
  *row = first + r % gsz;
  *col = r / gsz;
}

template <int BM, int WM, int WN, int X2>
__global__ __launch_bounds__(wide8::NT, 1) void coded_gemm_fp8_wide_kernel(Fp8Params p) {
  using namespace wide8;
  constexpr int TM = BM / WM, TN = BN / WN;   // wave tile
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int NA = X2 ? 2 : 1;              // A planes
  constexpr int PA = BM * 8 / NT;             // 16-byte pieces per thread per A plane
  constexpr int PB = BN * 8 / NT;             // and for B
  constexpr int STAGE = (NA * BM + BN) * CK;  // bytes per LDS stage
  static_assert(TM <= 128 && TN <= 128 && FN % 4 == 0 && PA >= 1, "wave tile");
  static_assert(NT / 8 == 64 && BM % 64 == 0 && BN % 64 == 0, "64-row staging groups");
  // two stages as two arrays: the compiler then sees that a stage being
  // filled is not the one being read
  __shared__ __attribute__((aligned(16))) unsigned char lds0[STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char lds1[STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int q = lane >> 4, c16 = lane & 15;

  int mt, nt;
  grouped_tile(xcd_remap(blockIdx.x, gridDim.x), p.tiles_m, p.tiles_n, p.group_m, &mt, &nt);
  const int64_t m0 = (int64_t)mt * BM, n0 = (int64_t)nt * BN;
  const int64_t Kp = p.Kp;

  // Staging by direct loads to LDS: one instruction of a wave fills 64
  // consecutive 16-byte LDS slots, lane l the slot base + 16 l, and the
  // global address is the lane's own.  Instruction u of wave w fills rows
  // 64 u + t of its operand's region, t = 8 w + l / 8, slot l % 8, which
  // holds granule (l % 8) ^ ((t >> 1) & 5) of that row (the swizzle is its
  // own inverse and depends on t only).  In the B region, LDS row 64 u + t
  // holds B row 64 u + nlow(t) (the inverse of b_slot).
  const int t = 8 * wave + (lane >> 3);
  const int g = (lane & 7) ^ ((t >> 1) & 5);
  const uint32_t va = (uint32_t)(t * Kp + g * 16);
  const uint32_t vb = (uint32_t)((((t & 15) << 2) | (t >> 4)) * Kp + g * 16);
  const uint32_t step64 = (uint32_t)(64 * Kp);
  auto dma = [&](unsigned char* st, int c) __attribute__((always_inline)) {
    const int64_t kc = (int64_t)c * CK;
    const auto r0 = rsrc(p.aq + m0 * Kp + kc);
#pragma unroll
    for (int u = 0; u < PA; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r0, lds_ptr(st + (64 * u + 8 * wave) * CK), 16, va,
                                               u * step64, 0, 0);
    if (X2) {
      const auto r1 = rsrc(p.aq2 + m0 * Kp + kc);
#pragma unroll
      for (int u = 0; u < PA; ++u)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            r1, lds_ptr(st + (BM + 64 * u + 8 * wave) * CK), 16, va, u * step64, 0, 0);
    }
    const auto r2 = rsrc(p.bq + n0 * Kp + kc);
#pragma unroll
    for (int u = 0; u < PB; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          r2, lds_ptr(st + (NA * BM + 64 * u + 8 * wave) * CK), 16, vb, u * step64, 0, 0);
  };

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  // The chunk scales are read as constant memory at wave-uniform addresses,
  // i.e. by scalar loads: a vector load of them at the top of a chunk would
  // make its wait (vmcnt) also wait for the next chunk's copies to LDS.
  const int64_t kc128 = Kp / 128;
  const int64_t np128 = p.Np / 128;
  const int rba = __builtin_amdgcn_readfirstlane((int)((m0 + wm * TM) / 128));
  const int cbb = __builtin_amdgcn_readfirstlane((int)((n0 + wn * TN) / 128));
  const cfloat* sa = (const cfloat*)p.sa + (int64_t)rba * kc128;
  const cfloat* sbp = (const cfloat*)p.sb + cbb;

  const int x0 = lds_off(c16, 2 * q) - c16 * CK;  // fragment rows are c16 mod 16
  auto compute = [&](const unsigned char* st, int c) __attribute__((always_inline)) {
    const int ea = __builtin_amdgcn_readfirstlane(e8m0(sa[c]));
    const int eb = __builtin_amdgcn_readfirstlane(e8m0(sbp[(int64_t)c * np128]));
    v8i a[NA][FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int pl = 0; pl < NA; ++pl) a[pl][i] = frag(st + (pl * BM + wm * TM + i * 16 + c16) * CK, x0);
#pragma unroll
    for (int jg = 0; jg < FN / 4; ++jg) {
      v8i b[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)  // output column jg 64 + 4 c16 + jj, at row 16 jj + c16
        b[jj] = frag(st + (NA * BM + wn * TN + jg * 64 + 16 * jj + c16) * CK, x0);
      // Per fragment row: the four residual-plane products first, then the
      // four main-plane products, so that no MFMA waits on the one just
      // issued; per output the same MFMAs in the same order as the
      // per-symbol tile.
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        if (X2)  // residual plane: scale 2^-4 more
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            acc[i][jg * 4 + jj] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                a[NA - 1][i], b[jj], acc[i][jg * 4 + jj], 0, 0, 0, ea - 4, 0, eb);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jg * 4 + jj] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              a[0][i], b[jj], acc[i][jg * 4 + jj], 0, 0, 0, ea, 0, eb);
      }
    }
  };

  // Chunk c sits in stage c & 1.  A stage is refilled only after the
  // barrier that ends the chunk before it, and each chunk ends with this
  // wave's loads done (vmcnt 0) and a barrier, so every wave's part of the
  // next stage has landed before any wave reads it.
  const int nc = (int)(Kp / CK);
  dma(lds0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int c = 0; c < nc; c += 2) {
    if (c + 1 < nc) dma(lds1, c + 1);
    compute(lds0, c);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nc) {
      if (c + 2 < nc) dma(lds0, c + 2);
      compute(lds1, c + 1);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }

  // The wave's rows lie in one 128-row block, hence in one symbol.
  const int64_t wrow = m0 + wm * TM;
  const int si = (int)(wrow / p.Mbp);
  const int64_t lrow0 = wrow - (int64_t)si * p.Mbp;
  const int dest = p.syms[4 * si + 2];
  float* out;
  int64_t ldo, rows;
  if (dest >= 0) {
    out = p.Y + (int64_t)dest * p.Mb * p.N;
    ldo = p.N;
    rows = p.Mb;
  } else {
    const int64_t sblk = -1 - dest;
    out = p.C + sblk * p.Mb * p.ldc;
    ldo = p.ldc;
    rows = p.M - sblk * p.Mb < p.Mb ? p.M - sblk * p.Mb : p.Mb;
  }
  const bool vec_ok = (ldo & 3) == 0;
#pragma unroll
  for (int jg = 0; jg < FN / 4; ++jg) {
    const int64_t col = n0 + wn * TN + jg * 64 + 4 * c16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = lrow0 + i * 16 + 4 * q + r;
        if (row >= rows) continue;
        float* dst = out + row * ldo + col;
        const v4f v = {acc[i][4 * jg + 0][r], acc[i][4 * jg + 1][r], acc[i][4 * jg + 2][r],
                       acc[i][4 * jg + 3][r]};
        if (col + 3 < p.N && vec_ok) {
          *reinterpret_cast<v4f*>(dst) = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < p.N) dst[e] = v[e];
        }
      }
  }
}

}  // namespace

hipError_t launch_quant_a(const Fp8Params& p, hipStream_t stream) {
  if (p.n_sym == 0) return hipSuccess;
  // a member's 128-row tile is one buffer of 32-bit byte offsets
  if (128 * p.lda * 4 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(p.Kp / 128), (unsigned)(p.Mbp / 128), (unsigned)p.n_sym);
  hipLaunchKernelGGL(quant_a_kernel, grid, dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_quant_b(const Fp8Params& p, hipStream_t stream) {
  const dim3 grid((unsigned)(p.Np / 128), (unsigned)(p.Kp / 128));
  hipLaunchKernelGGL(quant_b_kernel, grid, dim3(256), 0, stream, p);
  return hipGetLastError();
}

int32_t fp8_tile_count() { return 2; }

// Row panels per group of the wide kernel's tile order.
constexpr int32_t kFp8GroupM = 4;

// tile 0: 128 x 128 per symbol; tile 1: 128 x 256 tiles over all symbols'
// codes (used when Np is a multiple of 256, otherwise tile 0).  The wide
// kernel addresses each chunk from a 64-bit base (the tile's first row),
// so only a lane's offset inside one tile (128 rows of A codes, 256 rows of
// B codes: under 256 Kp bytes) has to fit the buffer instruction's 32
// bits; the code matrices themselves may pass 4 GiB.
hipError_t launch_coded_gemm_fp8(const Fp8Params& p0, int32_t tile, hipStream_t stream) {
  Fp8Params p = p0;
  if (p.n_sym == 0) return hipSuccess;
  const int64_t R = (int64_t)p.n_sym * p.Mbp;
  const int64_t bm = 128;
  if (tile == 1 && p.Np % 256 == 0 && R % bm == 0 && 256 * p.Kp < (int64_t)1 << 31) {
    p.tiles_m = (int32_t)(R / bm);
    if (p.group_m <= 0) p.group_m = kFp8GroupM;
    p.tiles_n = (int32_t)(p.Np / 256);
    const int64_t blocks = (int64_t)p.tiles_m * p.tiles_n;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (p.aq2)
      hipLaunchKernelGGL((coded_gemm_fp8_wide_kernel<128, 2, 4, 1>), dim3((unsigned)blocks),
                         dim3(wide8::NT), 0, stream, p);
    else
      hipLaunchKernelGGL((coded_gemm_fp8_wide_kernel<128, 2, 4, 0>), dim3((unsigned)blocks),
                         dim3(wide8::NT), 0, stream, p);
    return hipGetLastError();
  }
  p.tiles_m = (int32_t)((p.Mb + 127) / 128);
  p.tiles_n = (int32_t)((p.N + 127) / 128);
  const int64_t blocks = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (p.aq2)
    hipLaunchKernelGGL(coded_gemm_fp8_kernel<1>, dim3((unsigned)blocks), dim3(kThreads), 0,
                       stream, p);
  else
    hipLaunchKernelGGL(coded_gemm_fp8_kernel<0>, dim3((unsigned)blocks), dim3(kThreads), 0,
                       stream, p);
  return hipGetLastError();
}

}  // namespace bpx
