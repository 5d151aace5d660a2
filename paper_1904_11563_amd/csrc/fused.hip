// Coded product with the peel fused into the GEMM epilogue: one launch,
// the coded products never leave the chip.
//
// The BP decoder of Sec. I-A runs the same release program on every element
// of the Mb x N blocks, so a workgroup that owns one small output tile
// (rows r0 .. r0+15 of every data block, columns n0 .. n0+BN-1) can compute
// that tile of every computed coded product Y_g = C_g . B (C_g = sum of the
// symbol's data blocks, the encode of Sec. II with XOR read as a real sum),
// keep the releasers' tiles in LDS, and peel them there: X_s = Y_{g_s} -
// sum over u in N(g_s)\{s} of X_u, in (depth, s) order, FP32 with Kahan
// compensation for depth <= 4 and FP64 deeper, subtrahends ascending.  The
// decoded tiles go straight to C; Y never reaches HBM.
//
// This trades GEMM efficiency (16-row tiles, and only Mb/16 x N/BN
// workgroups) for one launch and no Y traffic, which is the right trade
// where the whole product is small enough for launches and latency to
// dominate (the library picks it by size; larger products take the
// two-launch path of coded GEMM + streaming peel).
//
// Layout of a workgroup (8 waves): the B column strip B[0:K, n0:n0+BN] is
// staged in LDS once (FP32: row-major k x BN; BF16: transposed per column,
// k contiguous, split into hi / lo planes); the tile's 16 rows of every
// data block pass through LDS one k group at a time (double-buffered, the
// next groups' loads in flight), and wave w computes the computed symbols
// w, w+8, ... from them, summing each symbol's members in FP32 registers
// (BF16: then splitting the sum into hi / lo); releasers' tiles are stored
// to LDS; after one barrier every thread peels its own elements.
//
// MFMA fragments: FP32 v_mfma_f32_16x16x4_f32 with lane (q, c) supplying
// A row c, k = 4q + t of each 16-wide chunk for MFMA t, and subtile j's
// column c being strip column JN c + j, so a lane reads its B values as one
// JN-wide vector; BF16 v_mfma_f32_16x16x32_bf16 with lane (q, c) supplying
// eight consecutive k (8q .. 8q+7) of A row c and of B column c, subtile j
// covering strip columns 16 j .. 16 j + 15.  Output fragments hold rows
// 4q .. 4q+3 of column c.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef unsigned short us;

constexpr int kThreads = 512;  // 8 waves: two per SIMD, so one wave's waits hide behind the other
constexpr int kWaves = kThreads / 64;
constexpr int BM = 16;
constexpr int kPadF32 = 4;  // FP32 strip row stride BN + 4: rows 4 apart land 16 banks apart

template <int JN>
struct Vec;
template <>
struct Vec<1> {
  typedef float T;
};
template <>
struct Vec<2> {
  typedef v2f T;
};
template <>
struct Vec<4> {
  typedef v4f T;
};

__device__ __forceinline__ float lane_of(float v, int) { return v; }
__device__ __forceinline__ float lane_of(v2f v, int j) { return v[j]; }
__device__ __forceinline__ float lane_of(v4f v, int j) { return v[j]; }

// LDS carve-up shared by host and device:
// [B strip][Y tiles][X slots][peel steps | subs | symbol table | ids | ytile]
struct FusedLds {
  size_t strip, astage, ytiles, slots, prog, total;
};
__host__ __device__ inline FusedLds fused_lds(const FusedParams& p) {
  FusedLds L;
  const int BN = 16 * p.jn;
  if (p.prec == BPX_PREC_F32)
    L.strip = (size_t)p.kp * (BN + kPadF32) * 4;
  else
    L.strip = (size_t)BN * (p.kp + 8) * 2 * (p.prec == BPX_PREC_BF16X3 ? 2 : 1);
  L.strip = (L.strip + 15) / 16 * 16;
  L.astage = 2 * (size_t)p.kb * BM * p.kg * 4;  // two buffers of the k group's A rows
  L.ytiles = (size_t)p.n_ytiles * BM * BN * 4;
  L.slots = (size_t)p.nslots * BM * BN * 4;
  L.prog = ((size_t)p.blob_words * 4 + 15) / 16 * 16;
  L.total = L.strip + L.astage + L.ytiles + L.slots + L.prog;
  return L;
}

// The program and the symbol tables, copied to LDS by the whole workgroup.
struct FusedTables {
  const PeelStep* steps;
  const int32_t* subs;
  const int32_t* syms;   // 4 per computed symbol: id offset, degree, dest, g
  const int32_t* ids;
  const int32_t* ytile;
};
// Issues the loads of the table span (16 bytes per thread and pass; the
// span starts 256-byte aligned), returns them for store_tables; a second
// pass covers spans past 16 KiB.
constexpr int kTabPass = 4;  // int4 per thread per pass
typedef int v4i __attribute__((ext_vector_type(4)));
struct TabLoads {
  v4i v[kTabPass];
};
__device__ __forceinline__ int tab_int4(const FusedParams& p) { return (p.blob_words + 3) / 4; }
__device__ __forceinline__ TabLoads load_tables(const FusedParams& p, int pass) {
  TabLoads t;
  const v4i* src = reinterpret_cast<const v4i*>(p.syms);
#pragma unroll
  for (int u = 0; u < kTabPass; ++u) {
    const int i = (pass * kTabPass + u) * kThreads + (int)threadIdx.x;
    t.v[u] = i < tab_int4(p) ? src[i] : v4i{0, 0, 0, 0};
  }
  return t;
}
__device__ __forceinline__ void store_tables(const FusedParams& p, int pass, const TabLoads& t,
                                             unsigned char* base) {
  v4i* dst = reinterpret_cast<v4i*>(base);
#pragma unroll
  for (int u = 0; u < kTabPass; ++u) {
    const int i = (pass * kTabPass + u) * kThreads + (int)threadIdx.x;
    if (i < tab_int4(p)) dst[i] = t.v[u];
  }
}
__device__ __forceinline__ FusedTables tables_at(const FusedParams& p, unsigned char* base) {
  const int32_t* w = reinterpret_cast<const int32_t*>(base);
  FusedTables t;
  t.syms = w;
  t.ids = w + p.off_ids;
  t.steps = reinterpret_cast<const PeelStep*>(w + p.off_steps);
  t.subs = w + p.off_subs;
  t.ytile = w + p.off_ytile;
  return t;
}
// Copies the tables to LDS; the first pass's loads are issued before the
// caller's B-strip loads (stage_begin), its stores after them.
__device__ __forceinline__ void tables_rest(const FusedParams& p, unsigned char* base) {
  for (int pass = 1; pass * kTabPass * kThreads < tab_int4(p); ++pass)
    store_tables(p, pass, load_tables(p, pass), base);
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Data blocks as raw buffer resources: block s covers the rows of data
// block s that exist (min(Mb, M - s Mb) rows of lda floats), so loads of
// rows past them return zero without a branch; a k past K is sent out of
// range as well.  The host keeps (Mb + 16) * lda * 4 and K * ldb * 4 below
// 2^31.
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer, 32-bit elements
constexpr uint32_t kOut = 0x80000000u;  // beyond any resource's range
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const FusedParams& p, int64_t s) {
  const int64_t rows = p.M - s * p.Mb < p.Mb ? p.M - s * p.Mb : p.Mb;
  const int bytes = rows > 0 ? (int)(rows * p.lda * 4) : 0;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p.A + s * p.Mb * p.lda), (short)0,
                                           bytes, kRsrcWord3);
}
// B as one buffer of K rows.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t b_rsrc(const FusedParams& p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p.B), (short)0,
                                           (int)(p.K * p.ldb * 4), kRsrcWord3);
}
__device__ __forceinline__ v4f bload(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

// Peel phase: every thread runs the whole program for its own elements.
// Steps carry src = the releaser's Y tile, and every recovered block is
// written to C (nothing reached C earlier).
__device__ __forceinline__ bool row_ok(const FusedParams& p, int64_t s, int64_t r) {
  return r < p.Mb && s * p.Mb + r < p.M;
}
__device__ __forceinline__ void fused_peel(const FusedParams& p, const float* yt, float* xs,
                                           const FusedTables& t, int r0, int n0, int BN) {
  const int tile = BM * BN;
  for (int e = threadIdx.x; e < tile; e += kThreads) {
    const int row = e / BN, col = e - row * BN;
    const int64_t r = r0 + row, n = n0 + col;
    for (int st = 0; st < p.nsteps; ++st) {
      const PeelStep S = t.steps[st];
      const float y = yt[S.src * tile + e];
      const int32_t* sub = t.subs + S.sub_off;
      float x;
      if (S.f64) {
        double acc = (double)y;
        for (int u = 0; u < S.nsub; ++u) acc -= (double)xs[sub[u] * tile + e];
        x = (float)acc;
      } else {
        float sum = y, comp = 0.f;
        for (int u = 0; u < S.nsub; ++u) {
          const float v = -xs[sub[u] * tile + e] - comp;
          const float tt = sum + v;
          comp = (tt - sum) - v;
          sum = tt;
        }
        x = sum;
      }
      if (S.slot >= 0) xs[S.slot * tile + e] = x;
      if (n < p.N && row_ok(p, S.s, r)) p.C[((int64_t)S.s * p.Mb + r) * p.ldc + n] = x;
    }
  }
}

// ------------------------------------------------------ the A stage ----
// Each k group (KG = 32 or 64 of k) of the tile's 16 rows of every data
// block is staged in LDS once and shared by all the symbols that sum it
// (double-buffered: the next group's loads are in flight while this group
// is multiplied).  Layout per buffer: [block][k half (32 k)][row][32
// floats], the 16-byte granule g of row r at slot g ^ ((r >> 1) & 7), so
// that the 16 rows a fragment read touches fall on distinct bank groups.
__device__ __forceinline__ int a_slot(int row, int granule) {
  return granule ^ ((row >> 1) & 7);
}
// Per-thread plan of the A-stage loads, fixed for the whole K loop: load u
// of this thread is float4 item f = u kThreads + tid of the group, item f
// being (block, row, c4) with 16 KG / 4 items per block, a multiple of the
// wave size, so each wave's block is uniform and its resource scalar; only
// the k offset changes from group to group.
constexpr int kAPer = 4;  // float4 per thread per group (kb KG <= 512)
template <int KG>
struct AStage {
  static constexpr int kPerBlock = BM * KG / 4;
  static constexpr int kHalves = KG / 32;
  static constexpr int kFloats = BM * KG;  // one block's rows in a stage
  __amdgpu_buffer_rsrc_t rs[kAPer];
  uint32_t goff[kAPer];  // byte offset of the row in its block, plus 16 c4
  int kof[kAPer];        // k of the item within the group (4 c4)
  int soff[kAPer];       // float offset of the item in a stage
  bool ok[kAPer];
  __device__ void init(const FusedParams& p, int r0) {
    const int items = p.kb * kPerBlock;
#pragma unroll
    for (int u = 0; u < kAPer; ++u) {
      const int f = u * kThreads + (int)threadIdx.x;
      ok[u] = f < items;
      const int blk = uniform(min(f, items - 1) / kPerBlock);
      const int rem = f - blk * kPerBlock;
      const int row = rem / (KG / 4), c4 = rem % (KG / 4);
      rs[u] = block_rsrc(p, blk);
      goff[u] = 4u * (uint32_t)((r0 + row) * (int)p.lda);
      kof[u] = 4 * c4;
      soff[u] = blk * kFloats + ((c4 >> 3) * BM + row) * 32 + 4 * a_slot(row, c4 & 7);
    }
  }
  __device__ void issue(const FusedParams& p, int grp, v4f* v) const {
#pragma unroll
    for (int u = 0; u < kAPer; ++u) {
      const int k = grp * KG + kof[u];
      v[u] = bload(rs[u], (ok[u] && k < p.K) ? goff[u] + 4u * (uint32_t)k : kOut);
    }
  }
  __device__ void store(const v4f* v, float* As) const {
#pragma unroll
    for (int u = 0; u < kAPer; ++u)
      if (ok[u]) *reinterpret_cast<v4f*>(As + soff[u]) = v[u];
  }
};
// Granule g (k = 4 g .. 4 g + 3 of k half h) of the tile's row `row` of
// data block blk in an A stage.
template <int KG>
__device__ __forceinline__ v4f a_granule(const float* As, int blk, int h, int row, int g) {
  return *reinterpret_cast<const v4f*>(As + blk * AStage<KG>::kFloats + (h * BM + row) * 32 +
                                       4 * a_slot(row, g));
}

// The symbols of a wave: i = wave + 8 j for j < kMS, with their degree,
// member blocks (ascending) and Y tile held in scalar registers.
constexpr int kMS = 2;      // symbols per wave at most (16 per workgroup)
constexpr int kMaxDeg = 4;  // members per symbol at most
struct WaveSyms {
  int n;
  int deg[kMS];
  int ytile[kMS];
  int id[kMS][kMaxDeg];
};
__device__ __forceinline__ WaveSyms wave_syms(const FusedParams& p, const FusedTables& t) {
  WaveSyms w;
  const int wave = uniform((int)threadIdx.x >> 6);
  w.n = wave < p.n_sym ? (p.n_sym - wave + kWaves - 1) / kWaves : 0;
#pragma unroll
  for (int j = 0; j < kMS; ++j) {
    const int i = wave + kWaves * j;
    const bool ok = j < w.n;
    const int off = ok ? uniform(t.syms[4 * i + 0]) : 0;
    w.deg[j] = ok ? uniform(t.syms[4 * i + 1]) : 0;
    w.ytile[j] = ok ? uniform(t.ytile[i]) : -1;
#pragma unroll
    for (int m = 0; m < kMaxDeg; ++m) w.id[j][m] = m < w.deg[j] ? uniform(t.ids[off + m]) : 0;
  }
  return w;
}

// The K loop over k groups: group g is multiplied from stage g & 1 while
// the loads of groups g+1 and g+2 are in flight (registers hold[] and
// fresh[]); group g+1 is stored to the other stage after group g's MFMAs,
// and a barrier ends each group.  Loads get two groups of MFMAs to arrive.
template <int KG, typename F>
__device__ __forceinline__ void pipeline(int ng, int stage, float* As0, const AStage<KG>& ast,
                                         const FusedParams& p, v4f* r1, v4f* r2, F& compute) {
  auto step = [&](int g, v4f* hold, v4f* fresh) __attribute__((always_inline)) {
    if (g + 2 < ng) ast.issue(p, g + 2, fresh);
    compute(g);
    if (g + 1 < ng) ast.store(hold, As0 + ((g + 1) & 1) * stage);
    __syncthreads();
  };
  for (int g = 0; g < ng; g += 2) {
    step(g, r1, r2);
    if (g + 1 < ng) step(g + 1, r2, r1);
  }
}

// ------------------------------------------------------------------ FP32 --
template <int JN, int KG>
__global__ __launch_bounds__(kThreads) void fused_f32_kernel(FusedParams p) {
  constexpr int BN = 16 * JN, LDB = BN + kPadF32;
  typedef typename Vec<JN>::T vb;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const FusedLds L = fused_lds(p);
  float* Bs = reinterpret_cast<float*>(lds_raw);
  float* As0 = reinterpret_cast<float*>(lds_raw + L.strip);
  float* yt = reinterpret_cast<float*>(lds_raw + L.strip + L.astage);
  float* xs = reinterpret_cast<float*>(lds_raw + L.strip + L.astage + L.ytiles);
  unsigned char* tab_lds = lds_raw + L.strip + L.astage + L.ytiles + L.slots;

  const int tn = (int)blockIdx.x % p.tiles_n, tm = (int)blockIdx.x / p.tiles_n;
  const int r0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int ng = (int)(p.kp / KG);
  AStage<KG> ast;
  ast.init(p, r0);

  // Prologue: tables, B strip and the first A group; all loads of a pass
  // are issued before any of them is stored.  B strip, k in [0, kp): item f
  // is float4 (row k, columns 4 c4 ..); rows past K read out of range
  // (zero), a float4 reaching past N stays inside the row's leading
  // dimension and its extra columns are zeroed.
  {
    constexpr int SB = 8;  // float4 per thread per pass
    const int items = (int)p.kp * (BN / 4);
    const auto rb = b_rsrc(p);
    const TabLoads t0 = load_tables(p, 0);
    v4f a0[kAPer];
    ast.issue(p, 0, a0);
    for (int base = 0; base < items; base += SB * kThreads) {
      v4f v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int f = base + u * kThreads + tid;
        const int k = f / (BN / 4), c4 = (f - k * (BN / 4)) * 4;
        const int n = n0 + c4;
        v[u] = bload(rb, (f < items && k < p.K) ? 4u * (uint32_t)(k * (int)p.ldb + n) : kOut);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e >= p.N) v[u][e] = 0.f;
      }
      if (base == 0) {
        store_tables(p, 0, t0, tab_lds);
        ast.store(a0, As0);
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int f = base + u * kThreads + tid;
        const int k = f / (BN / 4), c4 = (f - k * (BN / 4)) * 4;
        if (f < items) *reinterpret_cast<v4f*>(Bs + k * LDB + c4) = v[u];
      }
    }
    tables_rest(p, tab_lds);
  }
  v4f r1[kAPer], r2[kAPer];  // the next two groups' A loads in flight
  if (ng > 1) ast.issue(p, 1, r1);
  __syncthreads();
  const FusedTables tab = tables_at(p, tab_lds);
  const WaveSyms ws = wave_syms(p, tab);

  v4f acc[kMS][JN];
#pragma unroll
  for (int j = 0; j < kMS; ++j)
#pragma unroll
    for (int jj = 0; jj < JN; ++jj) acc[j][jj] = v4f{0.f, 0.f, 0.f, 0.f};
  const int stage = p.kb * AStage<KG>::kFloats;
  auto compute = [&](int grp) __attribute__((always_inline)) {
    const float* As = As0 + (grp & 1) * stage;
    // Symbol j's whole k group with its degree D known at compile time (one
    // scalar branch on the wave-uniform degree per group): the D granule
    // reads of a chunk issue together, the next chunk's reads can go out
    // under this chunk's MFMAs, and the members are summed in ascending
    // order, unmasked.
    auto group = [&](int j, auto deg) __attribute__((always_inline)) {
      constexpr int D = decltype(deg)::value;
#pragma unroll
      for (int c = 0; c < KG / 16; ++c) {  // 16-wide k chunks
        const int h = c >> 1, g = (c & 1) * 4 + q;
        vb b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          b[t] = *reinterpret_cast<const vb*>(Bs + (grp * KG + 16 * c + 4 * q + t) * LDB +
                                              JN * c16);
        v4f gr[D];
#pragma unroll
        for (int m = 0; m < D; ++m) gr[m] = a_granule<KG>(As, ws.id[j][m], h, c16, g);
        v4f a = gr[0];
#pragma unroll
        for (int m = 1; m < D; ++m) a += gr[m];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int jj = 0; jj < JN; ++jj)
            acc[j][jj] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], lane_of(b[t], jj), acc[j][jj], 0, 0, 0);
      }
    };
#pragma unroll
    for (int j = 0; j < kMS; ++j) {
      if (j >= ws.n) break;
      const int d = ws.deg[j];
      if (d == 1)
        group(j, std::integral_constant<int, 1>{});
      else if (d == 2)
        group(j, std::integral_constant<int, 2>{});
      else if (d == 3)
        group(j, std::integral_constant<int, 3>{});
      else if (d == kMaxDeg)
        group(j, std::integral_constant<int, kMaxDeg>{});
      // (a symbol with no members adds nothing: its product stays zero)
    }
  };
  pipeline(ng, stage, As0, ast, p, r1, r2, compute);
#pragma unroll
  for (int j = 0; j < kMS; ++j) {
    if (j >= ws.n || ws.ytile[j] < 0) continue;
#pragma unroll
    for (int jj = 0; jj < JN; ++jj)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        yt[(ws.ytile[j] * BM + 4 * q + rr) * BN + JN * c16 + jj] = acc[j][jj][rr];
  }
  __syncthreads();
  fused_peel(p, yt, xs, tab, r0, n0, BN);
}

// ------------------------------------------------------- BF16 / BF16x3 --
// hi = bf16(x) and lo = bf16(x - hi), both round to nearest even, converted
// two values at a time (one v_cvt_pk_bf16_f32 per pair; the same roundings
// as converting each value alone).
__device__ __forceinline__ void split2(float x, float y, __bf16* h, __bf16* l) {
  const v2f p = {x, y};
  const v2bf hp = __builtin_convertvector(p, v2bf);
  const v2bf lp = __builtin_convertvector(p - __builtin_convertvector(hp, v2f), v2bf);
  h[0] = hp[0];
  h[1] = hp[1];
  l[0] = lp[0];
  l[1] = lp[1];
}
__device__ __forceinline__ void split8(v4f x0, v4f x1, v8bf* hi, v8bf* lo) {
  __bf16 h[8], l[8];
#pragma unroll
  for (int e = 0; e < 4; e += 2) {
    split2(x0[e], x0[e + 1], h + e, l + e);
    split2(x1[e], x1[e + 1], h + 4 + e, l + 4 + e);
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    (*hi)[e] = h[e];
    (*lo)[e] = l[e];
  }
}

template <int JN, bool X3, int KG>
__global__ __launch_bounds__(kThreads) void fused_bf16_kernel(FusedParams p) {
  constexpr int BN = 16 * JN;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const FusedLds L = fused_lds(p);
  const int KS = p.kp + 8;  // strip row stride (bf16): one column's k run, padded 16 bytes
  us* Bh = reinterpret_cast<us*>(lds_raw);
  us* Bl = Bh + (size_t)BN * KS;
  float* As0 = reinterpret_cast<float*>(lds_raw + L.strip);
  float* yt = reinterpret_cast<float*>(lds_raw + L.strip + L.astage);
  float* xs = reinterpret_cast<float*>(lds_raw + L.strip + L.astage + L.ytiles);
  unsigned char* tab_lds = lds_raw + L.strip + L.astage + L.ytiles + L.slots;

  const int tn = (int)blockIdx.x % p.tiles_n, tm = (int)blockIdx.x / p.tiles_n;
  const int r0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int ng = (int)(p.kp / KG);
  AStage<KG> ast;
  ast.init(p, r0);

  // Prologue as in the FP32 kernel.  B strip, transposed and split: item f
  // is column col and eight consecutive k (one 16-byte LDS store per
  // plane); rows past K and columns past N are zero.
  {
    constexpr int SB = 4;  // items per thread per pass (eight loads each)
    const int items = BN * (int)(p.kp / 8);
    const auto rb = b_rsrc(p);
    const TabLoads t0 = load_tables(p, 0);
    v4f a0[kAPer];
    ast.issue(p, 0, a0);
    for (int base = 0; base < items; base += SB * kThreads) {
      float v[SB][8];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int f = base + u * kThreads + tid;
        const int col = f % BN, k0 = (f / BN) * 8;
        const int n = n0 + col;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[u][e] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(
                         rb, (int)((f < items && k0 + e < p.K && n < p.N)
                                       ? 4u * (uint32_t)((k0 + e) * (int)p.ldb + n)
                                       : kOut),
                         0, 0));
      }
      if (base == 0) {
        store_tables(p, 0, t0, tab_lds);
        ast.store(a0, As0);
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int f = base + u * kThreads + tid;
        if (f >= items) continue;
        const int col = f % BN, k0 = (f / BN) * 8;
        v8bf hi, lo;
        split8(v4f{v[u][0], v[u][1], v[u][2], v[u][3]}, v4f{v[u][4], v[u][5], v[u][6], v[u][7]},
               &hi, &lo);
        *reinterpret_cast<v8bf*>(Bh + (size_t)col * KS + k0) = hi;
        if (X3) *reinterpret_cast<v8bf*>(Bl + (size_t)col * KS + k0) = lo;
      }
    }
    tables_rest(p, tab_lds);
  }
  v4f r1[kAPer], r2[kAPer];  // the next two groups' A loads in flight
  if (ng > 1) ast.issue(p, 1, r1);
  __syncthreads();
  const FusedTables tab = tables_at(p, tab_lds);
  const WaveSyms ws = wave_syms(p, tab);

  v4f acc[kMS][JN];
#pragma unroll
  for (int j = 0; j < kMS; ++j)
#pragma unroll
    for (int jj = 0; jj < JN; ++jj) acc[j][jj] = v4f{0.f, 0.f, 0.f, 0.f};
  const int stage = p.kb * AStage<KG>::kFloats;
  auto compute = [&](int grp) __attribute__((always_inline)) {
    const float* As = As0 + (grp & 1) * stage;
    // Symbol j's whole k group with its degree D known at compile time (see
    // the FP32 kernel); the chunk body is VALU work (sums and splits) next
    // to three MFMAs, so every masked add saved counts.
    auto group = [&](int j, auto deg) __attribute__((always_inline)) {
      constexpr int D = decltype(deg)::value;
#pragma unroll
      for (int h = 0; h < KG / 32; ++h) {  // 32-wide k chunks: lane takes k = 8q .. 8q+7
        v8bf bh[JN], bl[JN];
#pragma unroll
        for (int jj = 0; jj < JN; ++jj) {
          const size_t off = (size_t)(16 * jj + c16) * KS + grp * KG + 32 * h + 8 * q;
          bh[jj] = *reinterpret_cast<const v8bf*>(Bh + off);
          if (X3) bl[jj] = *reinterpret_cast<const v8bf*>(Bl + off);
        }
        v4f g0[D], g1[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
          g0[m] = a_granule<KG>(As, ws.id[j][m], h, c16, 2 * q);
          g1[m] = a_granule<KG>(As, ws.id[j][m], h, c16, 2 * q + 1);
        }
        v4f a0 = g0[0], a1 = g1[0];
#pragma unroll
        for (int m = 1; m < D; ++m) {
          a0 += g0[m];
          a1 += g1[m];
        }
        v8bf ah, al;
        split8(a0, a1, &ah, &al);
#pragma unroll
        for (int jj = 0; jj < JN; ++jj) {
          if (X3) {
            acc[j][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[jj], acc[j][jj], 0, 0, 0);
            acc[j][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[jj], acc[j][jj], 0, 0, 0);
          }
          acc[j][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[jj], acc[j][jj], 0, 0, 0);
        }
      }
    };
#pragma unroll
    for (int j = 0; j < kMS; ++j) {
      if (j >= ws.n) break;
      const int d = ws.deg[j];
      if (d == 1)
        group(j, std::integral_constant<int, 1>{});
      else if (d == 2)
        group(j, std::integral_constant<int, 2>{});
      else if (d == 3)
        group(j, std::integral_constant<int, 3>{});
      else if (d == kMaxDeg)
        group(j, std::integral_constant<int, kMaxDeg>{});
      // (a symbol with no members adds nothing: its product stays zero)
    }
  };
  pipeline(ng, stage, As0, ast, p, r1, r2, compute);
#pragma unroll
  for (int j = 0; j < kMS; ++j) {
    if (j >= ws.n || ws.ytile[j] < 0) continue;
#pragma unroll
    for (int jj = 0; jj < JN; ++jj)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        yt[(ws.ytile[j] * BM + 4 * q + rr) * BN + 16 * jj + c16] = acc[j][jj][rr];
  }
  __syncthreads();
  fused_peel(p, yt, xs, tab, r0, n0, BN);
}

typedef void (*FusedKernel)(FusedParams);

template <int KG>
FusedKernel fused_kernel_kg(int32_t prec, int jn) {
  if (prec == BPX_PREC_F32)
    return jn == 1 ? fused_f32_kernel<1, KG>
                   : jn == 2 ? fused_f32_kernel<2, KG> : fused_f32_kernel<4, KG>;
  // BF16 tiles stop at 32 columns (wider ones spill at eight waves)
  if (prec == BPX_PREC_BF16)
    return jn == 1 ? fused_bf16_kernel<1, false, KG>
                   : jn == 2 ? fused_bf16_kernel<2, false, KG> : nullptr;
  if (prec == BPX_PREC_BF16X3)
    return jn == 1 ? fused_bf16_kernel<1, true, KG>
                   : jn == 2 ? fused_bf16_kernel<2, true, KG> : nullptr;
  return nullptr;
}
FusedKernel fused_kernel_for(int32_t prec, int jn, int kg) {
  return kg == 64 ? fused_kernel_kg<64>(prec, jn) : fused_kernel_kg<32>(prec, jn);
}

constexpr size_t kLdsLimit = 160 * 1024;

}  // namespace

// Column tile width 16 JN: the widest (fewest re-reads of A) that still
// gives every compute unit a workgroup, else 16; it must fit LDS.
bool fused_configure(FusedParams* p) {
  if (p->prec != BPX_PREC_F32 && p->prec != BPX_PREC_BF16 && p->prec != BPX_PREC_BF16X3)
    return false;
  // k group of the A stage: 64 where 16 rows of every block fit twice in
  // 64 KiB, else 32; the B strip is zero-padded to a whole group
  if (p->kb > 16 || p->n_sym > kWaves * kMS || p->max_deg > kMaxDeg) return false;
  p->kg = p->kb <= 8 ? 64 : 32;
  p->kp = (p->K + p->kg - 1) / p->kg * p->kg;
  // 32-bit buffer offsets: a block of A plus one tile's rows, all of B
  if ((p->Mb + BM) * p->lda * 4 >= ((int64_t)1 << 31)) return false;
  if ((p->K + 1) * p->ldb * 4 >= ((int64_t)1 << 31)) return false;
  const int64_t tiles_m = (p->Mb + BM - 1) / BM;
  const int64_t cus = device_cu_count();
  for (int jn : {4, 2, 1}) {
    if (!fused_kernel_for(p->prec, jn, p->kg)) continue;
    p->jn = jn;
    const int64_t tiles_n = (p->N + 16 * jn - 1) / (16 * jn);
    if (jn > 1 && tiles_m * tiles_n < cus) continue;
    if (fused_lds(*p).total > kLdsLimit) continue;
    if (tiles_m * tiles_n > 0x7fffffff) return false;
    p->tiles_n = (int32_t)tiles_n;
    p->tiles_m = (int32_t)tiles_m;
    return true;
  }
  return false;
}

size_t fused_lds_bytes(const FusedParams& p) { return fused_lds(p).total; }

hipError_t launch_fused(const FusedParams& p, hipStream_t stream) {
  const FusedKernel k = fused_kernel_for(p.prec, p.jn, p.kg);
  if (!k) return hipErrorInvalidValue;
  const size_t lds = fused_lds(p).total;
  if (lds > kLdsLimit) return hipErrorInvalidConfiguration;
  const int64_t blocks = (int64_t)p.tiles_m * p.tiles_n;
  if (blocks == 0 || p.nsteps == 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), lds, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
