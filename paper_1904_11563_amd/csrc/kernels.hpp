// Device kernels of libbpx: parameter blocks and host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "host.hpp"

namespace bpx {

// Coded GEMM: for every computed symbol i (table entry {id_off, deg, dest, g}
// in syms[4*i..4*i+3], member ids in ids[id_off .. id_off+deg)),
//   out_i = (sum over members s of A rows [s*Mb, s*Mb+Mb)) . B
// where out_i is Y slot dest (Mb x N, ld N) or, for dest < 0, the C rows of
// block -1-dest (ld ldc, rows past M skipped).
struct GemmParams {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  float* Y;
  int64_t M, K, N, Mb;
  const int32_t* syms;
  const int32_t* ids;
  int32_t n_sym;
  int32_t tiles_m, tiles_n;
  int32_t prec;  // bpx_prec
  int32_t group_m;  // tile order: row panels per group (1 = row-major order)
  // Remainder mode of the 256 x 256 tiling (FP32 only): when wide_rem is set,
  // tiles_m / tiles_n count 256 x 256 tiles and block b computes sub-tile
  // b % per of 256 x 256 tile wide_lin0 + b / per (per = sub-tiles per tile).
  int32_t wide_rem;
  int32_t wide_lin0;
  // Split-K mode of the 256 x 256 tiling: when wide_split = P > 0, block b
  // computes k-slice range (b % P) of tile wide_lin0 + b / P into partial
  // tile b of part (256 x 256 FP32, row-major); a reduction kernel sums the
  // P partials of each tile in piece order and writes the tile's output.
  int32_t wide_split;
  int32_t part_tiles;  // capacity of part in 256 x 256 tiles (0: no split-K)
  float* part;
  // Two-dimensional form (launch_coded_gemm_2d): data block s = r * grid + c
  // is A row block r times B column block c; Y slots are Mb x Nb.
  int32_t grid;
  int32_t pad1;
  int64_t Nb;
  // BF16 / BF16x3: B split into transposed bf16 planes (N x kp, k contiguous)
  const unsigned short* bt_hi;
  const unsigned short* bt_lo;
  int64_t kp;
};

// FP8 path (see gemm_fp8.hip for the workspace layout).
struct Fp8Params {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  float* Y;
  int64_t M, K, N, Mb;
  int64_t Mbp, Kp, Np;  // Mb, K, N rounded up to 128
  const int32_t* syms;
  const int32_t* ids;
  int32_t n_sym;
  int32_t tiles_m, tiles_n;
  unsigned char* aq;
  unsigned char* aq2;  // null unless FP8x2
  float* sa;
  unsigned char* bq;
  float* sb;
  int32_t group_m;  // wide tiles: row panels per group of the tile order (0: default)
};

// Peel: see PeelStep in host.hpp.
struct PeelParams {
  const float* Y;
  float* C;
  int64_t ldc;
  int64_t M, N, Mb;
  const PeelStep* steps;
  const int32_t* subs;
  int32_t nsteps;
  int32_t nslots;
  int32_t nsubs;  // length of subs
  // Block layout: data block s covers C rows (s / grid) * Mb .., columns
  // (s % grid) * Nb ..; Y slots are Mb x Nb.  grid = 1, Nb = N for row
  // blocks (the vector form assumes that layout).
  int32_t grid;
  int64_t Nb;
};
// Bytes of LDS a peel workgroup holds besides its slots: the step program
// (steps, then subs), staged once per workgroup.
__host__ __device__ inline size_t peel_program_bytes(int32_t nsteps, int32_t nsubs) {
  return ((size_t)nsteps * sizeof(PeelStep) + (size_t)nsubs * 4 + 15) / 16 * 16;
}

// Standalone encode: out block i (Mb x K, ld K) = sum of member blocks of A.
struct EncodeParams {
  const float* A;
  int64_t lda;
  float* out;
  int64_t M, K, Mb;
  const int32_t* syms;
  const int32_t* ids;
  int32_t n_sym;
};

// Tile shapes compiled for the GEMM.
struct TileShape {
  int32_t bm, bn, bk;
};
int32_t gemm_tile_count();
TileShape gemm_tile_shape(int32_t t);

hipError_t launch_coded_gemm(const GemmParams& p, int32_t tile, hipStream_t stream);
// FP32 coded GEMM of the two-dimensional form (64 x 128 tiles).
// tile: the FP32 tile shape chosen for the call; the 256 x 256 shapes (4-6)
// take the wide 2-D kernel where the blocks allow it, others 64 x 128.
hipError_t launch_coded_gemm_2d(const GemmParams& p, int32_t tile, hipStream_t stream);

int32_t bf16_tile_count();
TileShape bf16_tile_shape(int32_t t);
// Tile 4 is the flat-row tiling (tiles over all symbols' stacked rows); it
// needs K a multiple of 32 and offsets within 31 bits (bf16_flat_ok).
bool bf16_tile_is_flat(int32_t t);
bool bf16_flat_ok(const GemmParams& p);
// Bt_hi[n][k] = bf16(B[k][n]), Bt_lo = bf16(B - Bt_hi) (bt_lo may be null),
// zero for k in [K, Kp).
hipError_t launch_split_b(const float* B, int64_t ldb, int64_t K, int64_t N, int64_t Kp,
                          void* bt_hi, void* bt_lo, hipStream_t stream);
hipError_t launch_coded_gemm_bf16(const GemmParams& p, int32_t tile, hipStream_t stream);
// ------------------------------------------------------------ grouped --
// Per-product descriptor of a grouped launch (device memory).
struct GroupDesc {
  GemmParams g;      // tiles_m / tiles_n set for the product's tile shape
  PeelParams pe;
  int32_t b_tn, b_tk;  // split-B grid of the product (64 x 64 tiles)
  int32_t tile;        // tile shape index
  int32_t pad;
};
// A grouped GEMM tile: product and tile index inside that product's grid.
struct GroupTile {
  int32_t prod;
  int32_t lin;
};
// Grouped split-B: block b belongs to product bmap[b] and is block
// b - bstart[bmap[b]] of that product's grid.
hipError_t launch_split_b_grouped(const GroupDesc* d, const int64_t* bstart, const int32_t* bmap,
                                  int64_t total_blocks, hipStream_t stream);
// Persistent grouped BF16 / BF16x3 GEMM over a tile list of one tile shape.
hipError_t launch_gemm_bf16_grouped(const GroupDesc* d, const GroupTile* tiles, int32_t n_tiles,
                                    int32_t tile, int32_t split, int32_t grid,
                                    hipStream_t stream);
// Compute units of the current device (cached per device; 256 if unknown).
int device_cu_count();

// Grouped peel: block b belongs to product pmap[b] and is block
// b - pstart[pmap[b]] of that product's peel grid; workgroup w of the
// persistent grid runs blocks wstart[w] .. wstart[w + 1] - 1.  The grid is
// peel_grouped_grid(...) workgroups (as many as the CUs hold at once).
int64_t peel_grouped_grid(int64_t total_blocks, int32_t max_slots, size_t max_program);
hipError_t launch_peel_grouped(const GroupDesc* d, const int64_t* pstart, const int32_t* pmap,
                               const int64_t* wstart, int64_t grid, int32_t max_slots,
                               size_t max_program, hipStream_t stream);

// ------------------------------------------------------ fused peel --
// One launch computing every computed symbol's product for a 16 x BN output
// tile of all data blocks and peeling it in LDS (see fused.hip).  syms/ids
// as in GemmParams (GEMM-table order); ytile[i]: the LDS Y tile of computed
// symbol i, or -1 if it releases nothing; steps/subs: the fused peel
// program (src = Y tile of the releaser, every recovered block written).
struct FusedParams {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  int64_t M, K, N, Mb;
  const int32_t* syms;
  const int32_t* ids;
  const int32_t* ytile;
  int32_t n_sym;
  int32_t n_ytiles;
  int32_t n_ids;  // length of ids
  // The plan's device tables are one block; the kernel copies the span from
  // syms to the end of ytile to LDS in one pass (word offsets from syms).
  int32_t blob_words;
  int32_t off_ids, off_steps, off_subs, off_ytile;
  const PeelStep* steps;
  const int32_t* subs;
  int32_t nsteps;
  int32_t nsubs;
  int32_t nslots;
  int32_t prec;
  // set by fused_configure
  int32_t jn;  // column tile = 16 jn
  int32_t tiles_m, tiles_n;
  int32_t kb;       // data blocks
  int32_t max_deg;  // largest degree of a computed symbol
  int32_t kg;       // k per A-stage group (32 or 64)
  int32_t pad;
  int64_t kp;  // K rounded up to the k group
};
// Picks the tile width and checks that the workgroup's LDS fits; false if
// the fused form cannot run this product (precision or LDS).
bool fused_configure(FusedParams* p);
size_t fused_lds_bytes(const FusedParams& p);
hipError_t launch_fused(const FusedParams& p, hipStream_t stream);

hipError_t launch_quant_a(const Fp8Params& p, hipStream_t stream);
hipError_t launch_quant_b(const Fp8Params& p, hipStream_t stream);
int32_t fp8_tile_count();
hipError_t launch_coded_gemm_fp8(const Fp8Params& p, int32_t tile, hipStream_t stream);
hipError_t launch_peel(const PeelParams& p, hipStream_t stream);
hipError_t launch_encode(const EncodeParams& p, hipStream_t stream);

}  // namespace bpx
