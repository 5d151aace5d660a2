// Host-side objects of libbpx: codes, plans, and the device tables a plan
// uploads.  Integer work only; no HIP types appear here.
#pragma once

#include "../../include/bpx.h"

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

struct bpx_code {
  int32_t kind = 0;
  int32_t n = 0, k = 0, b = 0;
  std::vector<int32_t> col_ptr;   // n + 1
  std::vector<int32_t> sym_ptr;   // n_sym + 1
  std::vector<uint16_t> sym_data; // ids, ascending per symbol
  int32_t n_sym() const { return (int32_t)sym_ptr.size() - 1; }
  int32_t kb() const { return k * b; }
  int32_t deg(int32_t g) const { return sym_ptr[g + 1] - sym_ptr[g]; }
  int32_t max_degree() const;
};

// One step of the device peel program (see plan.cpp).
struct PeelStep {
  int32_t s;        // data block written / loaded
  int32_t src;      // Y slot of the releaser, or -1 when X_s already sits in C
  int32_t nsub;     // number of subtrahends
  int32_t sub_off;  // offset of the subtrahends' LDS slots in the slot list
  int32_t f64;      // 1: accumulate in FP64 (depth > 4), 0: FP32 Kahan
  int32_t slot;     // LDS slot that keeps X_s for later steps, or -1
  int32_t write;    // 1: write X_s to C
  int32_t brow;     // block row of s (s itself for row blocks)
  int32_t bcol;     // block column of s (0 for row blocks)
};

struct bpx_plan {
  // copy of the code (a plan outlives nothing it does not own)
  bpx_code code;
  int32_t mode = 0, prec = 0;
  int64_t M = 0, K = 0, N = 0, Mb = 0;
  // Two-dimensional form: data block s = r * grid + c is A row block r times
  // B column block c (Mb rows, Nb columns); grid = 1 is the row-block form
  // (Nb = N).
  int32_t grid = 1;
  int64_t Nb = 0;

  bool decodable = false;
  int32_t prefix_m = 0;
  int32_t depth_max = 0;
  std::vector<int32_t> computed;    // ascending g
  std::vector<int32_t> dest;        // per computed: Y slot or -1-s
  std::vector<int32_t> releaser;    // per data id
  std::vector<int32_t> depth;       // per data id
  std::vector<int32_t> sub_ptr;     // kb + 1
  std::vector<uint16_t> sub_data;
  std::vector<int32_t> unrecovered;
  int32_t n_yslots = 0;

  // device peel program
  std::vector<PeelStep> steps;
  std::vector<int32_t> step_subs;   // LDS slots of subtrahends
  int32_t n_lds_slots = 0;

  // GEMM symbol table: per computed symbol {id_off, deg, dest, 0} + ids
  std::vector<int32_t> gemm_syms;
  std::vector<int32_t> gemm_ids;

  // Fused peel program (every recovered block has a step; src is the
  // releaser's LDS Y tile) and, per GEMM-table entry, its Y tile or -1.
  std::vector<PeelStep> fused_steps;
  std::vector<int32_t> fused_subs;
  std::vector<int32_t> fused_ytile;
  int32_t n_ytiles = 0;

  // device copies
  void* dev_block = nullptr;
  int32_t dev_id = -1;
  const int32_t* d_gemm_syms = nullptr;
  const int32_t* d_gemm_ids = nullptr;
  const PeelStep* d_steps = nullptr;
  const int32_t* d_step_subs = nullptr;
  const PeelStep* d_fused_steps = nullptr;
  const int32_t* d_fused_subs = nullptr;
  const int32_t* d_fused_ytile = nullptr;

  size_t y_bytes() const { return (size_t)n_yslots * (size_t)Mb * (size_t)Nb * sizeof(float); }
  // K rounded up to the BF16 kernels' 32-wide k step
  int64_t kp() const { return (K + 31) / 32 * 32; }
  static size_t align256(size_t x) { return (x + 255) / 256 * 256; }
  // Workspace: [Y slots][Bt_hi][Bt_lo] for the BF16 precisions.
  size_t bt_plane_bytes() const { return align256((size_t)N * (size_t)kp() * 2); }
  // FP8: [Y][Aq][Aq2][sA][Bq][sB] with Mb, K, N rounded up to 128.
  int64_t r128(int64_t x) const { return (x + 127) / 128 * 128; }
  bool is_fp8() const { return prec == BPX_PREC_FP8 || prec == BPX_PREC_FP8X2; }
  bool is_bf16() const { return prec == BPX_PREC_BF16 || prec == BPX_PREC_BF16X3; }
  // FP32 plans whose shape takes the 256 x 256 tiling reserve room for the
  // split-K partial tiles of its last round: at most 4 pieces per tile and
  // at most 256 partial tiles (one per CU) of 256 x 256 FP32.
  size_t part_bytes() const {
    if (grid != 1 || prec != BPX_PREC_F32 || Mb % 256 != 0 || N % 256 != 0 || K % 32 != 0 ||
        M % Mb != 0)
      return 0;
    const int64_t T = (int64_t)computed.size() * (Mb / 256) * (N / 256);
    const int64_t tiles = T * 4 < 256 ? T * 4 : 256;
    return (size_t)tiles * 256 * 256 * sizeof(float);
  }
  // Offsets in bytes of the workspace parts:
  //   F32:    [0] Y, [1] split-K partial tiles (256 x 256 tiling only)
  //   BF16*:  [0] Y, [1] Bt_hi, [2] Bt_lo (BF16x3)
  //   FP8*:   [0] Y, [1] Aq, [2] Aq2 (FP8x2), [3] sA, [4] Bq, [5] sB
  // Missing parts get the offset of the next part (size 0).  [6] = total.
  void layout(size_t off[7]) const {
    size_t b = align256(y_bytes());
    for (int i = 0; i < 7; ++i) off[i] = 0;
    if (is_bf16()) {
      off[1] = b;
      b += bt_plane_bytes();
      off[2] = b;
      if (prec == BPX_PREC_BF16X3) b += bt_plane_bytes();
      for (int i = 3; i < 7; ++i) off[i] = b;
    } else if (is_fp8()) {
      const size_t nc = computed.size();
      const size_t aq = align256(nc * (size_t)r128(Mb) * (size_t)r128(K));
      off[1] = b;
      b += aq;
      off[2] = b;
      if (prec == BPX_PREC_FP8X2) b += aq;
      off[3] = b;
      b += align256(nc * (size_t)(r128(Mb) / 128) * (size_t)(r128(K) / 128) * 4);
      off[4] = b;
      b += align256((size_t)r128(N) * (size_t)r128(K));
      off[5] = b;
      b += align256((size_t)(r128(K) / 128) * (size_t)(r128(N) / 128) * 4);
      off[6] = b;
    } else {
      off[1] = b;
      b += part_bytes();
      for (int i = 2; i < 7; ++i) off[i] = b;
    }
    off[6] = b;
  }
  size_t ws_bytes() const {
    size_t off[7];
    layout(off);
    return off[6];
  }
};

namespace bpx {

// SplitMix64 (Steele, Lea, Flood 2014).
struct SplitMix64 {
  uint64_t state;
  explicit SplitMix64(uint64_t seed) : state(seed) {}
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint64_t below(uint64_t n) { return next() % n; }
};

// Thread-local error message.
void set_error(const std::string& msg);
const char* get_error();

// code.cpp
int build_code(const bpx_code_params& p, bpx_code* out, std::string* err);

// plan.cpp
struct PeelResult {
  std::vector<int32_t> releaser;  // -1 = unknown
  std::vector<int32_t> depth;
  int32_t n_known = 0;
  int32_t rounds = 0;
};
// Round-based peel over the given symbols (ids into code), canonical releaser.
PeelResult peel(const bpx_code& code, const std::vector<int32_t>& syms);
// grid = 1: row blocks of A; grid = m > 1: the two-dimensional form (k*b = m^2).
int make_plan(const bpx_code& code, const int32_t* arrival, int32_t n_arrival, int32_t n_lost,
              int32_t mode, int64_t M, int64_t K, int64_t N, int32_t prec, int32_t grid,
              bpx_plan* plan, std::string* err);

}  // namespace bpx

