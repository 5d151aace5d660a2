// The extern "C" boundary of libbpx (declared in include/bpx.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "host.hpp"
#include "kernels.hpp"

namespace bpx {

namespace {
thread_local std::string g_error;
int32_t g_fused_mode = 1;  // 0 never, 1 small products, 2 whenever it fits
int32_t g_force_tile = -1;
int32_t g_group_m = 2;
int32_t g_tile_table[8 * 8 * 8 * 5];
bool g_tile_table_set = false;
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }
const char* get_error() { return g_error.c_str(); }

namespace {

bpx_status fail(bpx_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

bpx_status hip_fail(hipError_t e, const char* what) {
  return fail(BPX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

int32_t log2_bucket(int64_t x) {
  int64_t v = (x + 127) / 128;
  int32_t b = 0;
  while (v > 1 && b < 7) {
    v >>= 1;
    ++b;
  }
  return b;
}

int32_t tile_count_for(int32_t prec) {
  if (prec == BPX_PREC_BF16 || prec == BPX_PREC_BF16X3) return bf16_tile_count();
  if (prec == BPX_PREC_FP8 || prec == BPX_PREC_FP8X2) return fp8_tile_count();
  return gemm_tile_count();
}

int32_t choose_tile(int32_t prec, int64_t Mb, int64_t N, int64_t K) {
  if (g_force_tile >= 0 && g_force_tile < tile_count_for(prec)) return g_force_tile;
  if (g_tile_table_set) {
    const int32_t idx =
        ((prec * 8 + log2_bucket(Mb)) * 8 + log2_bucket(N)) * 8 + log2_bucket(K);
    const int32_t t = g_tile_table[idx];
    if (t >= 0 && t < tile_count_for(prec)) return t;
  }
  // BF16 / BF16x3 default: the flat-row 128x256 tiling (its callers fall
  // back to 64x128 where K is not a multiple of 32)
  if (prec == BPX_PREC_BF16 || prec == BPX_PREC_BF16X3) return 4;
  if (prec == BPX_PREC_FP8 || prec == BPX_PREC_FP8X2) return 1;    // wide tiling
  // FP32 default: the 256 x 256 tile with 4 x 2 waves (measured fastest on
  // 8192x8192x4096); its launcher takes the 64 x 128 tile for shapes that
  // are not multiples of 256 and for grids under one round.
  (void)Mb;
  (void)N;
  (void)K;
  return 6;
}

// Plans upload their tables lazily on the first device call; the lock makes
// that first call safe when threads share a plan (the tables are written
// once and never change afterwards).
std::mutex g_upload_mutex;

bpx_status upload(bpx_plan* plan) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_upload_mutex);
  if (plan->dev_block) {
    if (plan->dev_id != dev)
      return fail(BPX_E_INVALID, "plan tables live on another device");
    return BPX_OK;
  }
  auto bytes_of = [](size_t n, size_t sz) { return (n * sz + 255) / 256 * 256; };
  const size_t b0 = bytes_of(plan->gemm_syms.size(), 4);
  const size_t b1 = bytes_of(plan->gemm_ids.size(), 4);
  const size_t b2 = bytes_of(plan->steps.size(), sizeof(PeelStep));
  const size_t b3 = bytes_of(plan->step_subs.size(), 4);
  const size_t b4 = bytes_of(plan->fused_steps.size(), sizeof(PeelStep));
  const size_t b5 = bytes_of(plan->fused_subs.size(), 4);
  const size_t b6 = bytes_of(plan->fused_ytile.size(), 4);
  const size_t total = std::max<size_t>(b0 + b1 + b2 + b3 + b4 + b5 + b6, 256);
  std::string host(total, '\0');
  std::memcpy(&host[0], plan->gemm_syms.data(), plan->gemm_syms.size() * 4);
  std::memcpy(&host[b0], plan->gemm_ids.data(), plan->gemm_ids.size() * 4);
  std::memcpy(&host[b0 + b1], plan->steps.data(), plan->steps.size() * sizeof(PeelStep));
  std::memcpy(&host[b0 + b1 + b2], plan->step_subs.data(), plan->step_subs.size() * 4);
  std::memcpy(&host[b0 + b1 + b2 + b3], plan->fused_steps.data(),
              plan->fused_steps.size() * sizeof(PeelStep));
  std::memcpy(&host[b0 + b1 + b2 + b3 + b4], plan->fused_subs.data(),
              plan->fused_subs.size() * 4);
  std::memcpy(&host[b0 + b1 + b2 + b3 + b4 + b5], plan->fused_ytile.data(),
              plan->fused_ytile.size() * 4);
  void* d = nullptr;
  e = hipMalloc(&d, total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan tables)");
  e = hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy(plan tables)");
  }
  char* base = static_cast<char*>(d);
  plan->dev_block = d;
  plan->dev_id = dev;
  plan->d_gemm_syms = reinterpret_cast<const int32_t*>(base);
  plan->d_gemm_ids = reinterpret_cast<const int32_t*>(base + b0);
  plan->d_steps = reinterpret_cast<const PeelStep*>(base + b0 + b1);
  plan->d_step_subs = reinterpret_cast<const int32_t*>(base + b0 + b1 + b2);
  plan->d_fused_steps = reinterpret_cast<const PeelStep*>(base + b0 + b1 + b2 + b3);
  plan->d_fused_subs = reinterpret_cast<const int32_t*>(base + b0 + b1 + b2 + b3 + b4);
  plan->d_fused_ytile = reinterpret_cast<const int32_t*>(base + b0 + b1 + b2 + b3 + b4 + b5);
  return BPX_OK;
}

bpx_status check_device_call(bpx_plan* plan) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (!plan->decodable) return fail(BPX_E_UNDECODABLE, "plan is not decodable");
  if (plan->K % 4 != 0) return fail(BPX_E_INVALID, "K must be a multiple of 4");
  if (plan->prec < BPX_PREC_F32 || plan->prec > BPX_PREC_FP8X2)
    return fail(BPX_E_UNSUPPORTED, "precision not built into this library");
  return upload(plan);
}

bpx_status check_matrix(const float* ptr, int64_t ld, int64_t cols, const char* name) {
  if (!ptr) return fail(BPX_E_INVALID, std::string(name) + " is null");
  if (!aligned16(ptr)) return fail(BPX_E_INVALID, std::string(name) + " not 16-byte aligned");
  if (ld < cols || ld % 4 != 0)
    return fail(BPX_E_INVALID, std::string("leading dimension of ") + name +
                                   " must be >= its columns and a multiple of 4");
  return BPX_OK;
}

bpx_status gemm_impl(bpx_plan* plan, const float* A, int64_t lda, const float* B, int64_t ldb,
                     float* C, int64_t ldc, void* ws, size_t ws_bytes, hipStream_t stream) {
  bpx_status st;
  if ((st = check_matrix(A, lda, plan->K, "A")) != BPX_OK) return st;
  if ((st = check_matrix(B, ldb, plan->N, "B")) != BPX_OK) return st;
  if ((st = check_matrix(C, ldc, plan->N, "C")) != BPX_OK) return st;
  if (plan->ws_bytes() > 0 && (!ws || ws_bytes < plan->ws_bytes() || ((uintptr_t)ws & 255u)))
    return fail(BPX_E_INVALID, "workspace missing, not 256-byte aligned or too small");
  GemmParams p{};
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;
  p.Y = static_cast<float*>(ws);
  p.M = plan->M;
  p.K = plan->K;
  p.N = plan->N;
  p.Mb = plan->Mb;
  p.syms = plan->d_gemm_syms;
  p.ids = plan->d_gemm_ids;
  p.n_sym = (int32_t)plan->computed.size();
  p.prec = plan->prec;
  p.group_m = g_group_m;
  if (plan->part_bytes() > 0) {  // FP32 split-K partial tiles of the 256 x 256 tiling
    size_t off[7];
    plan->layout(off);
    p.part = reinterpret_cast<float*>(static_cast<char*>(ws) + off[1]);
    p.part_tiles = (int32_t)(plan->part_bytes() / (256 * 256 * sizeof(float)));
  }
  // The GEMM kernels index A rows of a block and B rows of a K-slice with
  // 32-bit offsets.
  if ((plan->Mb + 256) * lda >= ((int64_t)1 << 30) || 64 * ldb + plan->N >= ((int64_t)1 << 30))
    return fail(BPX_E_UNSUPPORTED, "block too large for 32-bit tile offsets");
  const int32_t tile = choose_tile(plan->prec, plan->Mb, plan->N, plan->K);
  hipError_t e;
  if (plan->grid > 1) {
    p.grid = plan->grid;
    p.Nb = plan->Nb;
    e = launch_coded_gemm_2d(p, tile, stream);
    if (e == hipErrorInvalidValue)
      return fail(BPX_E_UNSUPPORTED, "block too large for 32-bit buffer offsets");
  } else if (plan->is_fp8()) {
    size_t off[7];
    plan->layout(off);
    char* w = static_cast<char*>(ws);
    Fp8Params f{};
    f.A = A;
    f.lda = lda;
    f.B = B;
    f.ldb = ldb;
    f.C = C;
    f.ldc = ldc;
    f.Y = static_cast<float*>(ws);
    f.M = plan->M;
    f.K = plan->K;
    f.N = plan->N;
    f.Mb = plan->Mb;
    f.Mbp = plan->r128(plan->Mb);
    f.Kp = plan->r128(plan->K);
    f.Np = plan->r128(plan->N);
    f.syms = plan->d_gemm_syms;
    f.ids = plan->d_gemm_ids;
    f.n_sym = (int32_t)plan->computed.size();
    f.aq = reinterpret_cast<unsigned char*>(w + off[1]);
    f.aq2 = plan->prec == BPX_PREC_FP8X2 ? reinterpret_cast<unsigned char*>(w + off[2]) : nullptr;
    f.sa = reinterpret_cast<float*>(w + off[3]);
    f.bq = reinterpret_cast<unsigned char*>(w + off[4]);
    f.sb = reinterpret_cast<float*>(w + off[5]);
    if (f.Np / 128 > 65535 || f.Kp / 128 > 65535 || f.Mbp / 128 > 65535 || f.n_sym > 65535)
      return fail(BPX_E_UNSUPPORTED, "FP8 grid too large");
    e = launch_quant_b(f, stream);
    if (e == hipSuccess) e = launch_quant_a(f, stream);
    if (e == hipSuccess) e = launch_coded_gemm_fp8(f, tile, stream);
  } else if (plan->prec == BPX_PREC_BF16 || plan->prec == BPX_PREC_BF16X3) {
    char* planes = static_cast<char*>(ws) + bpx_plan::align256(plan->y_bytes());
    void* hi = planes;
    void* lo = plan->prec == BPX_PREC_BF16X3 ? planes + plan->bt_plane_bytes() : nullptr;
    p.bt_hi = static_cast<const unsigned short*>(hi);
    p.bt_lo = static_cast<const unsigned short*>(lo);
    p.kp = plan->kp();
    e = launch_split_b(B, ldb, plan->K, plan->N, plan->kp(), hi, lo, stream);
    if (e != hipSuccess) return hip_fail(e, "split-B launch");
    e = launch_coded_gemm_bf16(p, tile, stream);
  } else {
    e = launch_coded_gemm(p, tile, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "coded gemm launch");
  return BPX_OK;
}

// ------------------------------------------------------------ scratch --
// Workspace of the no-allocation entry point: one static device array per
// GPU (each device that loads the library holds its own copy until the
// process ends).  In host code `scratch` is a host-side stand-in for the
// symbol, not a device address: its device address is looked up once per
// device with hipGetSymbolAddress and only that pointer is passed on.
constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB
__device__ __attribute__((aligned(256))) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[64] = {nullptr};

// Device address of this device's scratch array (looked up on first use).
bpx_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(BPX_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr & 255u)) return fail(BPX_E_HIP, "scratch array misplaced");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BPX_OK;
}

// The fused form (one launch, peel in the GEMM epilogue): row-block plans of
// F32 / BF16 / BF16x3 whose workgroup LDS fits; in the default mode only
// products small enough that launches and latency dominate the two-launch
// path (at most 2^31 multiply-adds over the computed symbols, e.g. 512^3
// with eight symbols is 2^27).
bool fused_params(bpx_plan* plan, const float* A, int64_t lda, const float* B, int64_t ldb,
                  float* C, int64_t ldc, FusedParams* f) {
  // a forced GEMM tile shape names the two-launch form's tiling
  if (g_fused_mode == 0 || g_force_tile >= 0 || plan->grid != 1 || plan->fused_steps.empty())
    return false;
  const double macs = (double)plan->computed.size() * (double)plan->Mb * (double)plan->K *
                      (double)plan->N;
  if (g_fused_mode == 1 && macs > 2147483648.0) return false;
  *f = FusedParams{};
  f->A = A;
  f->lda = lda;
  f->B = B;
  f->ldb = ldb;
  f->C = C;
  f->ldc = ldc;
  f->M = plan->M;
  f->K = plan->K;
  f->N = plan->N;
  f->Mb = plan->Mb;
  f->syms = plan->d_gemm_syms;
  f->ids = plan->d_gemm_ids;
  f->ytile = plan->d_fused_ytile;
  f->n_sym = (int32_t)plan->computed.size();
  f->n_ytiles = plan->n_ytiles;
  f->n_ids = (int32_t)plan->gemm_ids.size();
  f->off_ids = (int32_t)(plan->d_gemm_ids - plan->d_gemm_syms);
  f->off_steps = (int32_t)(reinterpret_cast<const int32_t*>(plan->d_fused_steps) -
                           plan->d_gemm_syms);
  f->off_subs = (int32_t)(plan->d_fused_subs - plan->d_gemm_syms);
  f->off_ytile = (int32_t)(plan->d_fused_ytile - plan->d_gemm_syms);
  f->blob_words = f->off_ytile + (int32_t)plan->fused_ytile.size();
  f->steps = plan->d_fused_steps;
  f->subs = plan->d_fused_subs;
  f->nsteps = (int32_t)plan->fused_steps.size();
  f->nsubs = (int32_t)plan->fused_subs.size();
  f->nslots = plan->n_lds_slots;
  f->prec = plan->prec;
  f->kb = plan->code.kb();
  f->max_deg = 0;
  for (size_t i = 0; i < plan->computed.size(); ++i)
    f->max_deg = std::max(f->max_deg, plan->gemm_syms[4 * i + 1]);
  return fused_configure(f);
}

bpx_status peel_impl(bpx_plan* plan, const void* ws, size_t ws_bytes, float* C, int64_t ldc,
                     hipStream_t stream) {
  bpx_status st;
  if ((st = check_matrix(C, ldc, plan->N, "C")) != BPX_OK) return st;
  if (plan->y_bytes() > 0 && (!ws || ws_bytes < plan->y_bytes() || ((uintptr_t)ws & 255u)))
    return fail(BPX_E_INVALID, "workspace missing, not 256-byte aligned or too small");
  PeelParams p{};
  p.Y = static_cast<const float*>(ws);
  p.C = C;
  p.ldc = ldc;
  p.M = plan->M;
  p.N = plan->N;
  p.Mb = plan->Mb;
  p.steps = plan->d_steps;
  p.subs = plan->d_step_subs;
  p.nsteps = (int32_t)plan->steps.size();
  p.nslots = plan->n_lds_slots;
  p.nsubs = (int32_t)plan->step_subs.size();
  p.grid = plan->grid;
  p.Nb = plan->Nb;
  hipError_t e = launch_peel(p, stream);
  if (e == hipErrorInvalidConfiguration)
    return fail(BPX_E_UNSUPPORTED, "peel needs more LDS than a workgroup has");
  if (e != hipSuccess) return hip_fail(e, "peel launch");
  return BPX_OK;
}


// ------------------------------------------------------------ groups --
struct GroupLaunch {
  int32_t tile, offset, n, grid;
};

bpx_status group_build(bpx_plan* const* plans, const float* const* A, const float* const* B,
                       float* const* C, int32_t count, void* ws, size_t ws_bytes,
                       bpx_group* g);

}  // namespace
}  // namespace bpx

struct bpx_group {
  int32_t count = 0, prec = 0;
  void* dev = nullptr;
  int32_t dev_id = -1;
  const bpx::GroupDesc* d_desc = nullptr;
  const int64_t* d_bstart = nullptr;
  const int64_t* d_pstart = nullptr;
  const bpx::GroupTile* d_tiles = nullptr;
  const int32_t* d_bmap = nullptr;  // product of each split-B block
  const int32_t* d_pmap = nullptr;  // product of each peel block
  const int64_t* d_wstart = nullptr;  // first peel block of each peel workgroup
  int64_t total_b = 0, total_p = 0, peel_grid = 0;
  int32_t max_slots = 0;
  size_t max_program = 0;
  std::vector<bpx::GroupLaunch> launches;
};

namespace bpx {
namespace {

size_t group_ws_bytes(bpx_plan* const* plans, int32_t count) {
  size_t b = 0;
  for (int32_t i = 0; i < count; ++i) b += bpx_plan::align256(plans[i]->ws_bytes());
  return b;
}

bpx_status group_build(bpx_plan* const* plans, const float* const* A, const float* const* B,
                       float* const* C, int32_t count, void* ws, size_t ws_bytes,
                       bpx_group* g) {
  if (!plans || !A || !B || !C || count < 1) return fail(BPX_E_INVALID, "null argument");
  const int32_t prec = plans[0]->prec;
  if (prec != BPX_PREC_BF16 && prec != BPX_PREC_BF16X3)
    return fail(BPX_E_UNSUPPORTED, "grouped launch runs BF16 or BF16x3 plans");
  for (int32_t i = 0; i < count; ++i) {
    bpx_plan* pl = plans[i];
    if (!pl) return fail(BPX_E_INVALID, "null plan");
    if (!pl->decodable) return fail(BPX_E_UNDECODABLE, "a plan of the group is not decodable");
    if (pl->prec != prec) return fail(BPX_E_INVALID, "plans of a group must share a precision");
    if (pl->grid != 1)
      return fail(BPX_E_UNSUPPORTED, "grouped launch runs row-block (one-dimensional) plans");
    if (pl->K % 4 != 0 || pl->N % 4 != 0)
      return fail(BPX_E_INVALID, "grouped products need K and N multiples of 4");
    if (!A[i] || !B[i] || !C[i] || !aligned16(A[i]) || !aligned16(B[i]) || !aligned16(C[i]))
      return fail(BPX_E_INVALID, "operand null or not 16-byte aligned");
    if ((pl->Mb + 256) * pl->K >= ((int64_t)1 << 30))
      return fail(BPX_E_UNSUPPORTED, "block too large for 32-bit tile offsets");
    bpx_status st = upload(pl);
    if (st != BPX_OK) return st;
  }
  if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < group_ws_bytes(plans, count))
    return fail(BPX_E_INVALID, "workspace missing, not 256-byte aligned or too small");

  std::vector<GroupDesc> desc(count);
  std::vector<int64_t> bstart(count), pstart(count);
  std::vector<std::vector<GroupTile>> by_tile(bf16_tile_count());
  std::vector<std::vector<int64_t>> key(bf16_tile_count());
  char* w = static_cast<char*>(ws);
  int64_t tb = 0, tp = 0;
  int32_t max_slots = 0;
  size_t max_program = 0;
  for (int32_t i = 0; i < count; ++i) {
    bpx_plan* pl = plans[i];
    GroupDesc& d = desc[i];
    d = GroupDesc{};
    GemmParams& p = d.g;
    p.A = A[i];
    p.lda = pl->K;
    p.B = B[i];
    p.ldb = pl->N;
    p.C = C[i];
    p.ldc = pl->N;
    p.Y = reinterpret_cast<float*>(w);
    p.M = pl->M;
    p.K = pl->K;
    p.N = pl->N;
    p.Mb = pl->Mb;
    p.syms = pl->d_gemm_syms;
    p.ids = pl->d_gemm_ids;
    p.n_sym = (int32_t)pl->computed.size();
    p.prec = prec;
    char* planes = w + bpx_plan::align256(pl->y_bytes());
    p.bt_hi = reinterpret_cast<const unsigned short*>(planes);
    p.bt_lo = prec == BPX_PREC_BF16X3
                  ? reinterpret_cast<const unsigned short*>(planes + pl->bt_plane_bytes())
                  : nullptr;
    p.kp = pl->kp();
    int32_t t = choose_tile(prec, pl->Mb, pl->N, pl->K);
    if (bf16_tile_is_flat(t) && !bf16_flat_ok(p)) t = 1;
    const TileShape sh = bf16_tile_shape(t);
    int64_t nt;
    if (bf16_tile_is_flat(t)) {  // tiles over the stacked rows of all symbols
      p.tiles_m = (int32_t)(((int64_t)p.n_sym * pl->Mb + sh.bm - 1) / sh.bm);
      p.tiles_n = (int32_t)((pl->N + sh.bn - 1) / sh.bn);
      nt = (int64_t)p.tiles_m * p.tiles_n;
    } else {
      p.tiles_m = (int32_t)((pl->Mb + sh.bm - 1) / sh.bm);
      p.tiles_n = (int32_t)((pl->N + sh.bn - 1) / sh.bn);
      nt = (int64_t)p.n_sym * p.tiles_m * p.tiles_n;
    }
    d.tile = t;
    // Tiles are listed in groups of kRowGroup row panels, column panel by
    // column panel, so the run of consecutive tiles one XCD takes covers a
    // few column panels of B for several row panels and shares both in that
    // XCD's L2 (row by row, a run spans every column panel of B and uses
    // each only about twice).  Row panel rp is a stacked-row panel (flat
    // tiles) or symbol rp / tiles_m's m-tile (per-symbol tiles, which all
    // multiply the same B); either way the tile index is rp tiles_n + column.
    constexpr int64_t kRowGroup = 8;
    const int64_t panels = p.tiles_n > 0 ? nt / p.tiles_n : 0;
    for (int64_t q = 0; q < nt; ++q) {
      const int64_t per_group = kRowGroup * p.tiles_n;
      const int64_t first = q / per_group * kRowGroup;
      const int64_t rows = std::min<int64_t>(kRowGroup, panels - first);
      const int64_t r = q % per_group;
      const int64_t l = (first + r % rows) * p.tiles_n + r / rows;
      by_tile[t].push_back(GroupTile{i, (int32_t)l});
      key[t].push_back(pl->K);
    }
    PeelParams& pe = d.pe;
    pe.Y = p.Y;
    pe.C = C[i];
    pe.ldc = pl->N;
    pe.M = pl->M;
    pe.N = pl->N;
    pe.Mb = pl->Mb;
    pe.steps = pl->d_steps;
    pe.subs = pl->d_step_subs;
    pe.nsteps = (int32_t)pl->steps.size();
    pe.nslots = pl->n_lds_slots;
    pe.nsubs = (int32_t)pl->step_subs.size();
    pe.grid = 1;
    pe.Nb = pl->N;
    max_program = std::max(max_program, peel_program_bytes(pe.nsteps, pe.nsubs));
    max_slots = std::max(max_slots, pl->n_lds_slots);
    d.b_tn = (int32_t)((pl->N + 63) / 64);
    d.b_tk = (int32_t)((pl->kp() + 63) / 64);
    bstart[i] = tb;
    tb += (int64_t)d.b_tn * d.b_tk;
    pstart[i] = tp;
    if (pe.nsteps > 0) tp += (pl->Mb * (pl->N / 4) + 127) / 128;
    w += bpx_plan::align256(pl->ws_bytes());
  }
  if ((size_t)max_slots * 128 * 16 + max_program > 160 * 1024)
    return fail(BPX_E_UNSUPPORTED, "peel needs more LDS than a workgroup has");
  // tile lists: longest K first (stable), one persistent launch per shape
  std::vector<GroupTile> tiles;
  std::vector<GroupLaunch> launches;
  for (int32_t t = 0; t < (int32_t)by_tile.size(); ++t) {
    if (by_tile[t].empty()) continue;
    std::vector<size_t> idx(by_tile[t].size());
    for (size_t j = 0; j < idx.size(); ++j) idx[j] = j;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](size_t a, size_t b) { return key[t][a] > key[t][b]; });
    GroupLaunch L{t, (int32_t)tiles.size(), (int32_t)idx.size(), 0};
    for (size_t j : idx) tiles.push_back(by_tile[t][j]);
    const TileShape sh = bf16_tile_shape(t);
    const int32_t slots = 256 * ((sh.bm * sh.bn <= 128 * 128) ? 2 : 1);
    L.grid = std::min(L.n, slots);
    launches.push_back(L);
  }
  // block -> product maps of the split-B and peel grids
  std::vector<int32_t> bmap(tb), pmap(tp);
  for (int32_t i = 0; i < count; ++i) {
    const int64_t bend = i + 1 < count ? bstart[i + 1] : tb;
    const int64_t pend = i + 1 < count ? pstart[i + 1] : tp;
    for (int64_t b = bstart[i]; b < bend; ++b) bmap[b] = i;
    for (int64_t b = pstart[i]; b < pend; ++b) pmap[b] = i;
  }
  // Peel workgroup ranges: a block of product i costs its program's steps
  // plus one (the per-block work); workgroup w of G starts at the first
  // block whose cumulative cost reaches w T / G (T the total), so that every
  // workgroup gets about the same number of steps.
  const int64_t pgrid = tp > 0 ? peel_grouped_grid(tp, max_slots, max_program) : 0;
  std::vector<int64_t> wstart(pgrid + 1, tp);
  if (pgrid > 0) {
    int64_t T = 0;
    for (int32_t i = 0; i < count; ++i) {
      const int64_t pend = i + 1 < count ? pstart[i + 1] : tp;
      T += (pend - pstart[i]) * ((int64_t)plans[i]->steps.size() + 1);
    }
    int64_t w = 0, cum = 0;
    for (int32_t i = 0; i < count && w <= pgrid; ++i) {
      const int64_t n = (i + 1 < count ? pstart[i + 1] : tp) - pstart[i];
      const int64_t c = (int64_t)plans[i]->steps.size() + 1;
      while (w <= pgrid) {
        const int64_t t = w * T / pgrid;
        if (t >= cum + n * c) break;
        wstart[w] = pstart[i] + (t - cum + c - 1) / c;
        ++w;
      }
      cum += n * c;
    }
  }
  // one device block: descriptors | bstart | pstart | tiles | bmap | pmap | wstart
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t s0 = al(desc.size() * sizeof(GroupDesc));
  const size_t s1 = al(bstart.size() * 8);
  const size_t s2 = al(pstart.size() * 8);
  const size_t s3 = al(std::max<size_t>(tiles.size(), 1) * sizeof(GroupTile));
  const size_t s4 = al(std::max<size_t>(bmap.size(), 1) * 4);
  const size_t s5 = al(std::max<size_t>(pmap.size(), 1) * 4);
  const size_t s6 = al(wstart.size() * 8);
  std::string host(s0 + s1 + s2 + s3 + s4 + s5 + s6, '\0');
  std::memcpy(&host[0], desc.data(), desc.size() * sizeof(GroupDesc));
  std::memcpy(&host[s0], bstart.data(), bstart.size() * 8);
  std::memcpy(&host[s0 + s1], pstart.data(), pstart.size() * 8);
  std::memcpy(&host[s0 + s1 + s2], tiles.data(), tiles.size() * sizeof(GroupTile));
  std::memcpy(&host[s0 + s1 + s2 + s3], bmap.data(), bmap.size() * 4);
  std::memcpy(&host[s0 + s1 + s2 + s3 + s4], pmap.data(), pmap.size() * 4);
  std::memcpy(&host[s0 + s1 + s2 + s3 + s4 + s5], wstart.data(), wstart.size() * 8);
  void* dptr = nullptr;
  hipError_t e = hipMalloc(&dptr, host.size());
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(group descriptors)");
  e = hipMemcpy(dptr, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dptr);
    return hip_fail(e, "hipMemcpy(group descriptors)");
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  char* base = static_cast<char*>(dptr);
  g->count = count;
  g->prec = prec;
  g->dev = dptr;
  g->dev_id = dev;
  g->d_desc = reinterpret_cast<const GroupDesc*>(base);
  g->d_bstart = reinterpret_cast<const int64_t*>(base + s0);
  g->d_pstart = reinterpret_cast<const int64_t*>(base + s0 + s1);
  g->d_tiles = reinterpret_cast<const GroupTile*>(base + s0 + s1 + s2);
  g->d_bmap = reinterpret_cast<const int32_t*>(base + s0 + s1 + s2 + s3);
  g->d_pmap = reinterpret_cast<const int32_t*>(base + s0 + s1 + s2 + s3 + s4);
  g->d_wstart = reinterpret_cast<const int64_t*>(base + s0 + s1 + s2 + s3 + s4 + s5);
  g->peel_grid = pgrid;
  g->total_b = tb;
  g->total_p = tp;
  g->max_slots = max_slots;
  g->max_program = max_program;
  g->launches = launches;
  return BPX_OK;
}

bpx_status group_launch(bpx_group* g, int32_t phase, hipStream_t stream) {
  hipError_t e;
  if (phase < 0 || phase == 0) {
    e = launch_split_b_grouped(g->d_desc, g->d_bstart, g->d_bmap, g->total_b, stream);
    if (e != hipSuccess) return hip_fail(e, "grouped split-B launch");
  }
  if (phase < 0 || phase == 1) {
    const int32_t split = g->prec == BPX_PREC_BF16X3 ? 3 : 1;
    for (const GroupLaunch& L : g->launches) {
      e = launch_gemm_bf16_grouped(g->d_desc, g->d_tiles + L.offset, L.n, L.tile, split, L.grid,
                                   stream);
      if (e != hipSuccess) return hip_fail(e, "grouped GEMM launch");
    }
  }
  if (phase < 0 || phase == 2) {
    e = launch_peel_grouped(g->d_desc, g->d_pstart, g->d_pmap, g->d_wstart, g->peel_grid,
                            g->max_slots, g->max_program, stream);
    if (e != hipSuccess) return hip_fail(e, "grouped peel launch");
  }
  return BPX_OK;
}

}  // namespace
}  // namespace bpx

using namespace bpx;

extern "C" {

const char* bpx_last_error(void) { return get_error(); }

bpx_status bpx_code_build(const bpx_code_params* params, bpx_code** out) {
  if (!params || !out) return fail(BPX_E_INVALID, "null argument");
  *out = nullptr;
  bpx_code* c = new (std::nothrow) bpx_code();
  if (!c) return fail(BPX_E_NOMEM, "out of host memory");
  std::string err;
  int st = build_code(*params, c, &err);
  if (st != BPX_OK) {
    delete c;
    return fail((bpx_status)st, err);
  }
  *out = c;
  return BPX_OK;
}

bpx_status bpx_code_from_csr(int32_t n, int32_t k, int32_t b, const int32_t* col_ptr,
                             const int32_t* sym_ptr, const uint16_t* sym_data, bpx_code** out) {
  if (!out || !col_ptr || !sym_ptr) return fail(BPX_E_INVALID, "null argument");
  *out = nullptr;
  if (n < 1 || k < 1 || b < 1 || (int64_t)k * b > 65535)
    return fail(BPX_E_INVALID, "need n, k, b >= 1 and k*b <= 65535");
  if (col_ptr[0] != 0) return fail(BPX_E_INVALID, "col_ptr[0] must be 0");
  for (int32_t j = 0; j < n; ++j)
    if (col_ptr[j + 1] < col_ptr[j]) return fail(BPX_E_INVALID, "col_ptr not ascending");
  const int32_t ns = col_ptr[n];
  if (sym_ptr[0] != 0) return fail(BPX_E_INVALID, "sym_ptr[0] must be 0");
  if (ns > 0 && sym_ptr[ns] > 0 && !sym_data) return fail(BPX_E_INVALID, "null sym_data");
  for (int32_t g = 0; g < ns; ++g) {
    if (sym_ptr[g + 1] < sym_ptr[g]) return fail(BPX_E_INVALID, "sym_ptr not ascending");
    for (int32_t e = sym_ptr[g]; e < sym_ptr[g + 1]; ++e) {
      if (sym_data[e] >= k * b) return fail(BPX_E_INVALID, "data id out of range");
      if (e > sym_ptr[g] && sym_data[e] <= sym_data[e - 1])
        return fail(BPX_E_INVALID, "ids of a symbol must be strictly ascending");
    }
  }
  bpx_code* c = new (std::nothrow) bpx_code();
  if (!c) return fail(BPX_E_NOMEM, "out of host memory");
  c->kind = -1;
  c->n = n;
  c->k = k;
  c->b = b;
  c->col_ptr.assign(col_ptr, col_ptr + n + 1);
  c->sym_ptr.assign(sym_ptr, sym_ptr + ns + 1);
  c->sym_data.assign(sym_data, sym_data + sym_ptr[ns]);
  *out = c;
  return BPX_OK;
}

bpx_status bpx_code_info(const bpx_code* code, int32_t* n, int32_t* k, int32_t* b,
                         int32_t* n_sym, int32_t* nnz, int32_t* max_degree) {
  if (!code) return fail(BPX_E_INVALID, "null code");
  if (n) *n = code->n;
  if (k) *k = code->k;
  if (b) *b = code->b;
  if (n_sym) *n_sym = code->n_sym();
  if (nnz) *nnz = (int32_t)code->sym_data.size();
  if (max_degree) *max_degree = code->max_degree();
  return BPX_OK;
}

bpx_status bpx_code_csr(const bpx_code* code, const int32_t** col_ptr, const int32_t** sym_ptr,
                        const uint16_t** sym_data) {
  if (!code) return fail(BPX_E_INVALID, "null code");
  if (col_ptr) *col_ptr = code->col_ptr.data();
  if (sym_ptr) *sym_ptr = code->sym_ptr.data();
  if (sym_data) *sym_data = code->sym_data.data();
  return BPX_OK;
}

void bpx_code_free(bpx_code* code) { delete code; }

bpx_status bpx_plan_create(const bpx_code* code, const int32_t* arrival, int32_t n_arrival,
                           int32_t n_lost, int32_t mode, int64_t M, int64_t K, int64_t N,
                           int32_t prec, bpx_plan** out) {
  if (!code || !out) return fail(BPX_E_INVALID, "null argument");
  *out = nullptr;
  bpx_plan* p = new (std::nothrow) bpx_plan();
  if (!p) return fail(BPX_E_NOMEM, "out of host memory");
  std::string err;
  int st = make_plan(*code, arrival, n_arrival, n_lost, mode, M, K, N, prec, 1, p, &err);
  if (st == BPX_E_INVALID) {
    delete p;
    return fail(BPX_E_INVALID, err);
  }
  *out = p;
  if (st == BPX_E_UNDECODABLE) return fail(BPX_E_UNDECODABLE, "available columns do not peel");
  return BPX_OK;
}

bpx_status bpx_plan_create2d(const bpx_code* code, const int32_t* arrival, int32_t n_arrival,
                             int32_t n_lost, int32_t mode, int64_t M, int64_t K, int64_t N,
                             int32_t prec, bpx_plan** out) {
  if (!code || !out) return fail(BPX_E_INVALID, "null argument");
  *out = nullptr;
  const int32_t kb = code->kb();
  int32_t m = 1;
  while ((int64_t)(m + 1) * (m + 1) <= kb) ++m;
  if ((int64_t)m * m != kb || m < 2)
    return fail(BPX_E_INVALID, "the two-dimensional form needs k*b a square of at least 4");
  if (prec != BPX_PREC_F32) return fail(BPX_E_UNSUPPORTED, "the two-dimensional form runs FP32");
  if (K % 4 != 0 || N % m != 0 || (N / m) % 4 != 0)
    return fail(BPX_E_UNSUPPORTED, "the two-dimensional form needs K % 4 == 0 and N / grid a "
                                   "multiple of 4");
  bpx_plan* p = new (std::nothrow) bpx_plan();
  if (!p) return fail(BPX_E_NOMEM, "out of host memory");
  std::string err;
  int st = make_plan(*code, arrival, n_arrival, n_lost, mode, M, K, N, prec, m, p, &err);
  if (st == BPX_E_INVALID) {
    delete p;
    return fail(BPX_E_INVALID, err);
  }
  *out = p;
  if (st == BPX_E_UNDECODABLE) return fail(BPX_E_UNDECODABLE, "available columns do not peel");
  return BPX_OK;
}

bpx_status bpx_plan_grid(const bpx_plan* plan, int32_t* grid, int64_t* Nb) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (grid) *grid = plan->grid;
  if (Nb) *Nb = plan->Nb;
  return BPX_OK;
}

bpx_status bpx_plan_info(const bpx_plan* plan, int32_t* decodable, int32_t* prefix_m,
                         int32_t* n_computed, int32_t* depth_max, int32_t* n_unrecovered,
                         int64_t* Mb) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (decodable) *decodable = plan->decodable ? 1 : 0;
  if (prefix_m) *prefix_m = plan->prefix_m;
  if (n_computed) *n_computed = (int32_t)plan->computed.size();
  if (depth_max) *depth_max = plan->depth_max;
  if (n_unrecovered) *n_unrecovered = (int32_t)plan->unrecovered.size();
  if (Mb) *Mb = plan->Mb;
  return BPX_OK;
}

bpx_status bpx_plan_schedule(const bpx_plan* plan, const int32_t** computed, const int32_t** dest,
                             const int32_t** releaser, const int32_t** depth,
                             const int32_t** sub_ptr, const uint16_t** sub_data,
                             const int32_t** unrecovered) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (computed) *computed = plan->computed.data();
  if (dest) *dest = plan->dest.data();
  if (releaser) *releaser = plan->releaser.data();
  if (depth) *depth = plan->depth.data();
  if (sub_ptr) *sub_ptr = plan->sub_ptr.data();
  if (sub_data) *sub_data = plan->sub_data.data();
  if (unrecovered) *unrecovered = plan->unrecovered.data();
  return BPX_OK;
}

bpx_status bpx_plan_peel_program(const bpx_plan* plan, const int32_t** steps, int32_t* n_steps,
                                 int32_t* step_words, const int32_t** subs, int32_t* n_subs,
                                 int32_t* n_slots) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  static_assert(sizeof(PeelStep) == 9 * sizeof(int32_t), "peel step record");
  if (steps) *steps = reinterpret_cast<const int32_t*>(plan->steps.data());
  if (n_steps) *n_steps = (int32_t)plan->steps.size();
  if (step_words) *step_words = (int32_t)(sizeof(PeelStep) / sizeof(int32_t));
  if (subs) *subs = plan->step_subs.data();
  if (n_subs) *n_subs = (int32_t)plan->step_subs.size();
  if (n_slots) *n_slots = plan->n_lds_slots;
  return BPX_OK;
}

bpx_status bpx_plan_workspace_bytes(const bpx_plan* plan, size_t* ws_bytes,
                                    size_t* encode_bytes) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (ws_bytes) *ws_bytes = plan->ws_bytes();
  if (encode_bytes)
    *encode_bytes = plan->computed.size() * (size_t)plan->Mb * (size_t)plan->K * sizeof(float);
  return BPX_OK;
}

bpx_status bpx_plan_workspace_layout(const bpx_plan* plan, size_t* offsets, int32_t n) {
  if (!plan || !offsets || n < 1) return fail(BPX_E_INVALID, "null argument");
  size_t off[7];
  plan->layout(off);
  for (int32_t i = 0; i < n && i < 7; ++i) offsets[i] = off[i];
  return BPX_OK;
}

bpx_status bpx_plan_upload(bpx_plan* plan) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  return upload(plan);
}

void bpx_plan_free(bpx_plan* plan) {
  if (!plan) return;
  if (plan->dev_block) (void)hipFree(plan->dev_block);
  delete plan;
}

bpx_status bpx_encode(bpx_plan* plan, const float* A, int64_t lda, float* coded_out,
                      bpx_stream stream) {
  bpx_status st = check_device_call(plan);
  if (st != BPX_OK) return st;
  if ((st = check_matrix(A, lda, plan->K, "A")) != BPX_OK) return st;
  if (plan->grid > 1)
    return fail(BPX_E_UNSUPPORTED, "stand-alone encode is for row-block plans");
  if (!coded_out || !aligned16(coded_out))
    return fail(BPX_E_INVALID, "coded_out null or misaligned");
  EncodeParams p{};
  p.A = A;
  p.lda = lda;
  p.out = coded_out;
  p.M = plan->M;
  p.K = plan->K;
  p.Mb = plan->Mb;
  p.syms = plan->d_gemm_syms;
  p.ids = plan->d_gemm_ids;
  p.n_sym = (int32_t)plan->computed.size();
  hipError_t e = launch_encode(p, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "encode launch");
  return BPX_OK;
}

bpx_status bpx_coded_gemm(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                          int64_t ldb, float* C, int64_t ldc, void* ws, size_t ws_bytes,
                          bpx_stream stream) {
  bpx_status st = check_device_call(plan);
  if (st != BPX_OK) return st;
  return gemm_impl(plan, A, lda, B, ldb, C, ldc, ws, ws_bytes,
                   reinterpret_cast<hipStream_t>(stream));
}

bpx_status bpx_peel_decode(bpx_plan* plan, const void* ws, size_t ws_bytes, float* C,
                           int64_t ldc, bpx_stream stream) {
  bpx_status st = check_device_call(plan);
  if (st != BPX_OK) return st;
  return peel_impl(plan, ws, ws_bytes, C, ldc, reinterpret_cast<hipStream_t>(stream));
}

bpx_status bpx_coded_matmul(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                            int64_t ldb, float* C, int64_t ldc, void* ws, size_t ws_bytes,
                            bpx_stream stream) {
  bpx_status st = check_device_call(plan);
  if (st != BPX_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FusedParams f;
  if (fused_params(plan, A, lda, B, ldb, C, ldc, &f)) {
    // same argument contract as the two-launch form (the caller cannot
    // tell which form runs), though the fused launch leaves ws untouched
    if ((st = check_matrix(A, lda, plan->K, "A")) != BPX_OK) return st;
    if ((st = check_matrix(B, ldb, plan->N, "B")) != BPX_OK) return st;
    if ((st = check_matrix(C, ldc, plan->N, "C")) != BPX_OK) return st;
    if (plan->ws_bytes() > 0 && (!ws || ws_bytes < plan->ws_bytes() || ((uintptr_t)ws & 255u)))
      return fail(BPX_E_INVALID, "workspace missing, not 256-byte aligned or too small");
    const hipError_t e = launch_fused(f, s);
    if (e != hipSuccess) return hip_fail(e, "fused coded product launch");
    return BPX_OK;
  }
  st = gemm_impl(plan, A, lda, B, ldb, C, ldc, ws, ws_bytes, s);
  if (st != BPX_OK) return st;
  return peel_impl(plan, ws, ws_bytes, C, ldc, s);
}

bpx_status bpx_coded_matmul_noalloc(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                                    int64_t ldb, float* C, int64_t ldc, bpx_stream stream) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (!plan->decodable) return fail(BPX_E_UNDECODABLE, "plan is not decodable");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  // the plan's tables must already be on this device: uploading allocates
  if (!plan->dev_block || plan->dev_id != dev)
    return fail(BPX_E_INVALID, "plan tables not uploaded to this device (call bpx_plan_upload)");
  if (plan->K % 4 != 0) return fail(BPX_E_INVALID, "K must be a multiple of 4");
  const size_t need = plan->ws_bytes();
  if (need > kScratchBytes)
    return fail(BPX_E_UNSUPPORTED, "plan needs " + std::to_string(need) +
                                       " bytes of workspace; the scratch array holds " +
                                       std::to_string(kScratchBytes));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bpx_status st;
  FusedParams f;
  if (fused_params(plan, A, lda, B, ldb, C, ldc, &f)) {  // needs no workspace
    if ((st = check_matrix(A, lda, plan->K, "A")) != BPX_OK) return st;
    if ((st = check_matrix(B, ldb, plan->N, "B")) != BPX_OK) return st;
    if ((st = check_matrix(C, ldc, plan->N, "C")) != BPX_OK) return st;
    const hipError_t e = launch_fused(f, s);
    if (e != hipSuccess) return hip_fail(e, "fused coded product launch");
    return BPX_OK;
  }
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != BPX_OK) return st;
  st = gemm_impl(plan, A, lda, B, ldb, C, ldc, ws, kScratchBytes, s);
  if (st != BPX_OK) return st;
  return peel_impl(plan, ws, kScratchBytes, C, ldc, s);
}

bpx_status bpx_group_workspace_bytes(bpx_plan* const* plans, int32_t count, size_t* bytes) {
  if (!plans || !bytes || count < 1) return fail(BPX_E_INVALID, "null argument");
  for (int32_t i = 0; i < count; ++i)
    if (!plans[i]) return fail(BPX_E_INVALID, "null plan");
  *bytes = group_ws_bytes(plans, count);
  return BPX_OK;
}

bpx_status bpx_group_create(bpx_plan* const* plans, const float* const* A, const float* const* B,
                            float* const* C, int32_t count, void* ws, size_t ws_bytes,
                            bpx_group** out) {
  if (!out) return fail(BPX_E_INVALID, "null argument");
  *out = nullptr;
  bpx_group* g = new (std::nothrow) bpx_group();
  if (!g) return fail(BPX_E_NOMEM, "out of host memory");
  bpx_status st = group_build(plans, A, B, C, count, ws, ws_bytes, g);
  if (st != BPX_OK) {
    delete g;
    return st;
  }
  *out = g;
  return BPX_OK;
}

bpx_status bpx_group_launch_phase(bpx_group* group, int32_t phase, bpx_stream stream) {
  if (!group || phase < -1 || phase > 2) return fail(BPX_E_INVALID, "null group or bad phase");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != group->dev_id) return fail(BPX_E_INVALID, "group lives on another device");
  return group_launch(group, phase, reinterpret_cast<hipStream_t>(stream));
}

bpx_status bpx_group_launch(bpx_group* group, bpx_stream stream) {
  return bpx_group_launch_phase(group, -1, stream);
}

void bpx_group_free(bpx_group* group) {
  if (!group) return;
  if (group->dev) (void)hipFree(group->dev);
  delete group;
}

bpx_status bpx_coded_matmul_grouped(bpx_plan* const* plans, const float* const* A,
                                    const float* const* B, float* const* C, int32_t count,
                                    void* ws, size_t ws_bytes, bpx_stream stream) {
  bpx_group* g = nullptr;
  bpx_status st = bpx_group_create(plans, A, B, C, count, ws, ws_bytes, &g);
  if (st != BPX_OK) return st;
  st = bpx_group_launch(g, stream);
  const hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  bpx_group_free(g);
  if (st != BPX_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return BPX_OK;
}

int32_t bpx_tile_count(int32_t prec) { return tile_count_for(prec); }

bpx_status bpx_set_tile_table(const int32_t* table, int32_t n_entries) {
  const int32_t need = (int32_t)(sizeof(g_tile_table) / sizeof(g_tile_table[0]));
  if (!table) {
    g_tile_table_set = false;
    return BPX_OK;
  }
  if (n_entries != need) return fail(BPX_E_INVALID, "tile table has the wrong size");
  std::memcpy(g_tile_table, table, sizeof(g_tile_table));
  g_tile_table_set = true;
  return BPX_OK;
}

bpx_status bpx_set_tile_order(int32_t group_m) {
  if (group_m < 1 || group_m > 64) return fail(BPX_E_INVALID, "group_m must be in [1, 64]");
  g_group_m = group_m;
  return BPX_OK;
}

bpx_status bpx_set_fused_peel(int32_t mode) {
  if (mode < 0 || mode > 2) return fail(BPX_E_INVALID, "fused-peel mode must be 0, 1 or 2");
  g_fused_mode = mode;
  return BPX_OK;
}

bpx_status bpx_plan_fused(bpx_plan* plan, int32_t* fused) {
  if (!plan || !fused) return fail(BPX_E_INVALID, "null argument");
  FusedParams f;
  *fused = plan->decodable &&
                   fused_params(plan, nullptr, plan->K, nullptr, plan->N, nullptr, plan->N, &f)
               ? 1
               : 0;
  return BPX_OK;
}

bpx_status bpx_plan_fused_program(const bpx_plan* plan, const int32_t** steps, int32_t* n_steps,
                                  const int32_t** subs, int32_t* n_subs, const int32_t** ytile,
                                  int32_t* n_ytiles) {
  if (!plan) return fail(BPX_E_INVALID, "null plan");
  if (steps) *steps = reinterpret_cast<const int32_t*>(plan->fused_steps.data());
  if (n_steps) *n_steps = (int32_t)plan->fused_steps.size();
  if (subs) *subs = plan->fused_subs.data();
  if (n_subs) *n_subs = (int32_t)plan->fused_subs.size();
  if (ytile) *ytile = plan->fused_ytile.data();
  if (n_ytiles) *n_ytiles = plan->n_ytiles;
  return BPX_OK;
}

bpx_status bpx_force_tile(int32_t tile) {
  if (tile >= std::max(gemm_tile_count(), bf16_tile_count()))
    return fail(BPX_E_INVALID, "no such tile shape");
  g_force_tile = tile < 0 ? -1 : tile;
  return BPX_OK;
}

}  // extern "C"
