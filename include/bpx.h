/*
 * bpx.h - C ABI of the array BP-XOR coded matrix multiplication library
 * (libbpx.so, HIP for gfx950).
 *
 * Method: Arslan, "Array BP-XOR Codes for Hierarchically Distributed Matrix
 * Multiplication" (arXiv 1904.11563).  The paper computes A^T B over n compute
 * nodes (Sec. II); a node (column of the code) holds b coded symbols, each the
 * XOR of a subset of the k*b information symbols (Sec. III-A, definition of
 * the [n,k,t,b] array BP-XOR code), and the sink recovers the product with the
 * belief-propagation (peeling) decoder of Sec. I-A from the columns that
 * arrive first.
 *
 * This library computes C = A.B with A (M x K) and B (K x N), all FP32
 * row-major.  The k*b information symbols are the k*b row-blocks of A
 * (block s = rows [s*Mb, (s+1)*Mb), Mb = ceil(M/(k*b)), rows past M are zero);
 * a coded symbol g is the real sum C_g = sum_{s in N(g)} A_s (XOR read as a
 * real sum, as Table I writes it); each virtual worker multiplies its coded
 * blocks by B; the peel recovers every A_s.B.
 *
 * Conventions for every function:
 *  - Return value is a bpx_status; on failure bpx_last_error() returns a
 *    message (thread-local, valid until the next call on the same thread).
 *  - Handles (bpx_code, bpx_plan) are created and freed by the library and
 *    their contents (code, schedule) do not change after creation; distinct
 *    handles may be used from distinct threads, and one plan may be shared
 *    by threads (its device tables are uploaded once, under a lock, by the
 *    first device call).  Arrays returned through "borrowed" pointers live
 *    as long as the handle.
 *  - The tuning setters (bpx_set_tile_table, bpx_force_tile,
 *    bpx_set_tile_order) change process-wide state read by every later
 *    device call; call them before device calls start, not concurrently
 *    with them.
 *  - Host functions (code and plan construction, queries) never touch the GPU.
 *  - Device functions take caller-owned device pointers, enqueue on the given
 *    HIP stream and return without synchronising.  They allocate nothing
 *    except the plan's small device tables, which are uploaded on the first
 *    device call with that plan (or by bpx_plan_upload); call
 *    bpx_plan_upload before capturing a device call in a HIP graph.
 *  - Matrices are row-major with leading dimensions in elements.  A, B, C,
 *    workspaces must be 16-byte aligned and lda, ldb, ldc multiples of 4.
 *    K must be a multiple of 4.  M, N are arbitrary (>= 1).
 */
#ifndef BPX_H
#define BPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BPX_OK = 0,
  BPX_E_INVALID = -1,      /* bad argument                                   */
  BPX_E_UNDECODABLE = -2,  /* the available columns do not peel               */
  BPX_E_NOMEM = -3,        /* host or device allocation failed                */
  BPX_E_HIP = -4,          /* a HIP runtime call failed                       */
  BPX_E_UNSUPPORTED = -5   /* valid request outside what this library handles */
} bpx_status;

typedef enum {
  BPX_CODE_ARRAY_SEARCH = 0, /* deterministic search for an [n,k,.,b] code    */
  BPX_CODE_TABLE1 = 1,       /* Table I, the [5,2,.,2] code, sigma = 2         */
  BPX_CODE_TABLE3 = 2,       /* Table III, the [5,3,2,3] code, sigma = 2       */
  BPX_CODE_MOJETTE = 3,      /* Mojette code, Construction A or B (Sec. III-C) */
  BPX_CODE_IDENTITY = 4      /* uncoded layout: n = k columns of b data blocks */
} bpx_code_kind;

typedef enum {
  BPX_PREC_F32 = 0,    /* FP32 operands, FP32 MFMA                            */
  BPX_PREC_BF16 = 1,   /* operands rounded to BF16 (RNE), one MFMA pass       */
  BPX_PREC_BF16X3 = 2, /* split BF16: hi.hi + hi.lo + lo.hi, FP32 accumulate  */
  BPX_PREC_FP8 = 3,    /* e4m3, one power-of-two scale per 128x128 block      */
  BPX_PREC_FP8X2 = 4   /* coded operand split into two e4m3 terms, B one term */
} bpx_prec;

typedef enum {
  BPX_MODE_ERASURE = 0,   /* first n - n_lost arrival columns exist; shortest
                             peelable prefix of them is computed             */
  BPX_MODE_STRAGGLER = 1, /* all columns arrive; shortest peelable prefix    */
  BPX_MODE_FULL = 2,      /* every column computed, schedule from all        */
  BPX_MODE_MIN = 3        /* as STRAGGLER but only the releasers computed    */
} bpx_mode;

typedef struct {
  int32_t kind;        /* bpx_code_kind                                       */
  int32_t n, k, b;     /* columns, data columns, symbols per data column      */
  int32_t sigma_max;   /* ARRAY_SEARCH: maximum symbol degree (1..k*b)        */
  int32_t restarts;    /* ARRAY_SEARCH: restarts of the hill-climb            */
  int32_t iters;       /* ARRAY_SEARCH: iterations per restart                */
  int32_t mojette_qe;  /* MOJETTE: 0 = Construction A (q = 1),
                          >= 1 = Construction B (q = 2^qe, odd p)            */
  uint64_t seed;       /* ARRAY_SEARCH: SplitMix64 seed                       */
  int32_t walk;        /* ARRAY_SEARCH: 0 = hill-climb (keep a change when the
                          whole objective does not get worse), 1 = plateau
                          walk (keep it when (failing subsets, all-columns
                          flag) does not get worse; return the best code seen) */
  int32_t reserved;    /* must be 0                                           */
} bpx_code_params;

typedef struct bpx_code bpx_code;
typedef struct bpx_plan bpx_plan;
typedef struct ihipStream_t* bpx_stream; /* a hipStream_t; NULL = null stream */

/* ---------------------------------------------------------------- codes -- */

/* Build a code (host, integer only).  Symbols are numbered column by column
 * (g = symbols in earlier columns + row); data ids of a symbol are sorted.
 * ARRAY_SEARCH: a local search over random codes driven by one
 *   SplitMix64(seed) stream, minimising (failing k-column subsets,
 *   all-columns-fail flag, unrecovered ids summed over failing subsets,
 *   peeling rounds summed over peelable subsets, total degree), as a
 *   hill-climb or a plateau walk (walk); the paper gives no general
 *   construction for array BP-XOR codes (Sec. III-A/B) so the code is
 *   searched.  Needs k*b <= 64.  Cost grows with restarts * iters * C(n, k).
 * TABLE1 / TABLE3: the worked codes of Table I / Table III; v_i -> id i-1.
 * MOJETTE: n projections over the k x b grid, ascending p; bin of cell
 *   (z, l) given by Eq. (moj1); data id of (z, l) is l*b + z; empty bins keep
 *   their index.  Construction A: p = -floor((n-1)/2)..ceil((n-1)/2), q = 1.
 *   Construction B: odd p = ceil_odd(1-n)..ceil_odd(n-1), q = 2^qe.
 * IDENTITY: n = k; symbol (j, i) = block j*b + i.
 * *out receives a new handle (free with bpx_code_free).
 * Errors: BPX_E_INVALID for out-of-range parameters. */
bpx_status bpx_code_build(const bpx_code_params* params, bpx_code** out);

/* Build a code from explicit CSR arrays (copied).  col_ptr has n+1 entries
 * (symbol ranges per column), sym_ptr n_sym+1 entries (id ranges per
 * symbol), sym_data the ids (each < k*b, strictly ascending per symbol).
 * Errors: BPX_E_INVALID on malformed arrays. */
bpx_status bpx_code_from_csr(int32_t n, int32_t k, int32_t b, const int32_t* col_ptr,
                             const int32_t* sym_ptr, const uint16_t* sym_data,
                             bpx_code** out);

/* Sizes of a code: columns, k, b, total symbols (empty bins included), total
 * degree (sum of |N(g)|), maximum degree.  Any pointer may be NULL. */
bpx_status bpx_code_info(const bpx_code* code, int32_t* n, int32_t* k, int32_t* b,
                         int32_t* n_sym, int32_t* nnz, int32_t* max_degree);

/* Borrowed views of the code's CSR arrays (see bpx_code_from_csr). */
bpx_status bpx_code_csr(const bpx_code* code, const int32_t** col_ptr,
                        const int32_t** sym_ptr, const uint16_t** sym_data);

void bpx_code_free(bpx_code* code);

/* ---------------------------------------------------------------- plans -- */

/* Plan one coded product (host, integer only; no GPU call).
 * arrival: permutation of the n column ids, earliest first.
 * n_lost: ERASURE mode only, the number of trailing arrival columns that
 *   never arrive.
 * Prefix: the smallest m such that the non-empty symbols of the first m
 *   arrival columns peel (peeling success only grows with m, so the scan is
 *   exact); the time-to-decode of Eq. (1) for this arrival order.
 * Schedule: round-based peeling (Sec. I-A).  In round r every symbol with
 *   exactly one unknown id is a candidate; each id released in round r takes
 *   the candidate with the smallest (degree, g) as releaser g_s, gets depth
 *   r, and sub_s = N(g_s) \ {s}; all ids of a round become known together.
 * Computed symbols: every non-empty symbol of the first m columns (FULL: of
 *   all columns; MIN: only the releasers), ascending g.
 * M, K, N: the product's shape; prec: bpx_prec of the device path.
 * Returns BPX_OK, or BPX_E_UNDECODABLE when the available columns do not
 * peel; in that case *out is still a valid, queryable plan (its schedule
 * covers what was recovered) and every device call with it returns
 * BPX_E_UNDECODABLE without writing anything. */
bpx_status bpx_plan_create(const bpx_code* code, const int32_t* arrival, int32_t n_arrival,
                           int32_t n_lost, int32_t mode, int64_t M, int64_t K, int64_t N,
                           int32_t prec, bpx_plan** out);

/* The same plan for the paper's two-dimensional form (Sec. III-A, Examples
 * 1 and 2): with k*b = grid^2, A is split into grid row blocks (Mb =
 * ceil(M/grid) rows) and B into grid column blocks (Nb = N/grid columns), and
 * data id s = r*grid + c is the block product A_r B_c, whose result fills C
 * rows r*Mb .., columns c*Nb ...  A coded symbol whose members share a B
 * block is computed as (sum of A blocks) . B_c, one whose members share an A
 * block as A_r . (sum of B blocks), and any other (the paper's gray cells)
 * as the sum of its members' block products (a K-concatenated product).
 * FP32 only; needs K % 4 == 0 and N a multiple of 4*grid
 * (BPX_E_UNSUPPORTED otherwise), k*b a perfect square >= 4 (BPX_E_INVALID).
 * Prefix, schedule and error behaviour as bpx_plan_create; Y slots are
 * Mb x Nb.  Full blocks (Mb and Nb multiples of 256, M = grid*Mb, N =
 * grid*Nb, K a multiple of 32) run on 256x256 tiles when the FP32 tile
 * shape is one of the 256x256 ones (the default), other shapes and calls on
 * 64x128 tiles; both sum every product in the same order (identical
 * results).  bpx_encode and grouped launches do not take such plans. */
bpx_status bpx_plan_create2d(const bpx_code* code, const int32_t* arrival, int32_t n_arrival,
                             int32_t n_lost, int32_t mode, int64_t M, int64_t K, int64_t N,
                             int32_t prec, bpx_plan** out);

/* Block grid of a plan: grid = 1 and Nb = N for row-block plans. */
bpx_status bpx_plan_grid(const bpx_plan* plan, int32_t* grid, int64_t* Nb);

/* Scalar facts of a plan; any pointer may be NULL.  Mb = ceil(M/(k*b))
 * (two-dimensional plans: ceil(M/grid)).  depth_max = the largest release
 * round. */
bpx_status bpx_plan_info(const bpx_plan* plan, int32_t* decodable, int32_t* prefix_m,
                         int32_t* n_computed, int32_t* depth_max, int32_t* n_unrecovered,
                         int64_t* Mb);

/* Borrowed views of the schedule.
 * computed[n_computed]: computed symbol ids, ascending.
 * dest[n_computed]: where the coded product of computed[i] is written by
 *   bpx_coded_gemm: dest >= 0 is a slot of the Y workspace (slot d occupies
 *   floats [d*Mb*N, (d+1)*Mb*N), row-major Mb x N); dest < 0 means the
 *   product is written straight into C rows of data block (-1 - dest)
 *   (a degree-1 releaser).
 * releaser[kb], depth[kb]: g_s and the release round of each data id (-1 and
 *   0 if not recovered).
 * sub_ptr[kb+1], sub_data: sub_s = N(g_s) \ {s}, ascending.
 * unrecovered[n_unrecovered]: ids not recovered.  Any pointer may be NULL. */
bpx_status bpx_plan_schedule(const bpx_plan* plan, const int32_t** computed,
                             const int32_t** dest, const int32_t** releaser,
                             const int32_t** depth, const int32_t** sub_ptr,
                             const uint16_t** sub_data, const int32_t** unrecovered);

/* The peel program the decode runs (read-only, owned by the plan; for
 * inspection and host-side checks).  steps: n_steps records of step_words
 * int32, in execution order: {s, src, nsub, sub_off, f64, slot, write, brow,
 * bcol}: data block s is Y[src] (src >= 0, a workspace Y slot) or the block
 * already in C (src = -1) minus the values held in the nsub slots
 * subs[sub_off ..], accumulated in FP64 (f64 = 1) or FP32 with
 * compensation; the result is kept in slot `slot` (>= 0) for later steps
 * and written to C (write = 1); brow, bcol locate s in the block grid.
 * Slots are per-thread storage (registers for a single product whose
 * program needs at most 12, else LDS), reused once their block's last
 * subtraction has run; n_slots is the number in use at most.  Sec. I-A's peeling, in the order of the
 * release rounds.  Any pointer may be NULL. */
bpx_status bpx_plan_peel_program(const bpx_plan* plan, const int32_t** steps, int32_t* n_steps,
                                 int32_t* step_words, const int32_t** subs, int32_t* n_subs,
                                 int32_t* n_slots);

/* Device workspace the plan needs for bpx_coded_gemm / bpx_coded_matmul
 * (Y slots and, for FP8, quantised operands and scales), and the size of the
 * buffer bpx_encode writes (n_computed coded blocks of Mb x K floats). */
bpx_status bpx_plan_workspace_bytes(const bpx_plan* plan, size_t* ws_bytes,
                                    size_t* encode_bytes);

/* Byte offsets of the parts of the plan's workspace (n entries written,
 * at most 7), every part 256-byte aligned; a part the precision does not
 * use has size 0 (its offset equals the next one); entry 6 is the total.
 *   F32:     [0] Y slots, [1] split-K partial tiles: when Mb and N are
 *            multiples of 256, K of 32 and M of Mb, room for min(256, 4 T)
 *            FP32 tiles of 256 x 256 (T = computed symbols x Mb/256 x N/256),
 *            used by the last round of the 256 x 256 tiling
 *   BF16*:   [0] Y, [1] Bt_hi, [2] Bt_lo: B rounded to bf16 (RNE) and the
 *            bf16 residual, transposed (N x Kp, k contiguous, Kp = K rounded
 *            up to 32, zero past K)
 *   FP8*:    [0] Y, [1] Aq, [2] Aq2, [3] sA, [4] Bq, [5] sB: e4m3 codes of
 *            the coded blocks ([n_computed][Mbp][Kp] bytes), of the FP8x2
 *            residual term, their scales as FP32 values ([n_computed][Mbp/128]
 *            [Kp/128]), the codes of B transposed ([Np][Kp]) and its scales
 *            ([Kp/128][Np/128]); Mbp, Kp, Np = Mb, K, N rounded up to 128.
 * Per 128 x 128 block: s = the smallest power of two with amax <= 448 s (1 if
 * amax = 0, at least 2^-122), code = e4m3(clamp(x / s, +-448)) with round to
 * nearest even; the FP8x2 residual code is e4m3(clamp((x / s - code) * 16,
 * +-448)).  The GEMM applies s through the MFMA's E8M0 scale operands. */
bpx_status bpx_plan_workspace_layout(const bpx_plan* plan, size_t* offsets, int32_t n);

/* Upload the plan's device tables now (hipMalloc + synchronous copy on the
 * current device).  Device calls do this on first use otherwise. */
bpx_status bpx_plan_upload(bpx_plan* plan);

void bpx_plan_free(bpx_plan* plan);

/* --------------------------------------------------------------- device -- */

/* Encode only: write C_g = sum_{s in N(g)} A_s (FP32, ascending s) for every
 * computed symbol, block i of coded_out (ld = K) holding computed[i].  The
 * master-side encode of Sec. II; exists for tests and encode bandwidth.
 * coded_out must hold encode_bytes (bpx_plan_workspace_bytes). */
bpx_status bpx_encode(bpx_plan* plan, const float* A, int64_t lda, float* coded_out,
                      bpx_stream stream);

/* Coded products: Y_g = C_g . B for every computed symbol.  F32 and BF16*:
 * the encode is fused into the A-operand load (the coded block is never
 * stored).  FP8*: a streaming encode+quantise pass writes the e4m3 codes of
 * every 128 x 128 coded tile (its scale needs the tile's amax), B is
 * quantised once per call, then the block-scaled FP8 product runs.  Products go to
 * the Y slots of ws or, for degree-1 releasers, straight into C (see dest in
 * bpx_plan_schedule).  Precision is the plan's.  ws must hold ws_bytes. */
bpx_status bpx_coded_gemm(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                          int64_t ldb, float* C, int64_t ldc, void* ws, size_t ws_bytes,
                          bpx_stream stream);

/* Peel: in (depth, s) order, X_s = Y_{g_s} - sum_{u in sub_s} X_u, written to
 * C rows of block s (rows past M are not written).  Accumulation is FP32
 * compensated (Kahan) where depth_s <= 4 and FP64 where depth_s > 4.
 * Reads the Y slots of ws and the C blocks of degree-1 releasers. */
bpx_status bpx_peel_decode(bpx_plan* plan, const void* ws, size_t ws_bytes, float* C,
                           int64_t ldc, bpx_stream stream);

/* The whole coded product: bpx_coded_gemm followed by bpx_peel_decode on the
 * same stream, or, for small products, one launch with the peel fused into
 * the GEMM epilogue (the BP decoder of Sec. I-A applies the same release
 * program to every element, so a workgroup that owns one 16-row tile of
 * every data block computes that tile of every computed coded product,
 * keeps the releasers' tiles in LDS and peels them there; the coded
 * products never reach memory and ws is not used).  The fused form runs
 * row-block F32 / BF16 / BF16x3 plans whose workgroup fits in LDS (the
 * whole K extent of a 16..64-column strip of B is staged on chip), by
 * default when the computed symbols hold at most 2^31 multiply-adds
 * (bpx_set_fused_peel).  Both forms compute the same values in the same
 * order of operations within each product: results match the two-launch
 * path. */
bpx_status bpx_coded_matmul(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                            int64_t ldb, float* C, int64_t ldc, void* ws, size_t ws_bytes,
                            bpx_stream stream);

/* When bpx_coded_matmul (and bpx_coded_matmul_noalloc) take the fused form:
 * 0 never, 1 for small products (the default), 2 whenever it fits.
 * Process-wide, like the tile settings. */
bpx_status bpx_set_fused_peel(int32_t mode);

/* *fused = 1 if bpx_coded_matmul takes the fused form for this plan with
 * dense operands (lda = K, ldb = ldc = N) under the current mode on the
 * current device, else 0. */
bpx_status bpx_plan_fused(bpx_plan* plan, int32_t* fused);

/* The fused form's peel program (read-only, owned by the plan): steps in
 * the bpx_plan_peel_program record format, but with src = the LDS Y tile
 * that holds the releaser's product and write = 1 for every recovered
 * block; ytile[i] is the Y tile of the i-th computed symbol (ascending g),
 * -1 if it releases nothing.  Slots as in bpx_plan_peel_program. */
bpx_status bpx_plan_fused_program(const bpx_plan* plan, const int32_t** steps, int32_t* n_steps,
                                  const int32_t** subs, int32_t* n_subs, const int32_t** ytile,
                                  int32_t* n_ytiles);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as bpx_coded_matmul, same kernels and results, with the workspace
 * taken from a static device array of the library (32 MiB per GPU, held by
 * every device that uses it until the process ends) instead of a caller
 * buffer.  Allocates nothing: the plan's tables must already be on the
 * current device (bpx_plan_upload), else BPX_E_INVALID; a plan whose
 * workspace (bpx_plan_workspace_bytes) exceeds 32 MiB gets
 * BPX_E_UNSUPPORTED.  Every call on one GPU shares that GPU's array, and
 * nothing in it needs to start at zero (each call writes every byte it
 * reads first): calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. */
bpx_status bpx_coded_matmul_noalloc(bpx_plan* plan, const float* A, int64_t lda, const float* B,
                                    int64_t ldb, float* C, int64_t ldc, bpx_stream stream);

/* ------------------------------------------------------------- groups -- */

/* Many independent coded products, each with its own code, arrival pattern
 * and shape, in one launch sequence that allocates nothing, so that it can
 * be captured once in a HIP graph and replayed.  Operands of product i are
 * dense row-major: A[i] (M x K, lda = K), B[i] (K x N, ldb = N), C[i]
 * (M x N, ldc = N), K and N multiples of 4, 16-byte aligned.  All plans must
 * share one precision, BF16 or BF16x3.
 *
 * bpx_group_workspace_bytes: device workspace for the plans (each plan's
 *   bpx_plan_workspace_bytes rounded up to 256, back to back).
 * bpx_group_create: host setup, done once: uploads the plans' tables and one
 *   block of per-product descriptors and a tile list (hipMalloc + one
 *   synchronous copy).  ws (256-byte aligned) and every operand pointer are
 *   baked into the descriptors and must stay valid while the group lives.
 *   Each product gets the GEMM tile shape bpx_set_tile_table selects for
 *   its (Mb, N, K); tiles of one shape form one persistent launch whose
 *   workgroups stride over the tile list, longest K first.
 *   Returns BPX_E_UNDECODABLE if any plan is undecodable (nothing created).
 * bpx_group_launch: enqueue, on stream: one grouped B-split launch, one
 *   persistent grouped GEMM launch per tile shape present, one grouped peel
 *   launch.  No allocation, copy or synchronisation: graph-capturable.
 *   Calls on one group must not overlap (they share the workspace).
 * bpx_coded_matmul_grouped: create, launch, synchronise the stream, free. */
typedef struct bpx_group bpx_group;
bpx_status bpx_group_workspace_bytes(bpx_plan* const* plans, int32_t count, size_t* bytes);
bpx_status bpx_group_create(bpx_plan* const* plans, const float* const* A, const float* const* B,
                            float* const* C, int32_t count, void* ws, size_t ws_bytes,
                            bpx_group** out);
bpx_status bpx_group_launch(bpx_group* group, bpx_stream stream);
/* One phase of bpx_group_launch (0: B split, 1: GEMMs, 2: peel; -1: all),
 * for timing the phases separately; the phases must run in order. */
bpx_status bpx_group_launch_phase(bpx_group* group, int32_t phase, bpx_stream stream);
void bpx_group_free(bpx_group* group);
bpx_status bpx_coded_matmul_grouped(bpx_plan* const* plans, const float* const* A,
                                    const float* const* B, float* const* C, int32_t count,
                                    void* ws, size_t ws_bytes, bpx_stream stream);

/* Tile-shape selection.  bpx_tile_count(prec) returns the number of compiled
 * GEMM tile shapes for a precision; bpx_set_tile_table installs an autotuned
 * table mapping shape buckets (log2 of ceil(x/128), clamped to [0, 7], for
 * x = Mb, N, K) and the precision to a tile-shape index, indexed
 * ((prec*8 + bMb)*8 + bN)*8 + bK (8*8*8*5 entries; NULL clears it; entries
 * < 0 fall back to the default shape).  bpx_force_tile forces one shape for
 * every call (for the autotuner and tests), which also keeps every call on
 * the two-launch form; -1 returns to the table.
 * BF16 / BF16x3 shapes 0-3 are 128x128, 64x128, 128x256 and 64x256 tiles of
 * one symbol; 4 (the default) is 128x256 tiles over the stacked rows of all
 * computed symbols, used when K is a multiple of 32 (otherwise shape 1).
 * FP32 shapes 0-3 are 128x128, 64x128, 128x256 and 256x128; 4-6 are 256x256
 * with 2x2, 2x4 and 4x2 waves (the default), used when Mb and N are
 * multiples of 256, K of 32 and every data block is full, otherwise the call
 * takes shape 1; a last round of 256x256 tiles under 90% of the CUs runs as
 * 2 to 4 pieces of each tile's K range (summed in piece order by a second
 * kernel; run in chunks that fit the workspace's partial tiles) when that
 * takes at most 0.8 of a round and the workspace holds partial tiles, else
 * as 64x128 sub-tiles.
 * Results are deterministic; shapes and the split change only the FP32
 * summation order.  FP8 / FP8x2: shape 0 is one 128x128 tile grid per
 * symbol, shape 1 (the default) one grid of 128x256 tiles over all symbols'
 * codes, used when N rounded up to 128 is a multiple of 256, otherwise
 * shape 0. */
int32_t bpx_tile_count(int32_t prec);
/* Order in which the FP32 GEMM walks its output tiles: row panels (symbol x
 * m-tile) in groups of group_m, each group finished column panel by column
 * panel (1 = plain row-major order).  Affects speed and L2 reuse only.  The
 * BF16 / BF16x3 kernels (and the grouped launch's tile lists) walk fixed
 * groups of 8 row panels, the FP8 kernel groups of 4. */
bpx_status bpx_set_tile_order(int32_t group_m);
bpx_status bpx_set_tile_table(const int32_t* table, int32_t n_entries);
bpx_status bpx_force_tile(int32_t tile);

const char* bpx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BPX_H */
