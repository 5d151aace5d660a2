// Peeling decode on the device: one HBM-streaming pass.
//
// The BP decoder of Sec. I-A, run on real numbers: in (depth, s) order every
// recovered block is X_s = Y_{g_s} - sum over u in N(g_s)\{s} of X_u.  The
// schedule is identical for every element of the Mb x N block, so each
// thread runs the whole program for its own element (row r, column c of
// every block) with no barriers between release rounds.  Values that later
// steps subtract are kept in this thread's LDS column, or, for a single
// product in the vector form whose program needs at most kRegSlots of
// them, in registers.
//
// Accumulation: FP32 with Kahan compensation for depth <= 4; FP64 for
// deeper releases; subtrahends in ascending id order.  Rows past M (padding
// of the last block) are exactly zero and are neither read nor written.
//
// Two forms: a vector form (N and ldc multiples of 4) where a thread owns
// four adjacent columns and moves 16 bytes per load and store, and a scalar
// form for ragged N.  Loads of kBatch steps are issued before their
// arithmetic so that many requests are in flight per thread.  The program
// (steps and subtrahend slot lists) is the same for every thread, so each
// workgroup copies it to LDS once, behind its slots; the step loop then
// reads descriptors from LDS instead of chasing them through global memory.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace bpx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBatch = 16;  // steps whose loads are issued together (all of a 16-step program)

__device__ __forceinline__ int64_t valid_rows(const PeelParams& p, int64_t base) {
  return p.M - base < p.Mb ? p.M - base : p.Mb;
}

// Copies the step program to LDS (prog = steps, then subs); returns after a
// barrier, so every thread of the workgroup sees it.
__device__ __forceinline__ void stage_program(const PeelParams& p, int32_t* prog, int nthreads) {
  const int n_step_words = p.nsteps * (int)(sizeof(PeelStep) / 4);
  const int32_t* steps = reinterpret_cast<const int32_t*>(p.steps);
  for (int i = threadIdx.x; i < n_step_words; i += nthreads) prog[i] = steps[i];
  for (int i = threadIdx.x; i < p.nsubs; i += nthreads) prog[n_step_words + i] = p.subs[i];
  __syncthreads();
}

// ------------------------------------------------------------- scalar form --
template <int THREADS>
__device__ __forceinline__ void peel_block(const PeelParams& p, int64_t block, float* xs,
                                           const PeelStep* steps, const int32_t* subs) {
  const int tid = threadIdx.x;
  const int64_t total = p.Mb * p.Nb;
  const int64_t e = block * THREADS + tid;
  const bool active = e < total;
  const int64_t r = active ? e / p.Nb : 0;
  const int64_t c = active ? e - r * p.Nb : 0;
  // data block s sits at C rows brow * Mb + r, column bcol * Nb + c
  auto c_index = [&](const PeelStep& S) __attribute__((always_inline)) -> int64_t {
    return ((int64_t)S.brow * p.Mb + r) * p.ldc + (int64_t)S.bcol * p.Nb + c;
  };
  auto valid = [&](const PeelStep& S) __attribute__((always_inline)) -> bool {
    return (int64_t)S.brow * p.Mb + r < p.M && (int64_t)S.bcol * p.Nb + c < p.N;
  };

  for (int st0 = 0; st0 < p.nsteps; st0 += kBatch) {
    float y[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      y[i] = 0.f;
      const int st = st0 + i;
      if (st < p.nsteps && active) {
        const PeelStep S = steps[st];
        if (valid(S)) {
          if (S.src >= 0)
            y[i] = p.Y[(int64_t)S.src * total + e];
          else
            y[i] = p.C[c_index(S)];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int st = st0 + i;
      if (st >= p.nsteps) break;
      const PeelStep S = steps[st];
      const bool ok = active && valid(S);
      float x = 0.f;
      if (ok) {
        const int32_t* sub = subs + S.sub_off;
        if (S.f64) {
          double acc = (double)y[i];
          for (int u = 0; u < S.nsub; ++u) acc -= (double)xs[sub[u] * THREADS + tid];
          x = (float)acc;
        } else {
          float sum = y[i], comp = 0.f;
          for (int u = 0; u < S.nsub; ++u) {
            const float v = -xs[sub[u] * THREADS + tid] - comp;
            const float t = sum + v;
            comp = (t - sum) - v;
            sum = t;
          }
          x = sum;
        }
      }
      if (S.slot >= 0) xs[S.slot * THREADS + tid] = x;
      if (S.write && ok) p.C[c_index(S)] = x;
    }
  }
}

// ------------------------------------------------------------- vector form --
// Y and C are reached through pointers read from memory (the grouped form's
// descriptors), which the compiler would access with flat instructions;
// those count on the LDS counter as well, so every wait for an LDS read of
// the program or a slot would also wait for the HBM loads in flight.  The
// product buffers are device memory: accessed as global.
typedef __attribute__((address_space(1))) v4f gv4f;
__device__ __forceinline__ v4f gload4(const float* ptr) {
  return *(const gv4f*)ptr;
}
__device__ __forceinline__ void gstore4(float* ptr, v4f v) { *(gv4f*)ptr = v; }

// Where a thread keeps the values later steps subtract (slot s of this
// thread's four columns): in LDS, one column of slots per thread ...
template <int THREADS>
struct LdsSlots {
  v4f* xs;
  __device__ __forceinline__ v4f get(int s) const { return xs[s * THREADS + threadIdx.x]; }
  __device__ __forceinline__ void put(int s, v4f x) { xs[s * THREADS + threadIdx.x] = x; }
};
// ... or in registers, for programs with at most kRegSlots live slots:
// slots 0-7 in a 32-float vector, 8-11 in a 16-float vector, reached
// through the GPR index mode by the slot number, which every lane shares
// (so the workgroup's LDS holds only the program, and the chip holds every
// row of a large block at once instead of in LDS-limited rounds).
typedef float v32f __attribute__((ext_vector_type(32)));
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr int kRegSlots = 12;
struct RegSlots {
  v32f a = {};
  v16f b = {};
  __device__ __forceinline__ v4f get(int s) const {
    s = __builtin_amdgcn_readfirstlane(s);
    if (s < 8) {
      const int i = 4 * s;
      return v4f{a[i], a[i + 1], a[i + 2], a[i + 3]};
    }
    const int i = 4 * (s - 8);
    return v4f{b[i], b[i + 1], b[i + 2], b[i + 3]};
  }
  __device__ __forceinline__ void put(int s, v4f x) {
    s = __builtin_amdgcn_readfirstlane(s);
    if (s < 8) {
      const int i = 4 * s;
      a[i] = x[0];
      a[i + 1] = x[1];
      a[i + 2] = x[2];
      a[i + 3] = x[3];
    } else {
      const int i = 4 * (s - 8);
      b[i] = x[0];
      b[i + 1] = x[1];
      b[i + 2] = x[2];
      b[i + 3] = x[3];
    }
  }
};

template <int THREADS, int KB, typename Slots>
__device__ __forceinline__ void peel_block4(const PeelParams& p, int64_t block, Slots& xs,
                                            const PeelStep* steps, const int32_t* subs) {
  const int tid = threadIdx.x;
  const int64_t n4 = p.N / 4;
  const int64_t total4 = p.Mb * n4;
  const int64_t e = block * THREADS + tid;
  const bool active = e < total4;
  const int64_t r = active ? e / n4 : 0;
  const int64_t c = active ? (e - r * n4) * 4 : 0;
  const int64_t slot_elems = p.Mb * p.N;

  for (int st0 = 0; st0 < p.nsteps; st0 += KB) {
    v4f y[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      y[i] = v4f{0.f, 0.f, 0.f, 0.f};
      const int st = st0 + i;
      if (st < p.nsteps && active) {
        const PeelStep S = steps[st];
        const int64_t base = (int64_t)S.s * p.Mb;
        if (r < valid_rows(p, base)) {
          if (S.src >= 0)
            y[i] = gload4(p.Y + (int64_t)S.src * slot_elems + r * p.N + c);
          else
            y[i] = gload4(p.C + (base + r) * p.ldc + c);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const int st = st0 + i;
      if (st >= p.nsteps) break;
      const PeelStep S = steps[st];
      const int64_t base = (int64_t)S.s * p.Mb;
      const int64_t valid = valid_rows(p, base);
      v4f x = {0.f, 0.f, 0.f, 0.f};
      if (r < valid) {
        const int32_t* sub = subs + S.sub_off;
        if (S.f64) {
          v4d acc = {(double)y[i][0], (double)y[i][1], (double)y[i][2], (double)y[i][3]};
          for (int u = 0; u < S.nsub; ++u) {
            const v4f v = xs.get(sub[u]);
            acc -= v4d{(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
          }
          x = v4f{(float)acc[0], (float)acc[1], (float)acc[2], (float)acc[3]};
        } else {
          v4f sum = y[i], comp = {0.f, 0.f, 0.f, 0.f};
          for (int u = 0; u < S.nsub; ++u) {
            const v4f v = -xs.get(sub[u]) - comp;
            const v4f t = sum + v;
            comp = (t - sum) - v;
            sum = t;
          }
          x = sum;
        }
      }
      if (S.slot >= 0) xs.put(S.slot, x);
      if (S.write && active && r < valid) gstore4(p.C + (base + r) * p.ldc + c, x);
    }
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void peel_kernel(PeelParams p) {
  extern __shared__ float xs[];  // [nslots][THREADS], then the program
  int32_t* prog = reinterpret_cast<int32_t*>(xs + (size_t)p.nslots * THREADS);
  stage_program(p, prog, THREADS);
  peel_block<THREADS>(p, blockIdx.x, xs, reinterpret_cast<const PeelStep*>(prog),
                      prog + p.nsteps * (int)(sizeof(PeelStep) / 4));
}

// Grouped peel: block b runs product pmap[b]'s program (vector form:
// grouped products have N a multiple of 4).
// Persistent over the 128-column-group items of all products (item b of
// product i is b - pstart[i], pmap[b] = i): workgroup w takes the
// contiguous range wstart[w] .. wstart[w + 1] - 1, split on the host so that
// every range holds about the same number of steps (products' programs
// differ in length), so consecutive items mostly belong to one product and
// its step program is staged once, not per item.  An item then costs one round
// of loads (its y values) instead of four dependent ones (item -> product ->
// descriptor -> program -> y).  The LDS slots are per thread and rewritten
// by each item before they are read, so items need no barrier between them;
// a new program is staged behind a barrier.
__global__ __launch_bounds__(128) void peel_grouped_kernel(const GroupDesc* __restrict__ d,
                                                           const int64_t* __restrict__ pstart,
                                                           const int32_t* __restrict__ pmap,
                                                           const int64_t* __restrict__ wstart,
                                                           int32_t max_slots) {
  extern __shared__ v4f xs4[];  // [max_slots][128], then the current product's program
  int32_t* prog = reinterpret_cast<int32_t*>(xs4 + (size_t)max_slots * 128);
  const int64_t b0 = wstart[blockIdx.x];
  const int64_t b1 = wstart[blockIdx.x + 1];
  int cur = -1;
  for (int64_t b = b0; b < b1; ++b) {
    // uniform by construction; readfirstlane lets the compiler keep the
    // descriptor in scalar registers, copied once per item (a reference
    // would be reloaded after every store to C, which might alias it)
    const int prod = __builtin_amdgcn_readfirstlane(pmap[b]);
    const PeelParams p = d[prod].pe;
    if (prod != cur) {
      if (cur >= 0) __syncthreads();  // every thread is done with the old program
      stage_program(p, prog, 128);
      cur = prod;
    }
    LdsSlots<128> slots{xs4};
    peel_block4<128, kBatch>(p, b - pstart[prod], slots, reinterpret_cast<const PeelStep*>(prog),
                             prog + p.nsteps * (int)(sizeof(PeelStep) / 4));
  }
}

}  // namespace

// As many workgroups as the CUs hold at once (LDS- or wave-limited), at
// most one per item.
int64_t peel_grouped_grid(int64_t total_blocks, int32_t max_slots, size_t max_program) {
  const size_t lds = (size_t)max_slots * 128 * 16 + max_program;
  const int64_t per_cu = std::min<int64_t>(16, (int64_t)(160 * 1024) / (int64_t)(lds ? lds : 1));
  return std::min<int64_t>(total_blocks, (int64_t)device_cu_count() * std::max<int64_t>(per_cu, 1));
}

hipError_t launch_peel_grouped(const GroupDesc* d, const int64_t* pstart, const int32_t* pmap,
                               const int64_t* wstart, int64_t grid, int32_t max_slots,
                               size_t max_program, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  const size_t lds = (size_t)max_slots * 128 * 16 + max_program;
  if (lds > 160 * 1024 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(peel_grouped_kernel, dim3((unsigned)grid), dim3(128), lds, stream, d, pstart,
                     pmap, wstart, max_slots);
  return hipGetLastError();
}

// Single products take the vector form (128 threads: 74 us on the
// 8192 x 4096 FP32 workload, against 87 us for the scalar form with 256
// threads) when N and ldc are multiples of 4 and the blocks are row blocks;
// otherwise the scalar form, which also handles the block grid of the
// two-dimensional form.
// Single product, row blocks, N and ldc multiples of 4: the vector form.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void peel4s_kernel(PeelParams p) {
  extern __shared__ v4f xs4s[];
  int32_t* prog = reinterpret_cast<int32_t*>(xs4s + (size_t)p.nslots * THREADS);
  stage_program(p, prog, THREADS);
  LdsSlots<THREADS> slots{xs4s};
  peel_block4<THREADS, kBatch>(p, blockIdx.x, slots, reinterpret_cast<const PeelStep*>(prog),
                               prog + p.nsteps * (int)(sizeof(PeelStep) / 4));
}
// The same with the slots in registers: 8 loads in flight per thread
// instead of 16 and at most 128 registers per lane, so that four waves per
// SIMD fit and a CU holds 8 workgroups (the 8192 x 4096 workload's 2048
// workgroups in one round, where LDS slots allowed 6 per CU: peel 61 -> 50
// us; 12 loads in flight gave 51 us).  The grouped peel keeps its LDS slots:
// its persistent workgroups are not limited by how many a CU holds (the
// batch's peel took the same 0.58 ms with register slots).
constexpr int kBatchReg = 8;
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(4))) void peel4r_kernel(
    PeelParams p) {
  extern __shared__ int32_t prog_r[];
  stage_program(p, prog_r, 128);
  RegSlots slots;
  peel_block4<128, kBatchReg>(p, blockIdx.x, slots, reinterpret_cast<const PeelStep*>(prog_r),
                              prog_r + p.nsteps * (int)(sizeof(PeelStep) / 4));
}
hipError_t launch_peel(const PeelParams& p, hipStream_t stream) {
  if (p.nsteps == 0) return hipSuccess;
  if (p.grid == 1 && (p.N & 3) == 0 && (p.ldc & 3) == 0) {
    const int64_t blocks = (p.Mb * (p.N / 4) + 127) / 128;
    const size_t prog = peel_program_bytes(p.nsteps, p.nsubs);
    if (p.nslots <= kRegSlots && prog <= 64 * 1024 && blocks <= 0x7fffffff) {
      hipLaunchKernelGGL(peel4r_kernel, dim3((unsigned)blocks), dim3(128), prog, stream, p);
      return hipGetLastError();
    }
    const size_t lds = (size_t)p.nslots * 128 * 16 + prog;
    if (lds <= 160 * 1024 && blocks <= 0x7fffffff) {
      hipLaunchKernelGGL(peel4s_kernel<128>, dim3((unsigned)blocks), dim3(128), lds, stream, p);
      return hipGetLastError();
    }
  }
  const int64_t total = p.Mb * p.Nb;
  int threads = 256;
  if ((int64_t)p.nslots * 256 * 4 > 64 * 1024) threads = 64;
  const size_t lds =
      (size_t)p.nslots * threads * sizeof(float) + peel_program_bytes(p.nsteps, p.nsubs);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const int64_t blocks = (total + threads - 1) / threads;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (threads == 256)
    hipLaunchKernelGGL(peel_kernel<256>, dim3((unsigned)blocks), dim3(256), lds, stream, p);
  else
    hipLaunchKernelGGL(peel_kernel<64>, dim3((unsigned)blocks), dim3(64), lds, stream, p);
  return hipGetLastError();
}

}  // namespace bpx
