// Persistent batch kernel: one launch (two for two-pass sizes) runs a list of
// limb tasks of mixed ring degree (2^10 .. 2^17), moduli and operation.
//
// RNS polynomials of different sizes and limb counts (Section 5) decompose
// into independent limb tasks.  The host groups the tasks into blocks of one
// class (operation, N, wide-range flag), longest units first and by (N, q)
// within a class; each workgroup of the persistent grid claims the next unit
// from a device-side counter and runs the units of that block until a claim
// lands in the next block:
//   * N <= 2^14: whole limbs held on chip (ntt_onchip.h) with the single-pass
//     kernel's own shape (16 or 32 coefficients per thread), 512 / (N / 2^logr)
//     limbs side by side per workgroup;
//   * N >= 2^15 transforms: 4096-coefficient tiles of the two-pass schedule
//     (ntt_tile.h), two per workgroup; the first pass runs in phase 0, the
//     last pass in a second launch (phase 1), whose boundary orders the two;
//   * products out = a * b (forward(a), forward(b) fused with the multiply,
//     inverse: the product listing of Section 4): on chip for N <= 2^14, else
//     one workgroup runs all three two-pass transforms.
// Forward outputs are lazy [0, 4q) or canonical, inverse outputs lazy [0, 2q)
// or canonical.  The blocks, the descriptors and their counts live in device
// memory, so a captured graph of [descriptor copy, phase 0, phase 1] can be
// replayed for any batch; each phase's claim counter is cleared by the
// workgroup that makes the phase's last claim.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"
#include "ntt_onchip.h"
#include "ntt_tile.h"

// Two staging sets are used in turn, so the host can prepare the next batch
// while the previous one still runs.
struct ntt_batch_stage {
  unsigned char* host;             // pinned staging: the head (blocks and counts), then the tasks
  unsigned char* dev;              // device: claim counters (own line), then the staging's copy
  hipEvent_t done;                 // completion of the last run from this set
  hipEvent_t copied;               // plain runs: the descriptor copy on the context's copy stream
  bool pending;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;       // [phase 0, phase 1]; the descriptor copy runs before each replay
};
struct ntt_batch {
  int device;
  size_t capacity;                 // tasks
  int grid;                        // persistent workgroups (0: automatic)
  int shape;                       // unit shapes: 0 the per-call kernels', 1 twice the threads per limb and tile, 2 per tile only
  int cur;                         // staging set of the next run
  hipStream_t copy_stream;         // runs copy their descriptors here, overlapping the previous run
  bool use_copy_stream;            // off: copies go on the launch stream (callers that own several streams)
  ntt_batch_stage stage[2];
};

namespace nttamd {

// Block classes: BatchBlock::cls = kind | logN << 3 | op << 8 | wide << 11 | shape << 12.
enum : uint32_t { kClassOnchip = 0, kClassProduct = 1, kClassTile0 = 2, kClassTile1 = 3 };
// A run of units of one class within a phase.
struct BatchBlock {
  uint32_t unit0, units;    // claim indices [unit0, unit0 + units) of the phase
  uint32_t desc0, subs;     // first descriptor; sub-tasks (limbs, or tiles: N / 4096 per descriptor)
  uint32_t cls;
  uint32_t last;            // set on the device: the phase's last claim value (its workgroup clears the counter)
  uint32_t pad[2];
};
// Every class present in a batch has one block per phase it runs in: at most
// 40 single-pass transform classes, 13 product classes and 12 two-pass
// transform classes in phase 0, and those 12 again in phase 1.
constexpr int kMaxBlocks = 80;
struct BatchHead {
  uint32_t units[2];        // per phase
  uint32_t blocks[2];       // per phase; phase 1's blocks follow phase 0's
  uint32_t pad[4];
  BatchBlock block[kMaxBlocks];
};

// Staging layout: the head, then one descriptor per task from kStageHead on.
// The device copy keeps the two claim counters in their own line in front
// (counters at 0, staging mirrored from kDevHead).
constexpr size_t kStageHead = (sizeof(BatchHead) + 127) & ~(size_t)127;
constexpr size_t kDevHead = 128;
static ntt_batch_stage& cur_stage(ntt_batch* b) { return b->stage[b->cur]; }
static BatchTask* staged_tasks(ntt_batch* b) { return reinterpret_cast<BatchTask*>(cur_stage(b).host + kStageHead); }
static BatchHead* staged_head(ntt_batch* b) { return reinterpret_cast<BatchHead*>(cur_stage(b).host); }
static size_t stage_bytes(size_t count) { return kStageHead + count * sizeof(BatchTask); }
static size_t dev_bytes(const ntt_batch* b) { return kDevHead + stage_bytes(b->capacity); }

constexpr int kBatchThreads = 512;
// LDS of one workgroup: two sub-groups' 4096-coefficient tiles, or the exchange
// buffers of the limbs it holds (68 KiB; two workgroups share a CU).
constexpr int kBatchLdsWords32 = 17408;

// ---- block classes --------------------------------------------------------------
//
// The host orders the tasks into blocks of one class each (kind, logN, op,
// wide-range flag).  A claimed unit of a block is G sub-tasks run side by side
// by G sub-groups of 512 / G threads: whole limbs (N <= 2^14) with the
// single-pass kernel's own shape, 2^onchip_logr(logN) coefficients per thread;
// or two 4096-coefficient tiles of one pass of a split two-pass transform.

// Shape 1 gives a limb (or tile) twice the threads of shape 0, with half the coefficients each.
__host__ __device__ constexpr int batch_logr(int logN, int shape) { return onchip_logr(logN) - shape; }
__host__ __device__ constexpr int onchip_groups(int logN, int shape = 0) {
  return kBatchThreads / ((1 << logN) >> batch_logr(logN, shape));
}

// Every sub-group is a whole number of waves, so the sub-task index, the
// descriptor and its plan are wave-uniform: taken through readfirstlane they
// live in scalar registers, as a kernel's arguments would.
// (The builtin returns a signed int: widened directly, a low word with bit 31
// set would sign-extend over the high word.)
__device__ __forceinline__ u32 rfl(u32 v) { return (u32)__builtin_amdgcn_readfirstlane((int)v); }
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = rfl((u32)v), hi = rfl((u32)(v >> 32));
  return reinterpret_cast<T*>(lo | hi << 32);
}
// Address-space views for a device function (the compiler infers them only
// for pointers that come from a kernel's arguments): descriptors and plan
// headers are read-only during a launch and read through the constant space
// (scalar loads), coefficients and tables through the global space.
#define NTTAMD_CONST __attribute__((address_space(4)))
#define NTTAMD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)(NTTAMD_GLOBAL T*)p;
}
__device__ __forceinline__ BatchTask load_task(const BatchTask* tasks, u32 i) {
  const NTTAMD_CONST BatchTask* c = (const NTTAMD_CONST BatchTask*)uniform_ptr(tasks);
  BatchTask t;
  t.out = as_global(c[i].out);
  t.in = as_global(c[i].in);
  t.in2 = as_global(c[i].in2);
  t.tmp = as_global(c[i].tmp);
  t.plan = c[i].plan;
  t.logN = c[i].logN;
  t.op = c[i].op;
  return t;
}
__device__ __forceinline__ PlanView load_plan_batch(const u64* plan, bool fwd, u64 N) {
  const NTTAMD_CONST PlanHeader* h = (const NTTAMD_CONST PlanHeader*)plan;
  PlanView v;
  v.q = h->q;
  v.q2 = h->q2;
  v.nq = h->nq;
  v.nq2 = 0 - h->q2;
  v.ninv = h->ninv;
  v.ninv_p = h->ninv_p;
  v.wn = h->wn;
  v.wn_p = h->wn_p;
  v.bk = h->barrett_k;
  v.qbits = (u32)h->qbits;
  v.q3 = h->q + h->q2;
  v.q4 = 2 * h->q2;
  v.nq4 = 0 - v.q4;
  v.rq = h->barrett_k >> (v.qbits - 1);
  v.tw = reinterpret_cast<const ulonglong2*>(as_global(plan) + kPlanHeaderWords) + (fwd ? 0 : N);
  v.twp = v.tw + 2 * N;
  return v;
}

// Runs the units of block bk from the claimed unit u on, claiming the next unit
// after each, and returns the first claimed unit outside the block.  body(k, t,
// active, h) runs sub-task k with sub-group thread t in sub-group h; a
// sub-group past the block's last sub-task repeats the unit's first one with
// active false (every barrier is still reached, nothing is stored).
template <typename F>
__device__ __forceinline__ u32 run_block(const BatchBlock& bk_in, u32* ctr_in, u32* claimed_in, u32 u, u32 g, F&& body) {
  const u32 unit0 = rfl(bk_in.unit0), units = rfl(bk_in.units);
  const u32 subs = rfl(bk_in.subs), last = rfl(bk_in.last);
  u32* ctr = uniform_ptr(ctr_in);
  u32* claimed = uniform_ptr(claimed_in);
  const u32 nt = kBatchThreads / g;             // a multiple of the wave size
  const u32 h = rfl(threadIdx.x / nt), t = threadIdx.x % nt;
#pragma unroll 1
  for (;;) {
    const u32 k0 = (u - unit0) * g;
    const bool active = k0 + h < subs;
    // the next claim is issued before this unit's work, which hides its latency
    u32 next = 0;
    if (threadIdx.x == 0) next = atomicAdd(ctr, 1u);
    // a fresh view of t per unit: the per-thread address terms are recomputed
    // inside the unit rather than held in registers across the loop
    body(active ? k0 + h : k0, opaque(t), active, h);
    __syncthreads();                            // LDS reuse, and every thread has read `claimed`
    if (threadIdx.x == 0) {
      *claimed = next;
      if (next == last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    u = rfl(*claimed);
    if (u - unit0 >= units) return u;
  }
}

// Class bodies are inlined into the kernel for the classes a batch holds most
// often (the wide-range single-pass transforms, the tiles at twice the threads:
// see pick_onchip and pick_tile); the other classes run as separate functions,
// which bounds the build's size and time but costs a call: the callee saves and
// restores 48 VGPRs per lane (192 KiB per workgroup) each time a workgroup
// enters such a block.

// Whole single-pass transforms (N <= 2^14).
template <bool FWD, int LOGN, int MODE, bool WIDE, int SHAPE = 0>
__device__ __forceinline__ u32 class_onchip_in(const BatchTask* tasks, const BatchBlock& bk, u32* ctr,
                                                      u32* claimed, u32 u, u32* lds) {
  constexpr int LOGR = batch_logr(LOGN, SHAPE);
  constexpr bool SPLIT = LOGN >= 13;
  using K = OnChip<FWD, LOGN, LOGR, SPLIT, true, WIDE>;
  constexpr int G = onchip_groups(LOGN, SHAPE);
  static_assert(G >= 1, "a limb needs more threads than a workgroup has");
  static_assert(G * K::LDSW * sizeof(typename K::W) <= kBatchLdsWords32 * 4, "sub-group exchange buffers exceed LDS");
  return run_block(bk, ctr, claimed, u, G, [&](u32 k, u32 t, bool active, u32 h) {
    const BatchTask tk = load_task(tasks, rfl(bk.desc0 + k));
    const PlanView pv = load_plan_batch(tk.plan, FWD, 1ull << LOGN);
    typename K::W* l = reinterpret_cast<typename K::W*>(lds) + h * K::LDSW;
    onchip_body<FWD, LOGN, LOGR, SPLIT, MODE, true, WIDE, true>(pv, tk.in, tk.out, nullptr, l, true, t, active);
  });
}

template <bool FWD, int LOGN, int MODE, bool WIDE, int SHAPE = 0>
__device__ __attribute__((noinline)) u32 class_onchip(const BatchTask* tasks, const BatchBlock bk, u32* ctr,
                                                      u32* claimed, u32 u, u32* lds) {
  return class_onchip_in<FWD, LOGN, MODE, WIDE, SHAPE>(tasks, bk, ctr, claimed, u, lds);
}

// Whole products on chip: out <- NTT(a) lazy, then out <- InvNTT(NTT(b) (.) out)
// canonical (the product listing of Section 4).
template <int LOGN, bool WIDE>
__device__ __attribute__((noinline)) u32 class_product_onchip(const BatchTask* tasks, const BatchBlock bk, u32* ctr,
                                                              u32* claimed, u32 u, u32* lds) {
  constexpr int LOGR = onchip_logr(LOGN);
  constexpr bool SPLIT = LOGN >= 13;
  using K = OnChip<true, LOGN, LOGR, SPLIT, true, WIDE>;
  constexpr int G = onchip_groups(LOGN);
  static_assert(G * K::LDSW * sizeof(typename K::W) <= kBatchLdsWords32 * 4, "sub-group exchange buffers exceed LDS");
  return run_block(bk, ctr, claimed, u, G, [&](u32 k, u32 t, bool active, u32 h) {
    const BatchTask tk = load_task(tasks, rfl(bk.desc0 + k));
    const PlanView pf = load_plan_batch(tk.plan, true, 1ull << LOGN);
    typename K::W* l = reinterpret_cast<typename K::W*>(lds) + h * K::LDSW;
    onchip_body<true, LOGN, LOGR, SPLIT, kOutLazy, true, WIDE, true>(pf, tk.in, tk.out, nullptr, l, true, t, active);
    __syncthreads();                            // NTT(a) in out, read back by other threads of the sub-group
    const PlanView pi = load_plan_batch(tk.plan, false, 1ull << LOGN);
    onchip_product_body<LOGN, LOGR, SPLIT, kOutCanon, true, WIDE, true>(pf, pi, tk.in2, tk.out, tk.out, l, true, t, active);
  });
}

// Both passes of a two-pass transform by one workgroup (512 threads, tiles of
// 4096 coefficients, 8 per thread); `mid` receives the first pass.
template <bool FWD, int LOGN, int MODE>
__device__ __forceinline__ void twopass_whole(const PlanView& pv, const u64* in, u64* mid, u64* out, const u64* mul,
                                              u64* lds, bool nt) {
  constexpr int LT_LO = mp_logt_lo(LOGN);
  constexpr int LT_HI = LOGN - LT_LO;
  constexpr int LC_HI = 12 - LT_HI;           // columns per high-pass tile
  constexpr int LH_LO = 12 - LT_LO;           // blocks per low-pass tile
  constexpr int TILES = 1 << (LOGN - 12);
  const u32 t = threadIdx.x;
#pragma unroll 1
  for (int step = 0; step < 2; ++step) {
    const bool hi = FWD ? step == 0 : step == 1;
    const bool last = step == 1;
    const u64* src = step == 0 ? in : mid;
    u64* dst = step == 0 ? mid : out;
#pragma unroll 1
    for (u32 tile = 0; tile < (u32)TILES; ++tile) {
      if (hi) {
        if (last) tile_body<FWD, LT_HI, 3, LC_HI, 0, MODE, true, -1, true>(pv, LOGN, LT_LO, tile, src, dst, mul, lds, false, t, true);
        else tile_body<FWD, LT_HI, 3, LC_HI, 0, kOutLazy, false, -1, true>(pv, LOGN, LT_LO, tile, src, dst, mul, lds, nt, t, true);
      } else {
        if (last) tile_body<FWD, LT_LO, 3, 0, LH_LO, MODE, true, -1, true>(pv, LOGN, 0, tile, src, dst, mul, lds, false, t, true);
        else tile_body<FWD, LT_LO, 3, 0, LH_LO, kOutLazy, false, -1, true>(pv, LOGN, 0, tile, src, dst, mul, lds, nt, t, true);
      }
      __syncthreads();
    }
  }
}

// Whole products with N >= 2^15, one per workgroup: out <- NTT(a) lazy;
// out <- NTT(b) (.) out (first pass of NTT(b) in tmp); out <- InvNTT(out).
template <int LOGN>
__device__ __attribute__((noinline)) u32 class_product_twopass(const BatchTask* tasks, const BatchBlock bk, u32* ctr,
                                                               u32* claimed, u32 u, u32* lds) {
  u64* l64 = reinterpret_cast<u64*>(lds);
  return run_block(bk, ctr, claimed, u, 1, [&](u32 k, u32, bool, u32) {
    const BatchTask tk = load_task(tasks, rfl(bk.desc0 + k));
    const PlanView pf = load_plan_batch(tk.plan, true, 1ull << LOGN);
    twopass_whole<true, LOGN, kOutLazy>(pf, tk.in, tk.out, tk.out, nullptr, l64, true);
    twopass_whole<true, LOGN, kOutMul>(pf, tk.in2, tk.tmp, tk.out, tk.out, l64, true);
    const PlanView pi = load_plan_batch(tk.plan, false, 1ull << LOGN);
    twopass_whole<false, LOGN, kOutCanon>(pi, tk.out, tk.out, tk.out, nullptr, l64, false);
  });
}

// Tiles of one pass (PASS 0: in -> out, lazy; PASS 1: out -> out with the output
// MODE) of split two-pass transforms: two 4096-coefficient tiles per unit, 256
// threads and 16 coefficients each, the multi-pass kernels' own tile shape (the
// low pass reads the transposed sub-tables).  Sub-task k is tile k mod T of the
// block's task k / T, T = N / 4096.
template <bool FWD, int LOGN, int MODE, int PASS, int SHAPE = 0>
__device__ __forceinline__ u32 class_tile_in(const BatchTask* tasks, const BatchBlock& bk, u32* ctr,
                                                    u32* claimed, u32 u, u32* lds) {
  constexpr int LT_LO = mp_logt_lo(LOGN);
  constexpr int LT_HI = LOGN - LT_LO;
  constexpr int LC_HI = 12 - LT_HI;
  constexpr int LH_LO = 12 - LT_LO;
  constexpr int TSH = LOGN - 12;
  constexpr bool HI = FWD ? PASS == 0 : PASS == 1;
  // shape 0: 16 coefficients per thread, the low pass on the transposed sub-tables; shape 1: 8,
  // twice the threads per tile, natural tables
  constexpr int LOGR = kMpLogrLo - SHAPE;
  constexpr int PTOP = SHAPE == 0 ? mp_perm_top(FWD, LOGN) : -1;
  constexpr int G = kBatchThreads / (4096 >> LOGR);
  constexpr int TILE_LDS = 4096 + (4096 >> LOGR);   // u64 words of one tile's exchange buffer
  static_assert(G * TILE_LDS * 2 <= kBatchLdsWords32, "tile exchange buffers exceed LDS");
  return run_block(bk, ctr, claimed, u, G, [&](u32 k, u32 t, bool active, u32 h) {
    const BatchTask tk = load_task(tasks, rfl(bk.desc0 + (k >> TSH)));
    const u32 tile = rfl(k & ((1u << TSH) - 1u));
    const PlanView pv = load_plan_batch(tk.plan, FWD, 1ull << LOGN);
    u64* l = reinterpret_cast<u64*>(lds) + h * TILE_LDS;
    if constexpr (HI) {
      if constexpr (PASS == 0)
        tile_body<FWD, LT_HI, LOGR, LC_HI, 0, kOutLazy, false, -1, true>(pv, LOGN, LT_LO, tile, tk.in, tk.out, nullptr, l, true, t, active);
      else
        tile_body<FWD, LT_HI, LOGR, LC_HI, 0, MODE, true, -1, true>(pv, LOGN, LT_LO, tile, tk.out, tk.out, nullptr, l, false, t, active);
    } else {
      if constexpr (PASS == 0)
        tile_body<FWD, LT_LO, LOGR, 0, LH_LO, kOutLazy, false, PTOP, true>(pv, LOGN, 0, tile, tk.in, tk.out, nullptr, l, true, t, active);
      else
        tile_body<FWD, LT_LO, LOGR, 0, LH_LO, MODE, true, PTOP, true>(pv, LOGN, 0, tile, tk.out, tk.out, nullptr, l, false, t, active);
    }
  });
}

template <bool FWD, int LOGN, int MODE, int PASS, int SHAPE = 0>
__device__ __attribute__((noinline)) u32 class_tile(const BatchTask* tasks, const BatchBlock bk, u32* ctr,
                                                    u32* claimed, u32 u, u32* lds) {
  return class_tile_in<FWD, LOGN, MODE, PASS, SHAPE>(tasks, bk, ctr, claimed, u, lds);
}

// A block of a class this kernel does not know: claims past it.
__device__ __attribute__((noinline)) u32 class_skip(const BatchBlock bk, u32* ctr, u32* claimed, u32 u) {
  return run_block(bk, ctr, claimed, u, 1, [](u32, u32, bool, u32) {});
}

template <bool FWD, int MODE, bool WIDE>
__device__ __forceinline__ u32 pick_onchip(u32 logN, u32 shape, const BatchTask* tasks, const BatchBlock& bk, u32* ctr,
                                           u32* claimed, u32 u, u32* lds) {
  if (shape) {
    switch (logN) {                            // shape 1 exists where a limb fits 512 threads
      case 10: return class_onchip<FWD, 10, MODE, WIDE, 1>(tasks, bk, ctr, claimed, u, lds);
      case 11: return class_onchip<FWD, 11, MODE, WIDE, 1>(tasks, bk, ctr, claimed, u, lds);
      case 12: return class_onchip<FWD, 12, MODE, WIDE, 1>(tasks, bk, ctr, claimed, u, lds);
      case 13: return class_onchip<FWD, 13, MODE, WIDE, 1>(tasks, bk, ctr, claimed, u, lds);
      default: return class_skip(bk, ctr, claimed, u);
    }
  }
  if constexpr (WIDE) {                         // inlined: the usual case (moduli below 2^58)
    switch (logN) {
      case 10: return class_onchip_in<FWD, 10, MODE, true>(tasks, bk, ctr, claimed, u, lds);
      case 11: return class_onchip_in<FWD, 11, MODE, true>(tasks, bk, ctr, claimed, u, lds);
      case 12: return class_onchip_in<FWD, 12, MODE, true>(tasks, bk, ctr, claimed, u, lds);
      case 13: return class_onchip_in<FWD, 13, MODE, true>(tasks, bk, ctr, claimed, u, lds);
      case 14: return class_onchip_in<FWD, 14, MODE, true>(tasks, bk, ctr, claimed, u, lds);
      default: break;
    }
  }
  switch (logN) {
    case 10: return class_onchip<FWD, 10, MODE, WIDE>(tasks, bk, ctr, claimed, u, lds);
    case 11: return class_onchip<FWD, 11, MODE, WIDE>(tasks, bk, ctr, claimed, u, lds);
    case 12: return class_onchip<FWD, 12, MODE, WIDE>(tasks, bk, ctr, claimed, u, lds);
    case 13: return class_onchip<FWD, 13, MODE, WIDE>(tasks, bk, ctr, claimed, u, lds);
    case 14: return class_onchip<FWD, 14, MODE, WIDE>(tasks, bk, ctr, claimed, u, lds);
    default: return class_skip(bk, ctr, claimed, u);
  }
}

template <bool FWD, int MODE, int PASS>
__device__ __forceinline__ u32 pick_tile(u32 logN, u32 shape, const BatchTask* tasks, const BatchBlock& bk, u32* ctr,
                                         u32* claimed, u32 u, u32* lds) {
  if (shape) {                                  // inlined: the autotuner's usual choice
    switch (logN) {
      case 15: return class_tile_in<FWD, 15, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
      case 16: return class_tile_in<FWD, 16, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
      case 17: return class_tile_in<FWD, 17, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
      default: break;
    }
  }
  switch (logN * 2 + (shape ? 1 : 0)) {
    case 30: return class_tile<FWD, 15, MODE, PASS>(tasks, bk, ctr, claimed, u, lds);
    case 31: return class_tile<FWD, 15, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
    case 32: return class_tile<FWD, 16, MODE, PASS>(tasks, bk, ctr, claimed, u, lds);
    case 33: return class_tile<FWD, 16, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
    case 34: return class_tile<FWD, 17, MODE, PASS>(tasks, bk, ctr, claimed, u, lds);
    case 35: return class_tile<FWD, 17, MODE, PASS, 1>(tasks, bk, ctr, claimed, u, lds);
    default: return class_skip(bk, ctr, claimed, u);
  }
}

template <int PASS>
__device__ __forceinline__ u32 pick_tile_op(u32 op, u32 logN, u32 shape, const BatchTask* tasks, const BatchBlock& bk,
                                            u32* ctr, u32* claimed, u32 u, u32* lds) {
  switch (op) {
    case kBatchFwdLazy: return pick_tile<true, kOutLazy, PASS>(logN, shape, tasks, bk, ctr, claimed, u, lds);
    case kBatchFwdCanon: return pick_tile<true, kOutCanon, PASS>(logN, shape, tasks, bk, ctr, claimed, u, lds);
    case kBatchInvLazy: return pick_tile<false, kOutLazy, PASS>(logN, shape, tasks, bk, ctr, claimed, u, lds);
    case kBatchInvCanon: return pick_tile<false, kOutCanon, PASS>(logN, shape, tasks, bk, ctr, claimed, u, lds);
    default: return class_skip(bk, ctr, claimed, u);
  }
}

__device__ __forceinline__ u32 run_class(const BatchTask* tasks, const BatchBlock& bk, u32* ctr, u32* claimed, u32 u,
                                         u32* lds) {
  const u32 kind = bk.cls & 7u, logN = (bk.cls >> 3) & 31u, op = (bk.cls >> 8) & 7u;
  const bool wide = (bk.cls >> 11) & 1u;
  const u32 shape = (bk.cls >> 12) & 1u;
  switch (kind) {
    case kClassOnchip:
      switch (op) {
        case kBatchFwdLazy:
          return wide ? pick_onchip<true, kOutLazy, true>(logN, shape, tasks, bk, ctr, claimed, u, lds)
                      : pick_onchip<true, kOutLazy, false>(logN, shape, tasks, bk, ctr, claimed, u, lds);
        case kBatchFwdCanon:
          return wide ? pick_onchip<true, kOutCanon, true>(logN, shape, tasks, bk, ctr, claimed, u, lds)
                      : pick_onchip<true, kOutCanon, false>(logN, shape, tasks, bk, ctr, claimed, u, lds);
        case kBatchInvLazy:
          return wide ? pick_onchip<false, kOutLazy, true>(logN, shape, tasks, bk, ctr, claimed, u, lds)
                      : pick_onchip<false, kOutLazy, false>(logN, shape, tasks, bk, ctr, claimed, u, lds);
        case kBatchInvCanon:
          return wide ? pick_onchip<false, kOutCanon, true>(logN, shape, tasks, bk, ctr, claimed, u, lds)
                      : pick_onchip<false, kOutCanon, false>(logN, shape, tasks, bk, ctr, claimed, u, lds);
        default: return class_skip(bk, ctr, claimed, u);
      }
    case kClassProduct:
      switch (logN) {
        case 10: return wide ? class_product_onchip<10, true>(tasks, bk, ctr, claimed, u, lds) : class_product_onchip<10, false>(tasks, bk, ctr, claimed, u, lds);
        case 11: return wide ? class_product_onchip<11, true>(tasks, bk, ctr, claimed, u, lds) : class_product_onchip<11, false>(tasks, bk, ctr, claimed, u, lds);
        case 12: return wide ? class_product_onchip<12, true>(tasks, bk, ctr, claimed, u, lds) : class_product_onchip<12, false>(tasks, bk, ctr, claimed, u, lds);
        case 13: return wide ? class_product_onchip<13, true>(tasks, bk, ctr, claimed, u, lds) : class_product_onchip<13, false>(tasks, bk, ctr, claimed, u, lds);
        case 14: return wide ? class_product_onchip<14, true>(tasks, bk, ctr, claimed, u, lds) : class_product_onchip<14, false>(tasks, bk, ctr, claimed, u, lds);
        case 15: return class_product_twopass<15>(tasks, bk, ctr, claimed, u, lds);
        case 16: return class_product_twopass<16>(tasks, bk, ctr, claimed, u, lds);
        case 17: return class_product_twopass<17>(tasks, bk, ctr, claimed, u, lds);
        default: return class_skip(bk, ctr, claimed, u);
      }
    case kClassTile0: return pick_tile_op<0>(op, logN, shape, tasks, bk, ctr, claimed, u, lds);
    case kClassTile1: return pick_tile_op<1>(op, logN, shape, tasks, bk, ctr, claimed, u, lds);
    default: return class_skip(bk, ctr, claimed, u);
  }
}

// One phase of a batch.  Phase 0 runs the whole tasks and the first pass of
// every split two-pass transform, phase 1 the last passes: the launch boundary
// orders the two passes of a split transform, so no workgroup waits on another.
// Units are claimed in increasing order, so each workgroup walks the phase's
// blocks forwards.
__global__ void __launch_bounds__(kBatchThreads, 4)
    ntt_batch_kernel(const BatchTask* __restrict__ tasks, const BatchHead* __restrict__ head, u32* counter, u32 phase) {
  __shared__ u32 lds[kBatchLdsWords32];
  __shared__ u32 claimed;
  const u32 b_first = phase ? head->blocks[0] : 0u;
  const u32 b_end = b_first + head->blocks[phase];
  u32* ctr = counter + phase;
  // Every workgroup makes exactly one claim past the phase's units, so the claim
  // values end at units + grid - 1; the workgroup that draws that value has seen
  // every claim of the launch performed and clears the counter for the next run.
  const u32 last = head->units[phase] + gridDim.x - 1u;
  if (threadIdx.x == 0) {
    claimed = atomicAdd(ctr, 1u);
    if (claimed == last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  u32 u = rfl(claimed);
  u32 b = b_first;
#pragma unroll 1
  for (;;) {
    while (b < b_end && u - head->block[b].unit0 >= head->block[b].units) ++b;
    if (b >= b_end) break;                      // every wave of every workgroup reaches this exit
    BatchBlock bk = head->block[b];
    bk.last = last;
    u = run_class(tasks, bk, ctr, &claimed, u, lds);
  }
}

// ---- host side ----------------------------------------------------------------

uint32_t batch_wide_flag(uint32_t logN, uint64_t q) {
  return (wide_range_enabled() && logN <= (uint32_t)kMaxOnchipLog && q < kWideModulusBound) ? kBatchWide : 0u;
}

// The task's operation from the item's op and modulus factors (0 = the op's own).
static uint32_t default_in_f(uint32_t op) { return (op == kBatchInvLazy || op == kBatchInvCanon) ? 2u : 1u; }

static ntt_status item_op(const ntt_batch_item& it, uint32_t* op, uint32_t* in_f) {
  const uint32_t fi = it.input_mod_factor ? it.input_mod_factor : default_in_f(it.op);
  const uint32_t fo = it.output_mod_factor;
  switch (it.op) {
    case kBatchFwdLazy:
    case kBatchFwdCanon:
      if (!(fi == 1 || fi == 2 || fi == 4) || !(fo == 0 || fo == 1 || fo == 4)) return NTT_EINVAL_FACTOR;
      *op = fo == 0 ? it.op : (fo == 1 ? kBatchFwdCanon : kBatchFwdLazy);
      break;
    case kBatchInvLazy:
    case kBatchInvCanon:
      if (!(fi == 1 || fi == 2) || !(fo == 0 || fo == 1 || fo == 2)) return NTT_EINVAL_FACTOR;
      *op = fo == 0 ? it.op : (fo == 1 ? kBatchInvCanon : kBatchInvLazy);
      break;
    case kBatchProduct:
      if (!(fi == 1 || fi == 2 || fi == 4) || !(fo == 0 || fo == 1)) return NTT_EINVAL_FACTOR;
      *op = kBatchProduct;
      break;
    default:
      return NTT_EINVAL_FACTOR;
  }
  *in_f = fi;
  return NTT_OK;
}

static ntt_status wait_staging(ntt_batch* b) {
  ntt_batch_stage& g = cur_stage(b);
  if (g.pending) {
    if (hipEventSynchronize(g.done) != hipSuccess) return NTT_EDEVICE;   // this staging set still in use
    g.pending = false;
  }
  return NTT_OK;
}

// Class of a task, sub-tasks per descriptor (log2) and sub-tasks per unit.
struct TaskClass {
  uint32_t cls, tshift, g;
  uint64_t cost;            // time of one unit, in coefficient-stages per thread (orders the blocks)
};
static TaskClass classify(const BatchTask& t, int shape) {
  const uint32_t op = t.op & kBatchOpMask;
  const uint32_t wide = (t.op & kBatchWide) ? 1u : 0u;
  const uint32_t logN = t.logN;
  TaskClass c{};
  if (logN <= (uint32_t)kMaxOnchipLog) {
    // shape 1 for transforms whose limb fits one workgroup at twice the threads (N <= 2^13)
    const uint32_t sh = (shape == 1 && op != kBatchProduct && logN < (uint32_t)kMaxOnchipLog) ? 1u : 0u;
    const uint64_t per_thread = (uint64_t)1 << batch_logr((int)logN, (int)sh);
    c.g = (uint32_t)onchip_groups((int)logN, (int)sh);
    if (op == kBatchProduct) {
      c.cls = kClassProduct | logN << 3 | op << 8 | wide << 11;
      c.cost = 3 * per_thread * logN;
    } else {
      c.cls = kClassOnchip | logN << 3 | op << 8 | wide << 11 | sh << 12;
      c.cost = per_thread * logN;
    }
  } else if (op == kBatchProduct) {
    c.cls = kClassProduct | logN << 3 | op << 8;
    c.g = 1;
    c.cost = 3 * 8 * (uint64_t)logN << (logN - 12);   // three two-pass transforms of N / 4096 tiles each
  } else {
    const uint32_t sh = shape >= 1 ? 1u : 0u;       // shapes 1 and 2
    c.cls = kClassTile0 | logN << 3 | op << 8 | sh << 12;
    c.tshift = logN - 12;
    c.g = sh ? 1 : 2;
    c.cost = (sh ? 8 : 16) * (uint64_t)(logN + 1) / 2;
  }
  return c;
}

// Groups of tasks of one (class, plan): found through a small open-addressing
// table, so that ordering a batch costs O(tasks) plus a sort of the groups.
struct TaskGroup {
  uint64_t cost;
  uint32_t cls;
  const uint64_t* plan;
  uint32_t count, next;
};
class GroupTable {
 public:
  explicit GroupTable(size_t expect) {
    size_t cap = 64;
    while (cap < 2 * expect && cap < ((size_t)1 << 20)) cap <<= 1;
    slots_.assign(cap, kEmpty);
  }
  // index of the group of (cls, plan) in groups, created (count 0) on first use
  uint32_t find(std::vector<TaskGroup>& groups, const TaskClass& c, const uint64_t* plan) {
    if (2 * (groups.size() + 1) > slots_.size()) grow(groups);
    const uint64_t key = ((uint64_t)(uintptr_t)plan << 12) ^ c.cls;
    size_t i = mix(key) & (slots_.size() - 1);
    for (;;) {
      const uint32_t g = slots_[i];
      if (g == kEmpty) {
        groups.push_back(TaskGroup{c.cost, c.cls, plan, 0, 0});
        slots_[i] = (uint32_t)(groups.size() - 1);
        return slots_[i];
      }
      if (groups[g].cls == c.cls && groups[g].plan == plan) return g;
      i = (i + 1) & (slots_.size() - 1);
    }
  }

 private:
  static constexpr uint32_t kEmpty = 0xffffffffu;
  static size_t mix(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (size_t)x;
  }
  void grow(const std::vector<TaskGroup>& groups) {
    slots_.assign(slots_.size() * 2, kEmpty);
    for (uint32_t g = 0; g < groups.size(); ++g) {
      const uint64_t key = ((uint64_t)(uintptr_t)groups[g].plan << 12) ^ groups[g].cls;
      size_t i = mix(key) & (slots_.size() - 1);
      while (slots_[i] != kEmpty) i = (i + 1) & (slots_.size() - 1);
      slots_[i] = g;
    }
  }
  std::vector<uint32_t> slots_;
};

static ntt_status stage_units(ntt_batch* b, const std::vector<BatchTask>& list, size_t* staged) {
  const size_t n = list.size();
  std::vector<TaskClass> cl(n);
  std::vector<uint32_t> gid(n);
  std::vector<TaskGroup> groups;
  GroupTable table(64);
  for (size_t k = 0; k < n; ++k) {
    cl[k] = classify(list[k], b->shape);
    gid[k] = table.find(groups, cl[k], list[k].plan);
    ++groups[gid[k]].count;
  }
  // groups in block order, then each task at its group's next slot (item order within a group)
  std::vector<uint32_t> gorder(groups.size());
  for (uint32_t g = 0; g < groups.size(); ++g) gorder[g] = g;
  std::sort(gorder.begin(), gorder.end(), [&](uint32_t x, uint32_t y) {
    const TaskGroup &a = groups[x], &c = groups[y];
    if (a.cost != c.cost) return a.cost > c.cost;
    if (a.cls != c.cls) return a.cls < c.cls;
    return a.plan < c.plan;
  });
  uint32_t pos = 0;
  for (uint32_t g : gorder) {
    groups[g].next = pos;
    pos += groups[g].count;
  }
  std::vector<size_t> order(n);
  for (size_t k = 0; k < n; ++k) order[groups[gid[k]].next++] = k;
  BatchTask* dst = staged_tasks(b);
  BatchHead* head = staged_head(b);
  std::vector<BatchBlock> p0, p1;
  for (size_t w = 0; w < n; ++w) {
    const size_t k = order[w];
    dst[w] = list[k];
    const TaskClass& c = cl[k];
    if (p0.empty() || p0.back().cls != c.cls) {
      BatchBlock bk{};
      bk.unit0 = p0.empty() ? 0u : p0.back().unit0 + p0.back().units;
      bk.desc0 = (uint32_t)w;
      bk.cls = c.cls;
      p0.push_back(bk);
    }
    BatchBlock& bk = p0.back();
    bk.subs += 1u << c.tshift;
    bk.units = (bk.subs + c.g - 1) / c.g;
  }
  for (const BatchBlock& bk : p0) {
    if ((bk.cls & 7u) != kClassTile0) continue;
    BatchBlock b1 = bk;
    b1.cls = (bk.cls & ~7u) | kClassTile1;
    b1.unit0 = p1.empty() ? 0u : p1.back().unit0 + p1.back().units;
    p1.push_back(b1);
  }
  if (p0.size() + p1.size() > (size_t)kMaxBlocks) return NTT_EINVAL_COUNT;   // not reachable: one block per class
  *head = BatchHead{};
  head->blocks[0] = (uint32_t)p0.size();
  head->blocks[1] = (uint32_t)p1.size();
  head->units[0] = p0.empty() ? 0u : p0.back().unit0 + p0.back().units;
  head->units[1] = p1.empty() ? 0u : p1.back().unit0 + p1.back().units;
  std::copy(p0.begin(), p0.end(), head->block);
  std::copy(p1.begin(), p1.end(), head->block + p0.size());
  *staged = n;
  return NTT_OK;
}

ntt_status batch_prepare(ntt_batch* b, const ntt_batch_item* items, size_t count, size_t* out_count) {
  ntt_status st0 = wait_staging(b);
  if (st0) return st0;
  for (size_t i = 0; i < count; ++i) {
    const ntt_batch_item& it = items[i];
    if (!it.out || !it.in) return NTT_EINVAL_POINTER;
    ntt_status st = validate_degree(it.N);
    if (st) return st;
    if (it.N < 1024) return NTT_EINVAL_DEGREE;
    int logN = 0;
    while ((1ull << logN) < it.N) ++logN;
    uint32_t op = 0, in_f = 1;
    st = item_op(it, &op, &in_f);
    if (st) return st;
    if (it.op == kBatchProduct && !it.in2) return NTT_EINVAL_POINTER;
    if (it.op == kBatchProduct && logN > kMaxOnchipLog && !it.tmp) return NTT_EINVAL_POINTER;
    const size_t bytes = (size_t)it.N * sizeof(uint64_t);
    const uintptr_t o0 = (uintptr_t)it.out, i0 = (uintptr_t)it.in;
    if (it.out != it.in && o0 < i0 + bytes && i0 < o0 + bytes) return NTT_EALIAS;
    if (it.op == kBatchProduct) {
      const uintptr_t b0 = (uintptr_t)it.in2;
      if (o0 < b0 + bytes && b0 < o0 + bytes) return NTT_EALIAS;
      if (logN > kMaxOnchipLog) {
        const uintptr_t w0 = (uintptr_t)it.tmp;
        if ((w0 < o0 + bytes && o0 < w0 + bytes) || (w0 < b0 + bytes && b0 < w0 + bytes) ||
            (w0 < i0 + bytes && i0 < w0 + bytes))
          return NTT_EALIAS;
      }
    }
  }
  // in item order: the staging sorts the tasks into class blocks.  One library cache lookup per
  // distinct (N, q), remembered in a small direct-mapped table in front of a map.
  struct Seen { uint64_t N, q; const ntt_plan* p; };
  Seen recent[64] = {};
  std::map<std::pair<uint64_t, uint64_t>, const ntt_plan*> seen;
  std::vector<BatchTask> list(count);
  for (size_t k = 0; k < count; ++k) {
    const ntt_batch_item& it = items[k];
    Seen& r = recent[(it.q ^ (it.q >> 17) ^ it.N) & 63u];
    const ntt_plan* p = (r.p && r.N == it.N && r.q == it.q) ? r.p : nullptr;
    if (!p) {
      const ntt_plan*& m = seen[{it.N, it.q}];
      if (!m) {
        ntt_status st = cached_plan(it.N, it.q, &m);
        if (st) return st;
      }
      p = m;
      r = Seen{it.N, it.q, p};
    }
    BatchTask& t = list[k];
    uint32_t op = 0, in_f = 1;
    (void)item_op(it, &op, &in_f);                 // validated above
    t.out = it.out;
    t.in = it.in;
    t.in2 = it.in2;
    t.tmp = it.tmp;
    t.plan = p->dev;
    t.logN = (uint32_t)p->logN;
    t.op = op | batch_wide_flag(t.logN, it.q);
  }
  return stage_units(b, list, out_count);
}

int batch_grid(const ntt_batch* b, size_t count) {
  int g = b->grid;
  if (g <= 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    g = 2 * cus;                                // two 512-thread workgroups per CU (66 KiB LDS each)
  }
  if ((size_t)g > count) g = (int)count;
  return g < 1 ? 1 : g;
}

// Copies the staged head and `staged` descriptors to the device, on the
// context's copy stream (ordered before `stream`'s next work by an event, so it
// overlaps whatever `stream` is still running; the staging set it overwrites
// is idle, see wait_staging), or on `stream` itself.
void batch_use_copy_stream(ntt_batch* b, bool on) { b->use_copy_stream = on; }

static ntt_status batch_copy(ntt_batch* b, size_t staged, hipStream_t stream) {
  ntt_batch_stage& g = cur_stage(b);
  if (b->use_copy_stream && !b->copy_stream &&
      hipStreamCreateWithFlags(&b->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    b->copy_stream = nullptr;
    b->use_copy_stream = false;                     // copies go on the launch stream
  }
  if (b->use_copy_stream) {
    if (hipMemcpyAsync(g.dev + kDevHead, g.host, stage_bytes(staged), hipMemcpyHostToDevice, b->copy_stream) !=
            hipSuccess ||
        hipEventRecord(g.copied, b->copy_stream) != hipSuccess || hipStreamWaitEvent(stream, g.copied, 0) != hipSuccess)
      return NTT_EDEVICE;
    return NTT_OK;
  }
  return hipMemcpyAsync(g.dev + kDevHead, g.host, stage_bytes(staged), hipMemcpyHostToDevice, stream) == hipSuccess
             ? NTT_OK
             : NTT_EDEVICE;
}

// Enqueues [phase 0, phase 1] of staging set g on `stream`; `phase1` false
// leaves out the second launch (nothing was split).
static ntt_status batch_enqueue(ntt_batch_stage& g, int grid, hipStream_t stream, bool phase1) {
  u32* counter = reinterpret_cast<u32*>(g.dev);
  const BatchHead* head = reinterpret_cast<const BatchHead*>(g.dev + kDevHead);
  const BatchTask* tasks = reinterpret_cast<const BatchTask*>(g.dev + kDevHead + kStageHead);
  hipLaunchKernelGGL(ntt_batch_kernel, dim3(grid), dim3(kBatchThreads), 0, stream, tasks, head, counter, 0u);
  if (phase1) hipLaunchKernelGGL(ntt_batch_kernel, dim3(grid), dim3(kBatchThreads), 0, stream, tasks, head, counter, 1u);
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

// Captures staging set sg's [phase 0, phase 1] with the full grid: the kernels
// read the blocks and counts from device memory.
static ntt_status batch_capture(ntt_batch* b, ntt_batch_stage& sg) {
  const int grid = batch_grid(b, (size_t)1 << 30);
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return NTT_EDEVICE;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return NTT_EDEVICE;
  }
  const ntt_status st = batch_enqueue(sg, grid, cap, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) return NTT_EDEVICE;
  if (hipGraphInstantiate(&sg.graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    sg.graph_exec = nullptr;
    (void)hipGraphDestroy(g);
    return NTT_EDEVICE;
  }
  sg.graph = g;
  return NTT_OK;
}

static ntt_status batch_launch_staged(ntt_batch* b, size_t n, hipStream_t s, bool graph) {
  ntt_batch_stage& sg = cur_stage(b);
  ntt_status st = batch_copy(b, n, s);
  if (st) return st;
  if (!graph) {
    const BatchHead* head = reinterpret_cast<const BatchHead*>(sg.host);
    st = batch_enqueue(sg, batch_grid(b, std::max(head->units[0], head->units[1])), s, head->units[1] != 0);
    if (st) return st;
  } else {
    // both staging sets are captured at once, so that no later run pays for an instantiation
    for (ntt_batch_stage& h : b->stage) {
      if (h.graph_exec) continue;
      st = batch_capture(b, h);
      if (st) return st;
    }
    if (hipGraphLaunch(sg.graph_exec, s) != hipSuccess) return NTT_EDEVICE;
  }
  if (hipEventRecord(sg.done, s) != hipSuccess) return NTT_EDEVICE;
  sg.pending = true;
  b->cur ^= 1;
  return NTT_OK;
}

ntt_status batch_launch_tasks(ntt_batch* b, const BatchTask* tasks, size_t count, hipStream_t stream, bool graph) {
  if (count == 0) return NTT_OK;
  if (count > b->capacity) return NTT_EINVAL_COUNT;
  ntt_status st = wait_staging(b);
  if (st) return st;
  std::vector<BatchTask> list(tasks, tasks + count);
  size_t n = 0;
  st = stage_units(b, list, &n);
  if (st) return st;
  return batch_launch_staged(b, n, stream, graph);
}

}  // namespace nttamd

using namespace nttamd;

namespace nttamd {

static std::mutex g_oneshot_mu;
static std::map<std::pair<std::thread::id, int>, ntt_batch*> g_oneshot;

// Runs items whose ops are op_a or op_b through the calling thread's context on
// the current device, growing it (a new context of at least twice the size)
// when the list does not fit.
ntt_status oneshot_run(const ntt_batch_item* items, size_t count, ntt_stream_t stream, uint32_t op_a,
                       uint32_t op_b) {
  if (!items && count) return NTT_EINVAL_POINTER;
  if (count == 0) return NTT_OK;
  for (size_t i = 0; i < count; ++i)
    if (items[i].op != op_a && items[i].op != op_b) return NTT_EINVAL_FACTOR;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_EDEVICE;
  const auto key = std::make_pair(std::this_thread::get_id(), dev);
  ntt_batch* b = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_oneshot_mu);
    auto it = g_oneshot.find(key);
    if (it != g_oneshot.end()) b = it->second;
  }
  if (!b || b->capacity < count) {
    const size_t cap = b ? std::max(count, 2 * b->capacity) : std::max<size_t>(count, 1024);
    ntt_batch* nb = nullptr;
    ntt_status st = ntt_batch_create(&nb, cap);
    if (st) return st;
    if (b) (void)ntt_batch_destroy(b);          // waits for its launches in flight
    std::lock_guard<std::mutex> lk(g_oneshot_mu);
    g_oneshot[key] = nb;
    b = nb;
  }
  return ntt_batch_run_graph(b, items, count, stream);
}

void free_oneshot_batches() {
  std::lock_guard<std::mutex> lk(g_oneshot_mu);
  for (auto& kv : g_oneshot) (void)ntt_batch_destroy(kv.second);
  g_oneshot.clear();
}

}  // namespace nttamd

extern "C" {

static void release_stage(ntt_batch_stage& g) {
  if (g.pending) (void)hipEventSynchronize(g.done);
  if (g.graph_exec) (void)hipGraphExecDestroy(g.graph_exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.done) (void)hipEventDestroy(g.done);
  if (g.copied) (void)hipEventDestroy(g.copied);
  if (g.dev) (void)hipFree(g.dev);
  if (g.host) (void)hipHostFree(g.host);
  g = ntt_batch_stage{};
}

ntt_status ntt_batch_create(ntt_batch** out, size_t capacity) {
  if (!out) return NTT_EINVAL_POINTER;
  *out = nullptr;
  if (capacity == 0 || capacity > (1u << 24)) return NTT_EINVAL_COUNT;
  ntt_batch* b = new (std::nothrow) ntt_batch();
  if (!b) return NTT_ENOMEM;
  b->capacity = capacity;
  const size_t bytes = stage_bytes(capacity);
  if (hipGetDevice(&b->device) != hipSuccess) { delete b; return NTT_EDEVICE; }
  for (ntt_batch_stage& g : b->stage) {
    ntt_status st = NTT_OK;
    if (hipHostMalloc((void**)&g.host, bytes, hipHostMallocDefault) != hipSuccess) { g.host = nullptr; st = NTT_ENOMEM; }
    if (!st && hipMalloc((void**)&g.dev, dev_bytes(b)) != hipSuccess) { g.dev = nullptr; st = NTT_ENOMEM; }
    if (!st && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) { g.done = nullptr; st = NTT_EDEVICE; }
    if (!st && hipEventCreateWithFlags(&g.copied, hipEventDisableTiming) != hipSuccess) { g.copied = nullptr; st = NTT_EDEVICE; }
    // the claim counters start at zero; every phase leaves them at zero
    if (!st && hipMemset(g.dev, 0, kDevHead) != hipSuccess) st = NTT_EDEVICE;
    if (st) {
      for (ntt_batch_stage& h : b->stage) release_stage(h);
      if (b->copy_stream) (void)hipStreamDestroy(b->copy_stream);
      delete b;
      return st;
    }
  }
  b->use_copy_stream = true;                        // the stream itself is created on first use
  *out = b;
  return NTT_OK;
}

ntt_status ntt_batch_destroy(ntt_batch* b) {
  if (!b) return NTT_EINVAL_POINTER;
  for (ntt_batch_stage& g : b->stage) release_stage(g);
  if (b->copy_stream) (void)hipStreamDestroy(b->copy_stream);
  delete b;
  return NTT_OK;
}

ntt_status ntt_batch_set_grid(ntt_batch* b, int workgroups) {
  if (!b) return NTT_EINVAL_POINTER;
  if (workgroups < 0 || workgroups > (1 << 20)) return NTT_EINVAL_COUNT;
  for (ntt_batch_stage& g : b->stage) {
    if (g.graph_exec && workgroups != b->grid) {   // the captured launch has a fixed grid
      if (g.pending) (void)hipEventSynchronize(g.done);
      (void)hipGraphExecDestroy(g.graph_exec);
      (void)hipGraphDestroy(g.graph);
      g.graph_exec = nullptr;
      g.graph = nullptr;
    }
  }
  b->grid = workgroups;
  return NTT_OK;
}

ntt_status ntt_batch_get_config(const ntt_batch* b, int* workgroups, int* shape) {
  if (!b) return NTT_EINVAL_POINTER;
  if (workgroups) *workgroups = b->grid;
  if (shape) *shape = b->shape;
  return NTT_OK;
}

ntt_status ntt_batch_set_shape(ntt_batch* b, int shape) {
  if (!b) return NTT_EINVAL_POINTER;
  if (shape < 0 || shape > 2) return NTT_EINVAL_COUNT;
  b->shape = shape;                             // read when a batch is staged; graphs do not depend on it
  return NTT_OK;
}

// Validation mode: each task's inputs against its range (forward and product
// inputs below q, inverse inputs below 2q).
static ntt_status check_items(const ntt_batch_item* items, size_t count, hipStream_t stream) {
  if (!validate_enabled()) return NTT_OK;
  for (size_t i = 0; i < count; ++i) {
    const ntt_batch_item& it = items[i];
    const uint64_t f = it.input_mod_factor ? it.input_mod_factor : default_in_f(it.op);
    ntt_status st = check_range(it.in, 64, it.N, &it.q, 1, 1, f, stream);
    if (!st && it.op == NTT_BATCH_PRODUCT) st = check_range(it.in2, 64, it.N, &it.q, 1, 1, f, stream);
    if (st) return st;
  }
  return NTT_OK;
}

ntt_status ntt_batch_run(ntt_batch* b, const ntt_batch_item* items, size_t count, ntt_stream_t stream) {
  if (!b || (!items && count)) return NTT_EINVAL_POINTER;
  if (count > b->capacity) return NTT_EINVAL_COUNT;
  if (count == 0) return NTT_OK;
  size_t n = 0;
  ntt_status st = batch_prepare(b, items, count, &n);
  if (st) return st;
  st = check_items(items, count, (hipStream_t)stream);
  if (st) return st;
  return batch_launch_staged(b, n, (hipStream_t)stream, false);
}

ntt_status ntt_batch_run_graph(ntt_batch* b, const ntt_batch_item* items, size_t count, ntt_stream_t stream) {
  if (!b || (!items && count)) return NTT_EINVAL_POINTER;
  if (count > b->capacity) return NTT_EINVAL_COUNT;
  if (count == 0) return NTT_OK;
  size_t n = 0;
  ntt_status st = batch_prepare(b, items, count, &n);
  if (st) return st;
  st = check_items(items, count, (hipStream_t)stream);
  if (st) return st;
  return batch_launch_staged(b, n, (hipStream_t)stream, true);
}

ntt_status ntt_batch_autotune(ntt_batch* b, const ntt_batch_item* items, size_t count, ntt_stream_t stream,
                              int* chosen) {
  if (!b || !items) return NTT_EINVAL_POINTER;
  if (count == 0 || count > b->capacity) return NTT_EINVAL_COUNT;
  for (size_t i = 0; i < count; ++i)
    if (items[i].out == items[i].in) return NTT_EALIAS;   // every trial must see the same inputs
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int cand[3] = {cus, (3 * cus) / 2, 2 * cus};
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return NTT_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return NTT_EDEVICE; }
  const int saved = b->grid, saved_shape = b->shape;
  int best = saved, best_shape = saved_shape;
  float best_ms = 1e30f;
  ntt_status st = NTT_OK;
  for (int c = 0; c < 9 && st == NTT_OK; ++c) {
    b->grid = cand[c % 3];
    b->shape = c / 3;
    st = ntt_batch_run(b, items, count, stream);                 // warm-up
    if (st) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = NTT_EDEVICE; break; }
    for (int r = 0; r < 3 && st == NTT_OK; ++r) st = ntt_batch_run(b, items, count, stream);
    if (st) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = NTT_EDEVICE; break; }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) { best_ms = ms; best = cand[c % 3]; best_shape = c / 3; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->grid = saved;
  b->shape = saved_shape;
  if (st) return st;
  st = ntt_batch_set_grid(b, best);
  if (!st) st = ntt_batch_set_shape(b, best_shape);
  if (chosen) *chosen = best;
  return st;
}


// One-shot batch calls: a library-owned context per (host thread, device),
// grown to the largest task count seen, run through its captured graph.
ntt_status ntt_batch_forward(const ntt_batch_item* items, size_t count, ntt_stream_t stream) {
  return nttamd::oneshot_run(items, count, stream, NTT_BATCH_FWD_LAZY, NTT_BATCH_FWD);
}
ntt_status ntt_batch_inverse(const ntt_batch_item* items, size_t count, ntt_stream_t stream) {
  return nttamd::oneshot_run(items, count, stream, NTT_BATCH_INV_LAZY, NTT_BATCH_INV);
}
ntt_status ntt_batch_product(const ntt_batch_item* items, size_t count, ntt_stream_t stream) {
  return nttamd::oneshot_run(items, count, stream, NTT_BATCH_PRODUCT, NTT_BATCH_PRODUCT);
}

}  // extern "C"
