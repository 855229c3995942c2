// Persistent batch kernel: one launch runs a list of limb tasks of mixed ring
// degree (2^10 .. 2^17), moduli and operation.
//
// RNS polynomials of different sizes and limb counts (Section 5) decompose
// into independent limb tasks.  Each workgroup of the persistent grid claims
// the next task from a device-side counter (tasks are ordered largest first)
// and runs it to completion by itself, so tasks never wait on each other:
//   * N <= 2^14: the single-pass transform held on chip (ntt_onchip.h), with
//     2^(logN-9) coefficients per thread so every size uses 512 threads;
//   * N >= 2^15: both passes of the two-pass transform (ntt_tile.h), one
//     4096-coefficient tile at a time; the intermediate stays in the limb's
//     output buffer and the workgroup barrier orders the passes.
// Operations: forward (lazy [0, 4q) or canonical), inverse (lazy [0, 2q) or
// canonical) and the negacyclic product out = a * b of the Section 4 listing
// (forward(a), forward(b) fused with the multiply, inverse).  The task list
// and its length live in device memory, so a captured graph of
// [descriptor copy, counter reset, kernel] can be replayed for any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  unsigned char* host;             // pinned staging: count word (128-byte line), then the tasks
  unsigned char* dev;              // device: claim counter (own line), count word, tasks
  hipEvent_t done;                 // completion of the last run from this set
  bool pending;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  hipGraphNode_t copy_node;        // the graph's descriptor copy, resized before each replay
};
struct ntt_batch {
  int device;
  size_t capacity;                 // tasks
  int grid;                        // persistent workgroups (0: automatic)
  int cur;                         // staging set of the next run
  ntt_batch_stage stage[2];
};

namespace nttamd {

// Staging layout: [0, 128) count word; tasks from byte 128.  The device copy
// keeps the claim counter in its own line in front: counter at 0, staging
// mirrored from byte 128.
constexpr size_t kStageHead = 128;
constexpr size_t kDevHead = 128;
static ntt_batch_stage& cur_stage(ntt_batch* b) { return b->stage[b->cur]; }
static BatchTask* staged_tasks(ntt_batch* b) { return reinterpret_cast<BatchTask*>(cur_stage(b).host + kStageHead); }
static size_t stage_bytes(size_t count) { return kStageHead + count * sizeof(BatchTask); }

constexpr int kBatchThreads = 512;
constexpr int kBatchLdsWords32 = (1 << 14) + (1 << 14) / 32;   // 2^14 split exchange, 66 KiB

// ---- one task -----------------------------------------------------------------

template <bool FWD, int LOGN, int MODE, bool WIDE>
__device__ __attribute__((noinline)) void task_onchip(const u64* plan, const u64* in, u64* out, const u64* mul, u32* lds,
                                            bool nt) {
  const PlanView pv = load_plan(plan, FWD, 1ull << LOGN);
  onchip_body<FWD, LOGN, LOGN - 9, true, MODE, true, WIDE>(pv, in, out, mul, lds, nt);
}

// Both passes of a two-pass transform by one workgroup (512 threads, tiles of
// 4096 coefficients, 8 per thread).
// `mid` receives the first pass (may equal out unless out holds the multiplier).
template <bool FWD, int LOGN, int MODE>
__device__ __attribute__((noinline)) void task_twopass(const u64* plan, const u64* in, u64* mid, u64* out, const u64* mul,
                                             u64* lds, bool nt) {
  constexpr int LT_LO = mp_logt_lo(LOGN);
  constexpr int LT_HI = LOGN - LT_LO;
  constexpr int LC_HI = 12 - LT_HI;           // columns per high-pass tile
  constexpr int LH_LO = 12 - LT_LO;           // blocks per low-pass tile
  constexpr int TILES = 1 << (LOGN - 12);
  const PlanView pv = load_plan(plan, FWD, 1ull << LOGN);
#pragma unroll 1
  for (int step = 0; step < 2; ++step) {
    const bool hi = FWD ? step == 0 : step == 1;
    const bool last = step == 1;
    const u64* src = step == 0 ? in : mid;
    u64* dst = step == 0 ? mid : out;
#pragma unroll 1
    for (u32 tile = 0; tile < (u32)TILES; ++tile) {
      if (hi) {
        if (last) tile_body<FWD, LT_HI, 3, LC_HI, 0, MODE, true, -1, true>(pv, LOGN, LT_LO, tile, src, dst, mul, lds, false);
        else tile_body<FWD, LT_HI, 3, LC_HI, 0, kOutLazy, false, -1, true>(pv, LOGN, LT_LO, tile, src, dst, mul, lds, nt);
      } else {
        if (last) tile_body<FWD, LT_LO, 3, 0, LH_LO, MODE, true, -1, true>(pv, LOGN, 0, tile, src, dst, mul, lds, false);
        else tile_body<FWD, LT_LO, 3, 0, LH_LO, kOutLazy, false, -1, true>(pv, LOGN, 0, tile, src, dst, mul, lds, nt);
      }
      __syncthreads();
    }
  }
}

// Second half of a product on chip: out = InvNTT(NTT(b) (.) out), canonical.
template <int LOGN, bool WIDE>
__device__ __attribute__((noinline)) void task_product_onchip(const u64* plan, const u64* b, u64* out, u32* lds) {
  const PlanView pf = load_plan(plan, true, 1ull << LOGN);
  const PlanView pi = load_plan(plan, false, 1ull << LOGN);
  onchip_product_body<LOGN, LOGN - 9, true, kOutCanon, true, WIDE>(pf, pi, b, out, out, lds, true);
}

template <bool WIDE>
__device__ __forceinline__ void run_product_onchip(u32 logN, const u64* plan, const u64* b, u64* out, void* lds) {
  u32* l32 = reinterpret_cast<u32*>(lds);
  switch (logN) {
    case 10: task_product_onchip<10, WIDE>(plan, b, out, l32); break;
    case 11: task_product_onchip<11, WIDE>(plan, b, out, l32); break;
    case 12: task_product_onchip<12, WIDE>(plan, b, out, l32); break;
    case 13: task_product_onchip<13, WIDE>(plan, b, out, l32); break;
    case 14: task_product_onchip<14, WIDE>(plan, b, out, l32); break;
    default: break;
  }
}

// WIDE applies to the single-pass sizes only; two-pass tasks run the paper's butterflies.
template <bool FWD, int MODE, bool WIDE>
__device__ __forceinline__ void run_transform(u32 logN, const u64* plan, const u64* in, u64* mid, u64* out,
                                              const u64* mul, void* lds, bool nt) {
  u32* l32 = reinterpret_cast<u32*>(lds);
  u64* l64 = reinterpret_cast<u64*>(lds);
  switch (logN) {
    case 10: task_onchip<FWD, 10, MODE, WIDE>(plan, in, out, mul, l32, nt); break;
    case 11: task_onchip<FWD, 11, MODE, WIDE>(plan, in, out, mul, l32, nt); break;
    case 12: task_onchip<FWD, 12, MODE, WIDE>(plan, in, out, mul, l32, nt); break;
    case 13: task_onchip<FWD, 13, MODE, WIDE>(plan, in, out, mul, l32, nt); break;
    case 14: task_onchip<FWD, 14, MODE, WIDE>(plan, in, out, mul, l32, nt); break;
    case 15: task_twopass<FWD, 15, MODE>(plan, in, mid, out, mul, l64, nt); break;
    case 16: task_twopass<FWD, 16, MODE>(plan, in, mid, out, mul, l64, nt); break;
    case 17: task_twopass<FWD, 17, MODE>(plan, in, mid, out, mul, l64, nt); break;
    default: break;
  }
}

template <bool WIDE>
__device__ __forceinline__ void run_task(const BatchTask& tk, void* lds) {
  switch (tk.op & kBatchOpMask) {
    case kBatchFwdLazy: run_transform<true, kOutLazy, WIDE>(tk.logN, tk.plan, tk.in, tk.out, tk.out, nullptr, lds, true); break;
    case kBatchFwdCanon: run_transform<true, kOutCanon, WIDE>(tk.logN, tk.plan, tk.in, tk.out, tk.out, nullptr, lds, true); break;
    case kBatchInvLazy: run_transform<false, kOutLazy, WIDE>(tk.logN, tk.plan, tk.in, tk.out, tk.out, nullptr, lds, true); break;
    case kBatchInvCanon: run_transform<false, kOutCanon, WIDE>(tk.logN, tk.plan, tk.in, tk.out, tk.out, nullptr, lds, true); break;
    case kBatchProduct:
      // out <- NTT(a) lazy; out <- NTT(b) (.) out (first pass of NTT(b) in tmp); out <- InvNTT(out)
      run_transform<true, kOutLazy, WIDE>(tk.logN, tk.plan, tk.in, tk.out, tk.out, nullptr, lds, true);
      __syncthreads();
      if (tk.logN <= (u32)kMaxOnchipLog) {        // the rest on chip, in one step
        run_product_onchip<WIDE>(tk.logN, tk.plan, tk.in2, tk.out, lds);
        break;
      }
      run_transform<true, kOutMul, false>(tk.logN, tk.plan, tk.in2, tk.tmp, tk.out, tk.out, lds, true);
      __syncthreads();
      run_transform<false, kOutCanon, false>(tk.logN, tk.plan, tk.out, tk.out, tk.out, nullptr, lds, false);
      break;
    default: break;
  }
}

__global__ void batch_reset_kernel(u32* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void __launch_bounds__(kBatchThreads, 4)
    ntt_batch_kernel(const BatchTask* __restrict__ tasks, const u32* __restrict__ count, u32* counter) {
  __shared__ u32 lds[kBatchLdsWords32];
  __shared__ u32 claimed;
  const u32 n = *count;
#pragma unroll 1
  for (;;) {
    if (threadIdx.x == 0) claimed = atomicAdd(counter, 1u);
    __syncthreads();
    const u32 i = claimed;
    __syncthreads();
    if (i >= n) break;                          // every wave of every workgroup reaches this exit
    const BatchTask tk = tasks[i];
    if (tk.op & kBatchWide) run_task<true>(tk, lds);
    else run_task<false>(tk, lds);
    __syncthreads();
  }
}

// ---- host side ----------------------------------------------------------------

static uint64_t task_cost(uint32_t logN, uint32_t op) {
  const uint64_t n = 1ull << logN;
  return n * logN * ((op & kBatchOpMask) == kBatchProduct ? 3 : 1);
}

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

ntt_status batch_prepare(ntt_batch* b, const ntt_batch_item* items, size_t count, size_t* out_count) {
  ntt_status st0 = wait_staging(b);
  if (st0) return st0;
  std::vector<std::pair<uint64_t, size_t>> order(count);
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
    order[i] = {task_cost((uint32_t)logN, it.op), i};
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<uint64_t, size_t>& a, const std::pair<uint64_t, size_t>& c) {
                     return a.first > c.first;
                   });
  std::map<std::pair<uint64_t, uint64_t>, const ntt_plan*> seen;   // one cache lookup per distinct (N, q)
  for (size_t k = 0; k < count; ++k) {
    const ntt_batch_item& it = items[order[k].second];
    const ntt_plan*& p = seen[{it.N, it.q}];
    if (!p) {
      ntt_status st = cached_plan(it.N, it.q, &p);
      if (st) return st;
    }
    BatchTask& t = staged_tasks(b)[k];
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
  *reinterpret_cast<uint32_t*>(cur_stage(b).host) = (uint32_t)count;
  *out_count = count;
  return NTT_OK;
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

// Enqueues [descriptor copy of `staged` tasks, counter reset, persistent kernel] on `stream`.
ntt_status batch_enqueue(ntt_batch* b, size_t staged, int grid, hipStream_t stream) {
  ntt_batch_stage& g = cur_stage(b);
  if (hipMemcpyAsync(g.dev + kDevHead, g.host, stage_bytes(staged), hipMemcpyHostToDevice, stream) != hipSuccess)
    return NTT_EDEVICE;
  u32* counter = reinterpret_cast<u32*>(g.dev);
  const u32* count = reinterpret_cast<const u32*>(g.dev + kDevHead);
  const BatchTask* tasks = reinterpret_cast<const BatchTask*>(g.dev + kDevHead + kStageHead);
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
  hipLaunchKernelGGL(ntt_batch_kernel, dim3(grid), dim3(kBatchThreads), 0, stream, tasks, count, counter);
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

static ntt_status batch_launch_staged(ntt_batch* b, size_t n, hipStream_t s, bool graph) {
  ntt_status st = NTT_OK;
  ntt_batch_stage& sg = cur_stage(b);
  if (!graph) {
    st = batch_enqueue(b, n, batch_grid(b, n), s);
    if (st) return st;
  } else {
    if (!sg.graph_exec) {
      // captured once per staging set with the full-capacity copy and grid; the kernel reads the count from device memory
      const int grid = batch_grid(b, b->capacity);
      hipStream_t cap = nullptr;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return NTT_EDEVICE;
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return NTT_EDEVICE;
      }
      st = batch_enqueue(b, b->capacity, grid, cap);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cap, &g);
      (void)hipStreamDestroy(cap);
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess || !g) return NTT_EDEVICE;
      if (hipGraphInstantiate(&sg.graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return NTT_EDEVICE;
      }
      sg.graph = g;
      // find the descriptor copy, so each replay copies only its own batch's descriptors
      size_t nn = 0;
      sg.copy_node = nullptr;
      if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess && nn > 0) {
        std::vector<hipGraphNode_t> nodes(nn);
        if (hipGraphGetNodes(g, nodes.data(), &nn) == hipSuccess) {
          for (size_t i = 0; i < nn; ++i) {
            hipGraphNodeType ty;
            if (hipGraphNodeGetType(nodes[i], &ty) == hipSuccess && ty == hipGraphNodeTypeMemcpy) sg.copy_node = nodes[i];
          }
        }
      }
    }
    if (sg.copy_node && hipGraphExecMemcpyNodeSetParams1D(sg.graph_exec, sg.copy_node, sg.dev + kDevHead, sg.host,
                                                          stage_bytes(n), hipMemcpyHostToDevice) != hipSuccess)
      sg.copy_node = nullptr;                      // keep the captured full-capacity copy from here on
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
  std::vector<std::pair<uint64_t, size_t>> order(count);
  for (size_t i = 0; i < count; ++i) order[i] = {task_cost(tasks[i].logN, tasks[i].op), i};
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<uint64_t, size_t>& a, const std::pair<uint64_t, size_t>& c) {
                     return a.first > c.first;
                   });
  BatchTask* dst = staged_tasks(b);
  for (size_t k = 0; k < count; ++k) dst[k] = tasks[order[k].second];
  *reinterpret_cast<uint32_t*>(cur_stage(b).host) = (uint32_t)count;
  return batch_launch_staged(b, count, stream, graph);
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
    if (!st && hipMalloc((void**)&g.dev, kDevHead + bytes) != hipSuccess) { g.dev = nullptr; st = NTT_ENOMEM; }
    if (!st && hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) { g.done = nullptr; st = NTT_EDEVICE; }
    if (st) {
      for (ntt_batch_stage& h : b->stage) release_stage(h);
      delete b;
      return st;
    }
  }
  *out = b;
  return NTT_OK;
}

ntt_status ntt_batch_destroy(ntt_batch* b) {
  if (!b) return NTT_EINVAL_POINTER;
  for (ntt_batch_stage& g : b->stage) release_stage(g);
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
  const int saved = b->grid;
  int best = saved;
  float best_ms = 1e30f;
  ntt_status st = NTT_OK;
  for (int c = 0; c < 3 && st == NTT_OK; ++c) {
    b->grid = cand[c];
    st = ntt_batch_run(b, items, count, stream);                 // warm-up
    if (st) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = NTT_EDEVICE; break; }
    for (int r = 0; r < 3 && st == NTT_OK; ++r) st = ntt_batch_run(b, items, count, stream);
    if (st) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = NTT_EDEVICE; break; }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) { best_ms = ms; best = cand[c]; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->grid = saved;
  if (st) return st;
  st = ntt_batch_set_grid(b, best);
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
