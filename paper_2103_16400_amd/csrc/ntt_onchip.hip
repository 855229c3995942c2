// Single-pass negacyclic NTT for N <= 2^14: one workgroup transforms one limb
// entirely on chip (HBM is read once and written once per coefficient).
//
// Same arithmetic as the multi-pass kernels (Algorithm 2 + Algorithm 4
// forward, Algorithm 3 + Algorithm 5 inverse with N^{-1} fused into the last
// stage); only the schedule differs.  Each thread keeps R = 2^LOGR
// coefficients in registers and runs up to LOGR stages per round; rounds
// exchange coefficients through LDS.  For N >= 2^13 the exchange goes through
// the LDS buffer in two halves (low then high 32-bit words), so two
// workgroups fit on a CU and one's memory and LDS phases overlap the other's
// arithmetic.
//
// Memory-system details that matter on gfx950:
//  * twiddles are loaded in blocks of at most 4 pairs, one block ahead of the
//    butterflies that use them, so their latency hides behind arithmetic
//    without holding a whole stage's twiddles in registers;
//  * in the round where each thread owns 2^LOGR consecutive coefficients, the
//    twiddle sub-tables are read from a transposed copy (lane-contiguous), and
//    coefficients enter or leave HBM through LDS so every access instruction
//    covers contiguous memory;
//  * coefficient loads are non-temporal: they stream through L2 without
//    evicting the (reused) twiddle tables.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"
#include "ntt_onchip.h"

namespace nttamd {

// MINW: waves per SIMD the register allocation must allow (occupancy target).
template <bool FWD, int LOGN, int LOGR, bool SPLIT, int MINW, int MODE, bool WIDE>
__global__ void __launch_bounds__(1 << (LOGN - LOGR), MINW) ntt_onchip_kernel(const PassArgs a) {
  using K = OnChip<FWD, LOGN, LOGR, SPLIT, true, WIDE>;
  __shared__ typename K::W lds[K::LDSW];
  const u32 item = a.item0 + blockIdx.x;
  const PlanView pv = load_plan(a.plan[item % a.num_limbs], FWD, (u64)K::N);
  const u64 base = (u64)item << LOGN;
  onchip_body<FWD, LOGN, LOGR, SPLIT, MODE, true, WIDE>(pv, a.in + base, a.out + base, a.mul ? a.mul + base : nullptr, lds, true,
                                                     threadIdx.x, true);
}

// Fused negacyclic product per limb: in = b, mul = NTT(a) (lazy), out =
// result (MODE canonical) or accumulator (MODE accumulate; may equal mul).
template <int LOGN, int LOGR, bool SPLIT, int MINW, int MODE, bool WIDE>
__global__ void __launch_bounds__(1 << (LOGN - LOGR), MINW) ntt_onchip_product_kernel(const PassArgs a) {
  using K = OnChip<true, LOGN, LOGR, SPLIT, true, WIDE>;
  __shared__ typename K::W lds[K::LDSW];
  const u32 item = a.item0 + blockIdx.x;
  const u64* plan = a.plan[item % a.num_limbs];
  const PlanView pf = load_plan(plan, true, (u64)K::N);
  const PlanView pi = load_plan(plan, false, (u64)K::N);
  const u64 base = (u64)item << LOGN;
  onchip_product_body<LOGN, LOGR, SPLIT, MODE, true, WIDE>(pf, pi, a.in + base, a.mul + base, a.out + base, lds, true,
                                                      threadIdx.x, true);
}

typedef void (*OnchipKernel)(const PassArgs);

// Variant 1 (N = 2^10 .. 2^14): half the coefficients per thread of variant 0,
// so twice the threads per limb: more waves hide latency when few limbs are in
// flight, at the price of one more LDS round and the natural twiddle table in
// every round (the transposed sub-tables are laid out for variant 0's shape).
template <bool FWD, int MODE, bool WIDE>
static OnchipKernel pick_onchip_mode_v1(int logN) {
  switch (logN) {
    case 10: return ntt_onchip_kernel<FWD, 10, 3, false, 8, MODE, WIDE>;
    case 11: return ntt_onchip_kernel<FWD, 11, 3, false, 8, MODE, WIDE>;
    case 12: return ntt_onchip_kernel<FWD, 12, 3, false, 8, MODE, WIDE>;
    case 13: return ntt_onchip_kernel<FWD, 13, 4, true, 4, MODE, WIDE>;
    case 14: return ntt_onchip_kernel<FWD, 14, 4, true, 4, MODE, WIDE>;
    default: return nullptr;
  }
}
static int onchip_logr_variant(int logN, int variant) { return onchip_logr(logN) - (variant == 1 ? 1 : 0); }

template <bool FWD, int MODE, bool WIDE>
static OnchipKernel pick_onchip_mode(int logN, int variant) {
  if (variant == 1) return pick_onchip_mode_v1<FWD, MODE, WIDE>(logN);
  if (variant != 0) return nullptr;
  switch (logN) {
    case 1: return ntt_onchip_kernel<FWD, 1, onchip_logr(1), false, 1, MODE, WIDE>;
    case 2: return ntt_onchip_kernel<FWD, 2, onchip_logr(2), false, 1, MODE, WIDE>;
    case 3: return ntt_onchip_kernel<FWD, 3, onchip_logr(3), false, 1, MODE, WIDE>;
    case 4: return ntt_onchip_kernel<FWD, 4, onchip_logr(4), false, 1, MODE, WIDE>;
    case 5: return ntt_onchip_kernel<FWD, 5, onchip_logr(5), false, 1, MODE, WIDE>;
    case 6: return ntt_onchip_kernel<FWD, 6, onchip_logr(6), false, 1, MODE, WIDE>;
    case 7: return ntt_onchip_kernel<FWD, 7, onchip_logr(7), false, 1, MODE, WIDE>;
    case 8: return ntt_onchip_kernel<FWD, 8, onchip_logr(8), false, 1, MODE, WIDE>;
    case 9: return ntt_onchip_kernel<FWD, 9, onchip_logr(9), false, 2, MODE, WIDE>;
    case 10: return ntt_onchip_kernel<FWD, 10, onchip_logr(10), false, 2, MODE, WIDE>;
    case 11: return ntt_onchip_kernel<FWD, 11, onchip_logr(11), false, 2, MODE, WIDE>;
    case 12: return ntt_onchip_kernel<FWD, 12, onchip_logr(12), false, 4, MODE, WIDE>;
    case 13: return ntt_onchip_kernel<FWD, 13, onchip_logr(13), true, 4, MODE, WIDE>;
    case 14: return ntt_onchip_kernel<FWD, 14, onchip_logr(14), true, 4, MODE, WIDE>;
    default: return nullptr;
  }
}

template <bool WIDE>
static OnchipKernel pick_onchip_w(bool fwd, int logN, u32 flags, int v) {
  if (fwd) {
    if (flags & kFlagMul) return pick_onchip_mode<true, kOutMul, WIDE>(logN, v);
    if (flags & kFlagCanon) return pick_onchip_mode<true, kOutCanon, WIDE>(logN, v);
    return pick_onchip_mode<true, kOutLazy, WIDE>(logN, v);
  }
  if (flags & kFlagAcc) return pick_onchip_mode<false, kOutAcc, WIDE>(logN, v);
  if (flags & kFlagCanon) return pick_onchip_mode<false, kOutCanon, WIDE>(logN, v);
  return pick_onchip_mode<false, kOutLazy, WIDE>(logN, v);
}

static OnchipKernel pick_onchip(bool fwd, int logN, u32 flags, bool wide, int v) {
  return wide ? pick_onchip_w<true>(fwd, logN, flags, v) : pick_onchip_w<false>(fwd, logN, flags, v);
}

template <int MODE, bool WIDE>
static OnchipKernel pick_product(int logN) {
  switch (logN) {
    case 1: return ntt_onchip_product_kernel<1, onchip_logr(1), false, 1, MODE, WIDE>;
    case 2: return ntt_onchip_product_kernel<2, onchip_logr(2), false, 1, MODE, WIDE>;
    case 3: return ntt_onchip_product_kernel<3, onchip_logr(3), false, 1, MODE, WIDE>;
    case 4: return ntt_onchip_product_kernel<4, onchip_logr(4), false, 1, MODE, WIDE>;
    case 5: return ntt_onchip_product_kernel<5, onchip_logr(5), false, 1, MODE, WIDE>;
    case 6: return ntt_onchip_product_kernel<6, onchip_logr(6), false, 1, MODE, WIDE>;
    case 7: return ntt_onchip_product_kernel<7, onchip_logr(7), false, 1, MODE, WIDE>;
    case 8: return ntt_onchip_product_kernel<8, onchip_logr(8), false, 1, MODE, WIDE>;
    case 9: return ntt_onchip_product_kernel<9, onchip_logr(9), false, 2, MODE, WIDE>;
    case 10: return ntt_onchip_product_kernel<10, onchip_logr(10), false, 2, MODE, WIDE>;
    case 11: return ntt_onchip_product_kernel<11, onchip_logr(11), false, 2, MODE, WIDE>;
    case 12: return ntt_onchip_product_kernel<12, onchip_logr(12), false, 4, MODE, WIDE>;
    case 13: return ntt_onchip_product_kernel<13, onchip_logr(13), true, 4, MODE, WIDE>;
    case 14: return ntt_onchip_product_kernel<14, onchip_logr(14), true, 4, MODE, WIDE>;
    default: return nullptr;
  }
}

ntt_status launch_onchip_product(const PassArgs& base_args, uint64_t items, bool acc, bool wide, hipStream_t stream) {
  const int logN = (int)base_args.logN;
  OnchipKernel k = wide ? (acc ? pick_product<kOutAcc, true>(logN) : pick_product<kOutCanon, true>(logN))
                        : (acc ? pick_product<kOutAcc, false>(logN) : pick_product<kOutCanon, false>(logN));
  if (!k) return NTT_EINVAL_DEGREE;
  PassArgs a = base_args;
  const uint64_t kMaxX = 1u << 30;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxX) {
    const uint64_t nx = (items - it0) < kMaxX ? (items - it0) : kMaxX;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(k, dim3((unsigned)nx), dim3(1 << (logN - onchip_logr(logN))), 0, stream, a);
  }
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

ntt_status launch_onchip(const PassArgs& base_args, uint64_t items, bool fwd, bool wide, hipStream_t stream,
                         int variant) {
  const int logN = (int)base_args.logN;
  OnchipKernel k = pick_onchip(fwd, logN, base_args.flags, wide, variant);
  if (!k) return NTT_EINVAL_DEGREE;
  PassArgs a = base_args;
  const uint64_t kMaxX = 1u << 30;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxX) {
    const uint64_t nx = (items - it0) < kMaxX ? (items - it0) : kMaxX;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(k, dim3((unsigned)nx), dim3(1 << (logN - onchip_logr_variant(logN, variant))), 0, stream, a);
  }
  return NTT_OK;
}

}  // namespace nttamd
