// Pieces shared by the NTT kernels: launch arguments, the per-limb plan view,
// the compile-time round geometry and the output step of the last pass.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "internal.h"
#include "modarith.h"

namespace nttamd {

constexpr int kMaxPlansPerLaunch = NTT_MAX_LIMBS;

enum : u32 { kFlagLast = 1u, kFlagCanon = 2u, kFlagMul = 4u, kFlagAcc = 8u };

struct PassArgs {
  u64* out;
  const u64* in;
  const u64* mul;                          // kFlagMul: multiplier; kFlagAcc: accumulator (== out); same layout as out
  const u64* plan[kMaxPlansPerLaunch];     // device plan buffers; item y uses plan[y % num_limbs]
  u32 num_limbs;
  u32 logN;
  u32 b0;                                  // lowest index bit of this pass
  u32 flags;
  u32 item0;                               // first item of this launch
};

// ---- round geometry (compile time) ----------------------------------------
template <bool FWD, int LOGT, int LOGR>
struct Geo {
  static constexpr int NR = (LOGT + LOGR - 1) / LOGR;
  // lowest row bit owned by a thread in round r
  static constexpr int lo(int r) {
    return FWD ? ((LOGT - (r + 1) * LOGR) > 0 ? (LOGT - (r + 1) * LOGR) : 0)
               : ((r * LOGR) < (LOGT - LOGR) ? (r * LOGR) : (LOGT - LOGR));
  }
  // first stage bit processed in round r and number of stages
  static constexpr int first_bit(int r) { return FWD ? (LOGT - 1 - r * LOGR) : (r * LOGR); }
  static constexpr int nst(int r) {
    return FWD ? ((LOGT - r * LOGR) < LOGR ? (LOGT - r * LOGR) : LOGR)
               : ((LOGT - r * LOGR) < LOGR ? (LOGT - r * LOGR) : LOGR);
  }
};

struct PlanView {
  u64 q, q2, nq, nq2;       // nq = 2^64 - q, nq2 = 2^64 - 2q
  u64 ninv, ninv_p, wn, wn_p;
  u64 bk;
  u64 q3, q4, nq4, rq;      // wide-range constants: 3q, 4q, 2^64 - 4q, floor(2^64 / q)
  u32 qbits;
  const ulonglong2* tw;     // natural table of this direction
  const ulonglong2* twp;    // transposed copy for the single-pass kernel (N <= 2^14)
};

__device__ __forceinline__ PlanView load_plan(const u64* plan, bool fwd, u64 N) {
  const PlanHeader* h = reinterpret_cast<const PlanHeader*>(plan);
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
  v.rq = h->barrett_k >> (v.qbits - 1);     // floor(2^(63+Q) / q) / 2^(Q-1) = floor(2^64 / q)
  v.tw = reinterpret_cast<const ulonglong2*>(plan + kPlanHeaderWords) + (fwd ? 0 : N);
  v.twp = v.tw + 2 * N;
  return v;
}

// Output step of the last pass: final correction, or the fused element-wise
// product with the multiplier operand (forward transform of a product).
// Output modes of the last pass, as template arguments of the kernels.
enum OutMode : int { kOutLazy = 0, kOutCanon = 1, kOutMul = 2, kOutAcc = 3 };

template <bool FWD, int MODE>
__device__ __forceinline__ u64 finish_mode(u64 v, u64 idx, const PassArgs& a, const PlanView& pv) {
  if (FWD && MODE == kOutMul) return barrett_mulmod<4>(v, a.mul[idx], pv.q, pv.q2, pv.bk, pv.qbits);
  if (!FWD && MODE == kOutAcc) return csub(a.mul[idx] + csub(v, pv.q), pv.q);   // acc + InvNTT, acc < q
  if (MODE == kOutCanon) return FWD ? reduce4(v, pv.q, pv.q2) : csub(v, pv.q);
  return v;
}

// Same output step with the multiplier / accumulator given per item (mul
// points at the item's first coefficient, i is the index inside the item).
template <bool FWD, int MODE>
__device__ __forceinline__ u64 finish_item(u64 v, const u64* mul, u64 i, const PlanView& pv) {
  if (FWD && MODE == kOutMul) return barrett_mulmod<4>(v, mul[i], pv.q, pv.q2, pv.bk, pv.qbits);
  if (!FWD && MODE == kOutAcc) return csub(mul[i] + csub(v, pv.q), pv.q);
  if (MODE == kOutCanon) return FWD ? reduce4(v, pv.q, pv.q2) : csub(v, pv.q);
  return v;
}

// Compiler-level fence: keeps the scheduler from hoisting the next stage's
// twiddle loads above the current stage (which would blow up register use).
__device__ __forceinline__ void stage_fence() { __asm__ volatile("" ::: "memory"); }

template <bool FWD>
__device__ __forceinline__ u64 finish(u64 v, u64 idx, const PassArgs& a, const PlanView& pv) {
  if (!(a.flags & kFlagLast)) return v;
  if (FWD) {
    if (a.flags & kFlagMul) return barrett_mulmod<4>(v, a.mul[idx], pv.q, pv.q2, pv.bk, pv.qbits);
    if (a.flags & kFlagCanon) return reduce4(v, pv.q, pv.q2);
    return v;
  }
  if (a.flags & kFlagAcc) return csub(a.mul[idx] + csub(v, pv.q), pv.q);
  return (a.flags & kFlagCanon) ? csub(v, pv.q) : v;
}

// wide: use the wide-range butterflies; valid when every modulus of the launch
// is below kWideModulusBound.
// variant 0: 2^onchip_logr(logN) coefficients per thread; 1 (N = 2^10 .. 2^14): half as many
ntt_status launch_onchip(const PassArgs& base_args, uint64_t items, bool fwd, bool wide, hipStream_t stream,
                         int variant);
// Fused product per limb for N <= 2^14: in = b, mul = NTT(a) lazy, out =
// canonical product (acc false) or accumulator += product (acc true).
ntt_status launch_onchip_product(const PassArgs& base_args, uint64_t items, bool acc, bool wide,
                                 hipStream_t stream);

}  // namespace nttamd
