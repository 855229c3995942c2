// Word-size-2^32 arithmetic (moduli below 2^30): the plan view, the
// butterflies of Algorithms 4 and 5 at beta = 2^32, Algorithm 8 with input
// factor 4 and the output step; shared by the single-pass and two-pass
// kernels of ntt_small.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ntt_common.h"

namespace nttamd {

struct View32 {
  u32 q, q2, ninv, ninv_p, wn, wn_p, qbits;
  u64 bk;
  const ulonglong2* tw;
  const ulonglong2* twp;
};

__device__ __forceinline__ View32 view32(const u64* plan, bool fwd, u64 N) {
  const PlanView p = load_plan(plan, fwd, N);
  View32 v;
  v.q = (u32)p.q;
  v.q2 = (u32)p.q2;
  v.ninv = (u32)p.ninv;
  v.ninv_p = (u32)(p.ninv_p >> 32);
  v.wn = (u32)p.wn;
  v.wn_p = (u32)(p.wn_p >> 32);
  v.qbits = p.qbits;
  v.bk = p.bk;
  v.tw = p.tw;
  v.twp = p.twp;
  return v;
}

// Algorithm 4 at beta = 2^32 (inputs and outputs in [0, 4q)).  nt = -T mod 2^32
// with T = W X1 - Q q in [0, 2q), so X0 + T = a - nt and X0 + 2q - T = a + 2q + nt.
__device__ __forceinline__ void fwd_bfly32(u32& x0, u32& x1, u32 w, u32 wp, u32 q, u32 q2) {
  const u32 a = min(x0, x0 - q2);
  const u32 nt = __umulhi(wp, x1) * q - w * x1;
  x0 = a - nt;
  x1 = a + q2 + nt;
}

// Algorithm 5 at beta = 2^32 (inputs and outputs in [0, 2q)).
__device__ __forceinline__ void inv_bfly32(u32& x0, u32& x1, u32 w, u32 wp, u32 q, u32 q2) {
  const u32 s = x0 + x1;
  const u32 d = x0 + q2 - x1;
  x0 = min(s, s - q2);
  x1 = w * d - __umulhi(wp, d) * q;
}

// Last Gentleman-Sande stage fused with the scaling by N^{-1}:
// X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 - X1 + 2q), both in [0, 2q).
__device__ __forceinline__ void inv_last32(u32& x0, u32& x1, const View32& v) {
  const u32 s = x0 + x1;
  const u32 d = x0 + v.q2 - x1;
  x0 = v.ninv * s - __umulhi(v.ninv_p, s) * v.q;
  x1 = v.wn * d - __umulhi(v.wn_p, d) * v.q;
}

// Algorithm 8 with input factor 4: x, y in [0, 4q) are reduced to [0, q), then
// z = x y < q^2, c1 = z >> (Q - 1) < 2^(Q+1) <= 2^31, c3 = floor(c1 k / 2^64)
// with k = floor(2^(63+Q) / q), and z - c3 q < 3q takes two conditional
// subtractions.  c1 fits one word, so c1 k / 2^64 is one 32 x 32 high product
// and one 32 x 32 -> 64 multiply-add.
__device__ __forceinline__ u32 mulmod32_f4(u32 x, u32 y, const View32& v) {
  x = min(x, x - v.q2);
  x = min(x, x - v.q);
  y = min(y, y - v.q2);
  y = min(y, y - v.q);
  const u64 z = (u64)x * y;
  const u32 c1 = (u32)(z >> (v.qbits - 1));
  const u64 t = (u64)c1 * (u32)(v.bk >> 32) + __umulhi(c1, (u32)v.bk);
  const u32 c3 = (u32)(t >> 32);
  u32 r = (u32)z - c3 * v.q;
  r = min(r, r - v.q);
  return min(r, r - v.q);
}

// Output step of the last pass: lazy, canonical, the forward fused with the
// Algorithm 8 multiply by mul[i] (in [0, 4q)), or the inverse added into mul[i].
template <bool FWD, int MODE>
__device__ __forceinline__ u32 finish32(u32 x, const u32* mul, u32 i, const View32& v) {
  if (FWD && MODE == kOutMul) return mulmod32_f4(x, mul[i], v);
  if (MODE == kOutCanon) {
    if (FWD) x = min(x, x - v.q2);
    return min(x, x - v.q);
  }
  if (!FWD && MODE == kOutAcc) {
    const u32 r = mul[i] + min(x, x - v.q);     // acc < q plus a canonical value
    return min(r, r - v.q);
  }
  return x;
}

}  // namespace nttamd
