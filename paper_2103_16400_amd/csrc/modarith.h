// Device-side word arithmetic for gfx950: 64-bit modular products built from
// the 32-bit multipliers of the vector ALU (v_mul_hi_u32, v_mad_u64_u32).
// CDNA4 has no 64 x 64-bit integer multiply, so every 64-bit product here is
// assembled from 32 x 32 -> 64 partial products; all results are exact.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttamd {

typedef uint64_t u64;
typedef uint32_t u32;

__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }

// floor(a * b / 2^64), exact.  One v_mul_hi_u32 and three v_mad_u64_u32.
__device__ __forceinline__ u64 mulhi64(u64 a, u64 b) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  u64 t = (u64)a0 * b1 + (u64)__umulhi(a0, b0);   // < 2^64
  u64 s = (u64)a1 * b0 + (u64)lo32(t);            // < 2^64
  u64 r = (u64)a1 * b1 + (u64)hi32(t);            // < 2^64
  return r + (u64)hi32(s);
}

// Full 128-bit product a * b as (hi, lo).
__device__ __forceinline__ void mul128(u64 a, u64 b, u64& hi, u64& lo) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  u64 p00 = (u64)a0 * b0;
  u64 t = (u64)a0 * b1 + (u64)hi32(p00);
  u64 s = (u64)a1 * b0 + (u64)lo32(t);
  hi = (u64)a1 * b1 + (u64)hi32(t) + (u64)hi32(s);
  lo = ((u64)lo32(s) << 32) | lo32(p00);
}

// (w * x + Q * nq) mod 2^64 with nq = 2^64 - q, i.e. (w * x - Q * q) mod 2^64:
// the remainder step T of the Harvey butterflies (Algorithms 4 and 5).  The
// negated modulus turns the subtraction into a multiply-add, as the paper's
// AVX512 butterflies (Algorithms 6 and 7) do.
__device__ __forceinline__ u64 mul_sub_lo(u64 w, u64 x, u64 Q, u64 nq) {
  const u32 w0 = lo32(w), w1 = hi32(w), x0 = lo32(x), x1 = hi32(x);
  const u32 q0 = lo32(Q), q1 = hi32(Q), n0 = lo32(nq), n1 = hi32(nq);
  u64 r = (u64)w0 * x0;
  r = (u64)q0 * n0 + r;                             // wraps mod 2^64: only the low 64 bits matter
  u32 h = hi32(r) + w0 * x1 + w1 * x0 + q0 * n1 + q1 * n0;
  return ((u64)h << 32) | lo32(r);
}

// Shoup multiplication: w * x mod q up to one multiple of q, result in
// [0, 2q) for any x < 2^64, given wp = floor(w * 2^64 / q) and w < q.
__device__ __forceinline__ u64 shoup_mul(u64 x, u64 w, u64 wp, u64 nq) {
  return mul_sub_lo(w, x, mulhi64(wp, x), nq);
}

// x - m if x >= m, else x (one conditional subtraction).
__device__ __forceinline__ u64 csub(u64 x, u64 m) { return x >= m ? x - m : x; }

// Algorithm 4 (Harvey forward butterfly), beta = 2^64, inputs in [0, 4q),
// outputs in [0, 4q):  X0 <- X0 + W X1,  X1 <- X0 - W X1  (mod q).
__device__ __forceinline__ void harvey_fwd(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq) {
  const u64 a = csub(x0, q2);
  const u64 t = shoup_mul(x1, w, wp, nq);          // [0, 2q)
  x0 = a + t;
  x1 = a + q2 - t;
}

// Algorithm 5 (Harvey inverse butterfly), inputs in [0, 2q), outputs in
// [0, 2q):  X0 <- X0 + X1,  X1 <- W (X0 - X1)  (mod q).
__device__ __forceinline__ void harvey_inv(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq) {
  const u64 y0 = csub(x0 + x1, q2);
  const u64 t = x0 + q2 - x1;
  x1 = shoup_mul(t, w, wp, nq);
  x0 = y0;
}

// Last inverse stage fused with the scaling by N^{-1} (Algorithm 3's final
// loop): X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 - X1), both in [0, 2q).
__device__ __forceinline__ void harvey_inv_last(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp,
                                                u64 q2, u64 nq) {
  const u64 s = x0 + x1;                           // < 4q < 2^64
  const u64 t = x0 + q2 - x1;                      // < 4q
  x0 = shoup_mul(s, ni, nip, nq);
  x1 = shoup_mul(t, wn, wnp, nq);
}

// x mod q for x in [0, 4q): the two-step small_mod of Section 4.
__device__ __forceinline__ u64 reduce4(u64 x, u64 q, u64 q2) { return csub(csub(x, q2), q); }

// Algorithm 8 semantics: x * y mod q for x, y in [0, f q) with f in {1, 2, 4}.
// Inputs are first reduced to [0, q); then Barrett reduction with
// Q = floor(log2 q) + 1, L = 63 + Q, k = floor(2^L / q):
//   c1 = (x y) >> (Q - 1);  c3 = floor(c1 k / 2^64);  c4 = x y - c3 q.
// The quotient estimate c3 can be short by up to 2, so c4 < 3q and two
// conditional subtractions give the canonical value.
template <int F>
__device__ __forceinline__ u64 barrett_mulmod(u64 x, u64 y, u64 q, u64 q2, u64 k, u32 qbits) {
  if (F >= 4) { x = csub(x, q2); y = csub(y, q2); }
  if (F >= 2) { x = csub(x, q); y = csub(y, q); }
  u64 hi, lo;
  mul128(x, y, hi, lo);
  const u32 s = qbits - 1;                          // 1 <= s <= 61
  const u64 c1 = (lo >> s) | (hi << (64 - s));
  const u64 c3 = mulhi64(c1, k);
  u64 c4 = lo - c3 * q;
  c4 = csub(c4, q);
  return csub(c4, q);
}

}  // namespace nttamd
