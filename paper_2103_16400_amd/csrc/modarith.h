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

// ---- Shoup products on 32-bit lanes -----------------------------------------
// W X mod q for a constant W < q with companion W' = floor(W 2^64 / q): the
// quotient estimate Q ~ floor(W' X / 2^64), then the remainder word
// T = W X - Q q computed mod 2^64 as W X + Q (2^64 - q).
//
// Register safety: every operand, temporary and carry below is allocated by
// the compiler (no fixed registers, nothing written that the compiler does not
// know of), so the allocator, the spiller and callee-save handling see every
// register the arithmetic touches.  Two short assembly statements cover the
// steps the compiler schedules poorly; each carry or mask an instruction
// writes is read inside the same statement, at least two instructions later
// (gfx950 needs two wait states between a VALU write of an SGPR and a VALU
// read of it as carry or mask; the compiler's hazard recognizer does not look
// inside assembly).  Everything else is plain C++.
__device__ __forceinline__ u64 mad32(u32 a, u32 b, u64 c) { return (u64)a * b + c; }

// Middle of the quotient estimate and the low product of the remainder, for
// X = (xh, xl), W' = (ph, pl), W = (wh, wl):
//   m  = (pl xh + z + ph xl) mod 2^64,  cb = its bit 64,  t0 = wl xl,
// with z = floor(pl xl / 2^32) (exact quotient) or 0 (estimate).  The sum
// needs 65 bits; its carry leaves the statement as the 32-bit value cb.  The
// statement also forms f = fa + fb, an addition the caller needs anyway, so
// that two instructions separate the carry's write from its read.
// UNI: W and W' are uniform (SGPR operands); FBS: fb is uniform.
#define NTTAMD_SHOUP_FRONT                                   \
  "v_mad_u64_u32 %[m], %[j], %[pl], %[xh], %[z]\n\t"         \
  "v_mad_u64_u32 %[m], %[c], %[ph], %[xl], %[m]\n\t"         \
  "v_mad_u64_u32 %[t], %[j], %[wl], %[xl], 0\n\t"            \
  "v_lshl_add_u64 %[f], %[fa], 0, %[fb]\n\t"                 \
  "v_addc_co_u32 %[cb], %[j], 0, 0, %[c]"
#define NTTAMD_SHOUP_FRONT_OUT \
  [m] "=&v"(m), [t] "=&v"(t0), [cb] "=&v"(cb), [f] "=&v"(f), [c] "=&s"(c), [j] "=&s"(j)
template <bool UNI, bool FBS>
__device__ __forceinline__ void shoup_front(u32 xl, u32 xh, u32 pl, u32 ph, u32 wl, u64 z, u64 fa, u64 fb, u64& m,
                                            u32& cb, u64& t0, u64& f) {
  u64 c, j;
  if constexpr (UNI && FBS)
    asm(NTTAMD_SHOUP_FRONT : NTTAMD_SHOUP_FRONT_OUT
        : [xl] "v"(xl), [xh] "v"(xh), [pl] "s"(pl), [ph] "s"(ph), [wl] "s"(wl), [z] "v"(z), [fa] "v"(fa), [fb] "s"(fb));
  else if constexpr (UNI)
    asm(NTTAMD_SHOUP_FRONT : NTTAMD_SHOUP_FRONT_OUT
        : [xl] "v"(xl), [xh] "v"(xh), [pl] "s"(pl), [ph] "s"(ph), [wl] "s"(wl), [z] "v"(z), [fa] "v"(fa), [fb] "v"(fb));
  else if constexpr (FBS)
    asm(NTTAMD_SHOUP_FRONT : NTTAMD_SHOUP_FRONT_OUT
        : [xl] "v"(xl), [xh] "v"(xh), [pl] "v"(pl), [ph] "v"(ph), [wl] "v"(wl), [z] "v"(z), [fa] "v"(fa), [fb] "s"(fb));
  else
    asm(NTTAMD_SHOUP_FRONT : NTTAMD_SHOUP_FRONT_OUT
        : [xl] "v"(xl), [xh] "v"(xh), [pl] "v"(pl), [ph] "v"(ph), [wl] "v"(wl), [z] "v"(z), [fa] "v"(fa), [fb] "v"(fb));
}
#undef NTTAMD_SHOUP_FRONT
#undef NTTAMD_SHOUP_FRONT_OUT

// High word of the remainder: th + lo(Q) hi(nq) + hi(Q) lo(nq) + wl xh + wh xl
// (mod 2^32), the products that reach bit 32 and above of T.  Kept in one
// statement so that the sum stays a 32-bit chain that lands in T's high half.
template <bool UNI>
__device__ __forceinline__ u32 shoup_high(u32 th, u32 ql, u32 qh, u32 nql, u32 nqh, u32 wl, u32 wh, u32 xl,
                                          u32 xh) {
  u32 a, b;
  // th is updated in place, so the compiler can keep it in T's high register
  if constexpr (UNI) {
    asm("v_mul_lo_u32 %[a], %[ql], %[nqh]\n\t"
        "v_mul_lo_u32 %[b], %[qh], %[nql]\n\t"
        "v_add3_u32 %[r], %[r], %[a], %[b]\n\t"
        "v_mul_lo_u32 %[a], %[wl], %[xh]\n\t"
        "v_mul_lo_u32 %[b], %[wh], %[xl]\n\t"
        "v_add3_u32 %[r], %[r], %[a], %[b]"
        : [r] "+v"(th), [a] "=&v"(a), [b] "=&v"(b)
        : [ql] "v"(ql), [qh] "v"(qh), [nql] "s"(nql), [nqh] "s"(nqh), [wl] "s"(wl), [wh] "s"(wh), [xl] "v"(xl),
          [xh] "v"(xh));
  } else {
    asm("v_mul_lo_u32 %[a], %[ql], %[nqh]\n\t"
        "v_mul_lo_u32 %[b], %[qh], %[nql]\n\t"
        "v_add3_u32 %[r], %[r], %[a], %[b]\n\t"
        "v_mul_lo_u32 %[a], %[wl], %[xh]\n\t"
        "v_mul_lo_u32 %[b], %[wh], %[xl]\n\t"
        "v_add3_u32 %[r], %[r], %[a], %[b]"
        : [r] "+v"(th), [a] "=&v"(a), [b] "=&v"(b)
        : [ql] "v"(ql), [qh] "v"(qh), [nql] "s"(nql), [nqh] "s"(nqh), [wl] "v"(wl), [wh] "v"(wh), [xl] "v"(xl),
          [xh] "v"(xh));
  }
  return th;
}

// Shoup multiplication: w x mod q in [0, 2q) for any x < 2^64 with the exact
// quotient (EXACT), or in [0, 3q) with the estimate that drops the lowest
// partial product pl xl (its carry into bit 64 is at most 1, so the estimate
// is Q or Q - 1).  nq = 2^64 - q.  Also returns f = fa + fb (see shoup_front).
template <bool EXACT = true, bool UNI = false, bool FBS = true>
__device__ __forceinline__ u64 shoup_mul_f(u64 x, u64 w, u64 wp, u64 nq, u64 fa, u64 fb, u64& f) {
  const u32 xl = lo32(x), xh = hi32(x), pl = lo32(wp), ph = hi32(wp), wl = lo32(w), wh = hi32(w);
  const u64 z = EXACT ? (u64)__umulhi(pl, xl) : 0;
  u64 m, t0;
  u32 cb;
  shoup_front<UNI, FBS>(xl, xh, pl, ph, wl, z, fa, fb, m, cb, t0, f);
  const u64 Q = mad32(ph, xh, ((u64)cb << 32) | hi32(m));      // the quotient (estimate)
  const u64 t = mad32(lo32(Q), lo32(nq), t0);
  const u32 th = shoup_high<UNI>(hi32(t), lo32(Q), hi32(Q), lo32(nq), hi32(nq), wl, wh, xl, xh);
  return ((u64)th << 32) | lo32(t);
}
template <bool EXACT = true, bool UNI = false>
__device__ __forceinline__ u64 shoup_mul(u64 x, u64 w, u64 wp, u64 nq) {
  u64 f;
  return shoup_mul_f<EXACT, UNI, true>(x, w, wp, nq, x, nq, f);   // f unused
}

// x - m if x >= m, else x (one conditional subtraction); nm = 2^64 - m.
__device__ __forceinline__ u64 csub(u64 x, u64 m) { return x >= m ? x - m : x; }
__device__ __forceinline__ u64 csub_n(u64 x, u64 m, u64 nm) { return x >= m ? x + nm : x; }

// ---- Harvey butterflies (Algorithms 4 and 5, word size 2^64) ----------------
// Forward, inputs and outputs in [0, 4q):
//   X0 <- (X0 mod 2q) + W X1,  X1 <- (X0 mod 2q) + 2q - W X1,
// with W X1 the Shoup product in [0, 2q).  q2 = 2q, nq = 2^64 - q, nq2 = 2^64 - 2q.
__device__ __forceinline__ void harvey_fwd(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  u64 d;                                               // x0 - 2q
  const u64 t = shoup_mul_f<true>(x1, w, wp, nq, x0, nq2, d);
  const u64 a = x0 >= q2 ? d : x0;
  x0 = a + t;
  x1 = a + q2 - t;
}

// Inverse, inputs and outputs in [0, 2q):
//   X0 <- (X0 + X1) mod 2q,  X1 <- W (X0 + 2q - X1) mod q in [0, 2q).
__device__ __forceinline__ void harvey_inv(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  const u64 d = x0 + q2 - x1;
  u64 s;                                               // x0 + x1
  x1 = shoup_mul_f<true, false, false>(d, w, wp, nq, x0, x1, s);
  x0 = csub_n(s, q2, nq2);
}

// Last inverse stage with the scaling by N^{-1} folded in (Algorithm 3's final
// loop): X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 + 2q - X1), both in [0, 2q).
__device__ __forceinline__ void harvey_inv_last(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp, u64 q2,
                                                u64 nq) {
  const u64 s = x0 + x1;
  u64 d;                                               // x0 + 2q - x1, formed in two steps
  const u64 y0 = shoup_mul_f<true, true, true>(s, ni, nip, nq, x0, q2, d);
  x1 = shoup_mul<true, true>(d - x1, wn, wnp, nq);
  x0 = y0;
}

// ---- Wide-range variants (moduli below 2^58, single-pass kernels) ----------
//
// Same butterflies with two changes that trade the paper's tight output ranges
// for fewer instructions, valid while every value stays below 2^64:
//   - the Shoup quotient is taken without the low partial product
//     lo(W') lo(X), whose carry into the high word is at most 1.  The estimate
//     Q' is then Q or Q - 1, so T = W X - Q' q lies in [0, 3q) (the bound
//     [0, 2q) of the exact quotient, plus q) for every X < 2^64;
//   - the forward skips the reduction of X0 to [0, 2q):
//     X0 <- X0 + T, X1 <- X0 + 3q - T, so both grow by less than 3q a stage.
// From inputs below f q, after s forward stages every value is below
// (f + 3 s) q: 46 q < 2^64 for f = 4, s = 14 and q < 2^58.  The inverse keeps
// its values in [0, 4q) (one conditional subtraction of 4q per sum), its
// products in [0, 3q).  Outputs are congruent to the paper's mod q; the last
// step of a transform brings them into the paper's output ranges.

// Forward, wide range: X0 <- X0 + T, X1 <- X0 + 3q - T with T = W X1 mod q in
// [0, 3q).  q3 = 3q, nq = 2^64 - q.
__device__ __forceinline__ void harvey_fwd_wide(u64& x0, u64& x1, u64 w, u64 wp, u64 q3, u64 nq) {
  u64 a3;                                              // x0 + 3q
  const u64 t = shoup_mul_f<false>(x1, w, wp, nq, x0, q3, a3);
  x0 = x0 + t;
  x1 = a3 - t;
}

// Inverse, wide range, inputs in [0, 4q): X0 <- (X0 + X1) reduced once by 4q,
// in [0, 4q); X1 <- W (X0 + 4q - X1) mod q in [0, 3q).  q4 = 4q, nq4 = 2^64 - 4q.
__device__ __forceinline__ void harvey_inv_wide(u64& x0, u64& x1, u64 w, u64 wp, u64 q4, u64 nq, u64 nq4) {
  const u64 d = x0 + q4 - x1;
  u64 s;                                               // x0 + x1
  x1 = shoup_mul_f<false, false, false>(d, w, wp, nq, x0, x1, s);
  x0 = csub_n(s, q4, nq4);
}

// Last inverse stage with N^{-1}, wide range, inputs in [0, 4q):
// X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 + 4q - X1), both in [0, 3q).
__device__ __forceinline__ void harvey_inv_last_wide(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp,
                                                     u64 q4, u64 nq) {
  const u64 s = x0 + x1;
  u64 d;                                               // x0 + 4q - x1, formed in two steps
  const u64 y0 = shoup_mul_f<false, true, true>(s, ni, nip, nq, x0, q4, d);
  x1 = shoup_mul<false, true>(d - x1, wn, wnp, nq);
  x0 = y0;
}

// x mod q in [0, 3q) for any x < 2^64: a Shoup multiplication by 1 with the
// companion r = floor(2^64 / q) and the quotient estimate of the wide
// butterflies.  Brings the forward's wide outputs back into [0, 4q).
__device__ __forceinline__ u64 reduce_wide(u64 x, u64 r, u64 nq) {
  const u32 xl = lo32(x), xh = hi32(x);
  u64 m, c, j;
  u32 cb;
  asm("v_mad_u64_u32 %[m], %[j], %[rl], %[xh], 0\n\t"
      "v_mad_u64_u32 %[m], %[c], %[rh], %[xl], %[m]\n\t"
      "s_nop 1\n\t"
      "v_addc_co_u32 %[cb], %[j], 0, 0, %[c]"
      : [m] "=&v"(m), [cb] "=&v"(cb), [c] "=&s"(c), [j] "=&s"(j)
      : [xl] "v"(xl), [xh] "v"(xh), [rl] "s"(lo32(r)), [rh] "s"(hi32(r)));
  const u64 Q = mad32(hi32(r), xh, ((u64)cb << 32) | hi32(m));
  const u64 t = mad32(lo32(Q), lo32(nq), x);                    // x - Q q mod 2^64, low products
  return ((u64)(hi32(t) + lo32(Q) * hi32(nq) + hi32(Q) * lo32(nq)) << 32) | lo32(t);
}

// The transform templates take a butterfly flavour flag; every flavour now
// runs the same compiler-scheduled code above.
template <bool HAND>
__device__ __forceinline__ void bfly_fwd(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  harvey_fwd(x0, x1, w, wp, q2, nq, nq2);
}
template <bool HAND>
__device__ __forceinline__ void bfly_inv(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  harvey_inv(x0, x1, w, wp, q2, nq, nq2);
}
template <bool HAND>
__device__ __forceinline__ void bfly_inv_last(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp, u64 q2, u64 nq) {
  harvey_inv_last(x0, x1, ni, nip, wn, wnp, q2, nq);
}

// x mod q for x in [0, 4q): the two-step small_mod of Section 4.
__device__ __forceinline__ u64 reduce4(u64 x, u64 q, u64 q2) { return csub(csub(x, q2), q); }

// Algorithm 8 semantics: x * y mod q for x, y in [0, f q) with f in {1, 2, 4}.
// Inputs are first reduced to [0, q); then Barrett reduction with
// Q = floor(log2 q) + 1, L = 63 + Q, k = floor(2^L / q):
//   c1 = (x y) >> (Q - 1);  c3 = floor(c1 k / 2^64);  c4 = x y - c3 q.
// The quotient estimate c3 can be short by up to 2, so c4 < 3q and two
// conditional subtractions give the canonical value.
template <int F, bool CANON = true>
__device__ __forceinline__ u64 barrett_mulmod(u64 x, u64 y, u64 q, u64 q2, u64 k, u32 qbits) {
  if (F >= 4) { x = csub(x, q2); y = csub(y, q2); }
  if (F >= 2) { x = csub(x, q); y = csub(y, q); }
  u64 hi, lo;
  mul128(x, y, hi, lo);
  const u32 s = qbits - 1;                          // 1 <= s <= 61
  const u64 c1 = (lo >> s) | (hi << (64 - s));
  const u64 c3 = mulhi64(c1, k);
  u64 c4 = lo - c3 * q;
  if constexpr (!CANON) return c4;                   // [0, 3q): for consumers that accept it
  c4 = csub(c4, q);
  return csub(c4, q);
}

}  // namespace nttamd
