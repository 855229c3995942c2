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

// ---- Harvey butterflies, plain C++ -----------------------------------------
// Algorithm 4 (forward, inputs and outputs in [0, 4q)) and Algorithm 5
// (inverse, [0, 2q)), written directly; the hand-scheduled versions below
// compute the same words.
__device__ __forceinline__ void harvey_fwd_c(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq) {
  const u64 a = csub(x0, q2);
  const u64 t = shoup_mul(x1, w, wp, nq);          // [0, 2q)
  x0 = a + t;
  x1 = a + q2 - t;
}
__device__ __forceinline__ void harvey_inv_c(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq) {
  const u64 y0 = csub(x0 + x1, q2);
  const u64 t = x0 + q2 - x1;
  x1 = shoup_mul(t, w, wp, nq);
  x0 = y0;
}
__device__ __forceinline__ void harvey_inv_last_c(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp, u64 q2,
                                                  u64 nq) {
  const u64 s = x0 + x1;
  const u64 t = x0 + q2 - x1;
  x0 = shoup_mul(s, ni, nip, nq);
  x1 = shoup_mul(t, wn, wnp, nq);
}

// ---- Harvey butterflies in gfx950 assembly --------------------------------
// The arithmetic of Algorithms 4 and 5 exactly as in shoup_mul / csub above
// (exact MulHi, low-word remainder, the same lazy corrections), scheduled by
// hand as one statement per butterfly.  Written in C++, every 32-bit value
// that enters a 64-bit addend ({x, 0}) costs the compiler a register copy and
// its carries cost hazard padding; here
//   - x0 and x1 are updated in place (tied operands) and every temporary
//     lives in six fixed scratch registers, the pairs P = v[122:123],
//     T = v[124:125], M = v[126:127], so a butterfly adds little register
//     pressure and halves of temporaries can be named;
//   - the MulHi is four 32 x 32 -> 64 products; the carry of its middle sum
//     travels in an SGPR pair;
//   - the remainder T = W X + Q nq (mod 2^64) is two products into the pair
//     plus four cross products that only reach the high word, summed in the
//     low word of M and shifted up;
//   - each VALU write of an SGPR (carry, compare mask, borrow) is followed by
//     at least two other instructions before a VALU reads it;
//   - every input is read before the tied output that may share its register
//     is written.
// Kernels that use these butterflies need a VGPR budget of at least 128.
#define NTTAMD_CLOBBERS "v122", "v123", "v124", "v125", "v126", "v127"

// Algorithm 4 (Harvey forward butterfly), beta = 2^64, inputs in [0, 4q),
// outputs in [0, 4q):  X0 <- X0 + W X1,  X1 <- X0 - W X1  (mod q).
// nq = 2^64 - q, nq2 = 2^64 - 2q.  Only P = v[124:125] and T = v[126:127]
// are used: once Q has served its low-word product, its pair holds the 32-bit
// cross products.  X1 is written last (its two halves by the final
// subtraction), so it may reuse an input register; X0 is written before the
// last read of 2q and is therefore early-clobber (an
// "s" operand can end up in a VGPR where the compiler cannot keep it uniform,
// e.g. inside a non-inlined function).
__device__ __forceinline__ void harvey_fwd(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  u64 k, c, j, b, y0;
  u32 y1l, y1h;
  asm volatile("v_cmp_le_u64 %[k], %[q2], %[x0]\n\t"                 // x0 >= 2q
      "v_mad_u64_u32 v[124:125], %[j], %[pl], %[x1l], 0\n\t"        // P = MulHi(W', X1) ...
      "v_lshrrev_b64 v[124:125], 32, v[124:125]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[pl], %[x1h], v[124:125]\n\t"
      "v_mad_u64_u32 v[124:125], %[c], %[ph], %[x1l], v[124:125]\n\t"
      "v_mov_b32 v124, v125\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[wl], %[x1l], 0\n\t"        // T = W X1 (low products)
      "v_addc_co_u32 v125, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[ph], %[x1h], v[124:125]\n\t"   // ... P = Q
      "v_mad_u64_u32 v[126:127], %[j], v124, %[nql], v[126:127]\n\t"    // T += Q0 nq0
      "v_mul_lo_u32 v124, v124, %[nqh]\n\t"                         // cross products (high word only)
      "v_mul_lo_u32 v125, v125, %[nql]\n\t"
      "v_add3_u32 v127, v127, v124, v125\n\t"
      "v_mul_lo_u32 v124, %[wl], %[x1h]\n\t"
      "v_mul_lo_u32 v125, %[wh], %[x1l]\n\t"
      "v_add3_u32 v127, v127, v124, v125\n\t"                       // T = W X1 mod q in [0, 2q)
      "v_lshl_add_u64 v[124:125], %[x0], 0, %[nq2]\n\t"            // x0 - 2q
      "v_cndmask_b32 v124, %[x0l], v124, %[k]\n\t"
      "v_cndmask_b32 v125, %[x0h], v125, %[k]\n\t"                  // A = x0 mod 2q in [0, 2q)
      "v_lshl_add_u64 %[y0], v[124:125], 0, v[126:127]\n\t"         // X0 = A + T
      "v_lshl_add_u64 v[124:125], v[124:125], 0, %[q2]\n\t"         // A + 2q
      "v_sub_co_u32 %[y1l], %[b], v124, v126\n\t"
      "s_nop 1\n\t"
      "v_subb_co_u32 %[y1h], %[b], v125, v127, %[b]"                 // X1 = A + 2q - T
      : [y0] "=&v"(y0), [y1l] "=v"(y1l), [y1h] "=v"(y1h), [k] "=&s"(k), [c] "=&s"(c), [j] "=&s"(j),
        [b] "=&s"(b)
      : [x0] "v"(x0), [x0l] "v"(lo32(x0)), [x0h] "v"(hi32(x0)), [x1l] "v"(lo32(x1)), [x1h] "v"(hi32(x1)),
        [wl] "v"(lo32(w)), [wh] "v"(hi32(w)), [pl] "v"(lo32(wp)), [ph] "v"(hi32(wp)), [q2] "s"(q2), [nq2] "s"(nq2),
        [nql] "s"(lo32(nq)), [nqh] "s"(hi32(nq))
      : "v124", "v125", "v126", "v127");
  x0 = y0;
  x1 = ((u64)y1h << 32) | y1l;
}

// Algorithm 5 (Harvey inverse butterfly), inputs in [0, 2q), outputs in
// [0, 2q):  X0 <- X0 + X1,  X1 <- W (X0 - X1)  (mod q).  The halves of X0
// are selected straight into their output registers, before the last input
// reads, so they are early-clobber; X1 is written last, so it may reuse the
// input registers.
__device__ __forceinline__ void harvey_inv(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  u64 k, c, j, b, y1;
  u32 y0l, y0h;
  asm volatile("v_lshl_add_u64 v[124:125], %[x0], 0, %[q2]\n\t"              // x0 + 2q
      "v_lshl_add_u64 v[126:127], %[x0], 0, %[x1]\n\t"              // S = x0 + x1 < 4q
      "v_sub_co_u32 v124, %[b], v124, %[x1l]\n\t"
      "v_cmp_le_u64 %[k], %[q2], v[126:127]\n\t"                    // S >= 2q
      "v_lshl_add_u64 v[122:123], v[126:127], 0, %[nq2]\n\t"        // S - 2q
      "v_subb_co_u32 v125, %[b], v125, %[x1h], %[b]\n\t"            // T = D = x0 + 2q - x1 < 4q
      "v_cndmask_b32 %[y0l], v126, v122, %[k]\n\t"
      "v_cndmask_b32 %[y0h], v127, v123, %[k]\n\t"                  // X0 = S mod 2q
      "v_mad_u64_u32 v[122:123], %[j], %[pl], v124, 0\n\t"          // P = MulHi(W', D) ...
      "v_lshrrev_b64 v[122:123], 32, v[122:123]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[pl], v125, v[122:123]\n\t"
      "v_mad_u64_u32 v[122:123], %[c], %[ph], v124, v[122:123]\n\t"
      "v_mov_b32 v122, v123\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[wh], v124, 0\n\t"          // M = cross products
      "v_addc_co_u32 v123, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[ph], v125, v[122:123]\n\t" // ... P = Q
      "v_mad_u64_u32 v[126:127], %[j], %[wl], v125, v[126:127]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[wl], v124, 0\n\t"          // T = W D (low products); D dies
      "v_mad_u64_u32 v[124:125], %[j], v122, %[nql], v[124:125]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v122, %[nqh], v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v123, %[nql], v[126:127]\n\t"
      "v_lshlrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_lshl_add_u64 %[y1], v[124:125], 0, v[126:127]"              // X1 = W D mod q in [0, 2q)
      : [y0l] "=&v"(y0l), [y0h] "=&v"(y0h), [y1] "=v"(y1), [k] "=&s"(k), [c] "=&s"(c), [j] "=&s"(j),
        [b] "=&s"(b)
      : [x0] "v"(x0), [x1] "v"(x1), [x1l] "v"(lo32(x1)), [x1h] "v"(hi32(x1)), [wl] "v"(lo32(w)), [wh] "v"(hi32(w)),
        [pl] "v"(lo32(wp)), [ph] "v"(hi32(wp)), [q2] "s"(q2), [nq2] "s"(nq2), [nql] "s"(lo32(nq)),
        [nqh] "s"(hi32(nq))
      : NTTAMD_CLOBBERS);
  x0 = ((u64)y0h << 32) | y0l;
  x1 = y1;
}

// Last inverse stage fused with the scaling by N^{-1} (Algorithm 3's final
// loop): X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 - X1), both in [0, 2q).
// X1 is first copied into M so that both outputs, updated in place, can
// serve as scratch pairs once S and D are formed.  The four constants are
// uniform and enter as SGPRs (each instruction reads at most one SGPR).
__device__ __forceinline__ void harvey_inv_last(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp,
                                                u64 q2, u64 nq) {
  u64 c, j, b;
  asm volatile("v_lshl_add_u64 v[126:127], %[x1], 0, 0\n\t"                  // M = x1
      "v_lshl_add_u64 v[124:125], %[x0], 0, %[q2]\n\t"              // x0 + 2q
      "v_lshl_add_u64 v[122:123], %[x0], 0, %[x1]\n\t"              // P = S = x0 + x1 < 4q
      "v_sub_co_u32 v124, %[b], v124, v126\n\t"
      "v_mad_u64_u32 %[x0], %[j], %[nil], v122, 0\n\t"              // X0 = N^-1 S (low products) ...
      "v_mad_u64_u32 %[x1], %[j], %[nih], v122, 0\n\t"              // X1 = its cross products
      "v_subb_co_u32 v125, %[b], v125, v127, %[b]\n\t"              // T = D = x0 + 2q - x1 < 4q
      "v_mad_u64_u32 %[x1], %[j], %[nil], v123, %[x1]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[npl], v122, 0\n\t"         // M = MulHi(N^-1', S) ...
      "v_lshrrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[npl], v123, v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[c], %[nph], v122, v[126:127]\n\t"
      "v_mov_b32 v126, v127\n\t"
      "s_nop 0\n\t"
      "v_addc_co_u32 v127, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[nph], v123, v[126:127]\n\t" // ... M = Q
      "v_mad_u64_u32 %[x0], %[j], v126, %[nql], %[x0]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v126, %[nqh], %[x1]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v127, %[nql], %[x1]\n\t"
      "v_lshlrev_b64 %[x1], 32, %[x1]\n\t"
      "v_lshl_add_u64 %[x0], %[x0], 0, %[x1]\n\t"                   // X0 = N^-1 S mod q in [0, 2q)
      "v_mad_u64_u32 v[122:123], %[j], %[wpl], v124, 0\n\t"         // P = MulHi((W N^-1)', D) ...
      "v_lshrrev_b64 v[122:123], 32, v[122:123]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[wpl], v125, v[122:123]\n\t"
      "v_mad_u64_u32 v[122:123], %[c], %[wph], v124, v[122:123]\n\t"
      "v_mov_b32 v122, v123\n\t"
      "v_mad_u64_u32 %[x1], %[j], %[wnl], v124, 0\n\t"              // X1 = W N^-1 D (low products)
      "v_addc_co_u32 v123, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[wph], v125, v[122:123]\n\t" // ... P = Q
      "v_mad_u64_u32 v[126:127], %[j], %[wnh], v124, 0\n\t"         // M = cross products
      "v_mad_u64_u32 v[126:127], %[j], %[wnl], v125, v[126:127]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v122, %[nql], %[x1]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v122, %[nqh], v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v123, %[nql], v[126:127]\n\t"
      "v_lshlrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_lshl_add_u64 %[x1], %[x1], 0, v[126:127]"                   // X1 = W N^-1 D mod q in [0, 2q)
      : [x0] "+v"(x0), [x1] "+v"(x1), [c] "=&s"(c), [j] "=&s"(j), [b] "=&s"(b)
      : [nil] "s"(lo32(ni)), [nih] "s"(hi32(ni)), [npl] "s"(lo32(nip)), [nph] "s"(hi32(nip)), [wnl] "s"(lo32(wn)),
        [wnh] "s"(hi32(wn)), [wpl] "s"(lo32(wnp)), [wph] "s"(hi32(wnp)), [q2] "s"(q2), [nql] "s"(lo32(nq)),
        [nqh] "s"(hi32(nq))
      : NTTAMD_CLOBBERS);
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

// Forward butterfly, wide range: X0 <- X0 + T, X1 <- X0 + 3q - T with
// T = W X1 mod q in [0, 3q).  q3 = 3q, nq = 2^64 - q.
__device__ __forceinline__ void harvey_fwd_wide(u64& x0, u64& x1, u64 w, u64 wp, u64 q3, u64 nq) {
  u64 c, j, b, y0;
  u32 y1l, y1h;
  asm volatile("v_mad_u64_u32 v[124:125], %[j], %[pl], %[x1h], 0\n\t"        // P = lo(W') hi(X1) ...
      "v_mad_u64_u32 v[124:125], %[c], %[ph], %[x1l], v[124:125]\n\t" // + hi(W') lo(X1), carry c
      "v_mad_u64_u32 v[126:127], %[j], %[wl], %[x1l], 0\n\t"        // T = W X1 (low products)
      "v_mov_b32 v124, v125\n\t"
      "v_addc_co_u32 v125, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[ph], %[x1h], v[124:125]\n\t" // ... Q' = P >> 32 + hi(W') hi(X1)
      "v_mad_u64_u32 v[126:127], %[j], v124, %[nql], v[126:127]\n\t"  // T += Q'0 nq0
      "v_mul_lo_u32 v124, v124, %[nqh]\n\t"                          // cross products (high word only)
      "v_mul_lo_u32 v125, v125, %[nql]\n\t"
      "v_add3_u32 v127, v127, v124, v125\n\t"
      "v_mul_lo_u32 v124, %[wl], %[x1h]\n\t"
      "v_mul_lo_u32 v125, %[wh], %[x1l]\n\t"
      "v_add3_u32 v127, v127, v124, v125\n\t"                        // T = W X1 mod q in [0, 3q)
      "v_lshl_add_u64 v[124:125], %[x0], 0, %[q3]\n\t"               // x0 + 3q
      "v_sub_co_u32 %[y1l], %[b], v124, v126\n\t"
      "v_lshl_add_u64 %[y0], %[x0], 0, v[126:127]\n\t"               // X0 = x0 + T
      "s_nop 0\n\t"
      "v_subb_co_u32 %[y1h], %[b], v125, v127, %[b]"                 // X1 = x0 + 3q - T
      : [y0] "=v"(y0), [y1l] "=&v"(y1l), [y1h] "=v"(y1h), [c] "=&s"(c), [j] "=&s"(j), [b] "=&s"(b)
      : [x0] "v"(x0), [x1l] "v"(lo32(x1)), [x1h] "v"(hi32(x1)), [wl] "v"(lo32(w)), [wh] "v"(hi32(w)),
        [pl] "v"(lo32(wp)), [ph] "v"(hi32(wp)), [q3] "s"(q3), [nql] "s"(lo32(nq)), [nqh] "s"(hi32(nq))
      : "v124", "v125", "v126", "v127");
  x0 = y0;
  x1 = ((u64)y1h << 32) | y1l;
}

// Inverse butterfly, wide range, inputs in [0, 4q): X0 <- (X0 + X1) reduced
// once by 4q, in [0, 4q); X1 <- W (X0 + 4q - X1) mod q in [0, 3q).
// q4 = 4q, nq4 = 2^64 - 4q.
__device__ __forceinline__ void harvey_inv_wide(u64& x0, u64& x1, u64 w, u64 wp, u64 q4, u64 nq, u64 nq4) {
  u64 k, c, j, b, y1;
  u32 y0l, y0h;
  asm volatile("v_lshl_add_u64 v[124:125], %[x0], 0, %[q4]\n\t"              // x0 + 4q
      "v_lshl_add_u64 v[126:127], %[x0], 0, %[x1]\n\t"              // S = x0 + x1 < 8q
      "v_sub_co_u32 v124, %[b], v124, %[x1l]\n\t"
      "v_cmp_le_u64 %[k], %[q4], v[126:127]\n\t"                    // S >= 4q
      "v_lshl_add_u64 v[122:123], v[126:127], 0, %[nq4]\n\t"        // S - 4q
      "v_subb_co_u32 v125, %[b], v125, %[x1h], %[b]\n\t"            // D = x0 + 4q - x1 < 8q
      "v_cndmask_b32 %[y0l], v126, v122, %[k]\n\t"
      "v_cndmask_b32 %[y0h], v127, v123, %[k]\n\t"                  // X0 in [0, 4q)
      "v_mad_u64_u32 v[122:123], %[j], %[pl], v125, 0\n\t"          // P = lo(W') hi(D) ...
      "v_mad_u64_u32 v[122:123], %[c], %[ph], v124, v[122:123]\n\t" // + hi(W') lo(D), carry c
      "v_mad_u64_u32 v[126:127], %[j], %[wh], v124, 0\n\t"          // M = cross products
      "v_mov_b32 v122, v123\n\t"
      "v_addc_co_u32 v123, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[ph], v125, v[122:123]\n\t" // ... P = Q'
      "v_mad_u64_u32 v[126:127], %[j], %[wl], v125, v[126:127]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[wl], v124, 0\n\t"          // T = W D (low products); D dies
      "v_mad_u64_u32 v[124:125], %[j], v122, %[nql], v[124:125]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v122, %[nqh], v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v123, %[nql], v[126:127]\n\t"
      "v_lshlrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_lshl_add_u64 %[y1], v[124:125], 0, v[126:127]"              // X1 = W D mod q in [0, 3q)
      : [y0l] "=&v"(y0l), [y0h] "=&v"(y0h), [y1] "=v"(y1), [k] "=&s"(k), [c] "=&s"(c), [j] "=&s"(j),
        [b] "=&s"(b)
      : [x0] "v"(x0), [x1] "v"(x1), [x1l] "v"(lo32(x1)), [x1h] "v"(hi32(x1)), [wl] "v"(lo32(w)), [wh] "v"(hi32(w)),
        [pl] "v"(lo32(wp)), [ph] "v"(hi32(wp)), [q4] "s"(q4), [nq4] "s"(nq4), [nql] "s"(lo32(nq)),
        [nqh] "s"(hi32(nq))
      : NTTAMD_CLOBBERS);
  x0 = ((u64)y0h << 32) | y0l;
  x1 = y1;
}

// Last inverse stage with N^{-1}, wide range, inputs in [0, 4q):
// X0 <- N^{-1} (X0 + X1), X1 <- (W N^{-1}) (X0 + 4q - X1), both in [0, 3q).
__device__ __forceinline__ void harvey_inv_last_wide(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp,
                                                     u64 q4, u64 nq) {
  u64 c, j, b;
  asm volatile("v_lshl_add_u64 v[126:127], %[x1], 0, 0\n\t"                  // M = x1
      "v_lshl_add_u64 v[124:125], %[x0], 0, %[q4]\n\t"              // x0 + 4q
      "v_lshl_add_u64 v[122:123], %[x0], 0, %[x1]\n\t"              // P = S = x0 + x1 < 8q
      "v_sub_co_u32 v124, %[b], v124, v126\n\t"
      "v_mad_u64_u32 %[x0], %[j], %[nil], v122, 0\n\t"              // X0 = N^-1 S (low products) ...
      "v_mad_u64_u32 %[x1], %[j], %[nih], v122, 0\n\t"              // X1 = its cross products
      "v_subb_co_u32 v125, %[b], v125, v127, %[b]\n\t"              // T = D = x0 + 4q - x1 < 8q
      "v_mad_u64_u32 %[x1], %[j], %[nil], v123, %[x1]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[npl], v123, 0\n\t"         // M = Q' for (N^-1', S) ...
      "v_mad_u64_u32 v[126:127], %[c], %[nph], v122, v[126:127]\n\t"
      "v_mov_b32 v126, v127\n\t"
      "s_nop 0\n\t"
      "v_addc_co_u32 v127, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], %[nph], v123, v[126:127]\n\t" // ... M = Q'
      "v_mad_u64_u32 %[x0], %[j], v126, %[nql], %[x0]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v126, %[nqh], %[x1]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v127, %[nql], %[x1]\n\t"
      "v_lshlrev_b64 %[x1], 32, %[x1]\n\t"
      "v_lshl_add_u64 %[x0], %[x0], 0, %[x1]\n\t"                   // X0 = N^-1 S mod q in [0, 3q)
      "v_mad_u64_u32 v[122:123], %[j], %[wpl], v125, 0\n\t"         // P = Q' for ((W N^-1)', D) ...
      "v_mad_u64_u32 v[122:123], %[c], %[wph], v124, v[122:123]\n\t"
      "v_mad_u64_u32 %[x1], %[j], %[wnl], v124, 0\n\t"              // X1 = W N^-1 D (low products)
      "v_mov_b32 v122, v123\n\t"
      "v_addc_co_u32 v123, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[122:123], %[j], %[wph], v125, v[122:123]\n\t" // ... P = Q'
      "v_mad_u64_u32 v[126:127], %[j], %[wnh], v124, 0\n\t"         // M = cross products
      "v_mad_u64_u32 v[126:127], %[j], %[wnl], v125, v[126:127]\n\t"
      "v_mad_u64_u32 %[x1], %[j], v122, %[nql], %[x1]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v122, %[nqh], v[126:127]\n\t"
      "v_mad_u64_u32 v[126:127], %[j], v123, %[nql], v[126:127]\n\t"
      "v_lshlrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_lshl_add_u64 %[x1], %[x1], 0, v[126:127]"                   // X1 = W N^-1 D mod q in [0, 3q)
      : [x0] "+v"(x0), [x1] "+v"(x1), [c] "=&s"(c), [j] "=&s"(j), [b] "=&s"(b)
      : [nil] "s"(lo32(ni)), [nih] "s"(hi32(ni)), [npl] "s"(lo32(nip)), [nph] "s"(hi32(nip)), [wnl] "s"(lo32(wn)),
        [wnh] "s"(hi32(wn)), [wpl] "s"(lo32(wnp)), [wph] "s"(hi32(wnp)), [q4] "s"(q4), [nql] "s"(lo32(nq)),
        [nqh] "s"(hi32(nq))
      : NTTAMD_CLOBBERS);
}

// x mod q in [0, 3q) for any x < 2^64: a Shoup multiplication by 1 with the
// companion r = floor(2^64 / q) and the quotient estimate of the wide
// butterflies.  Brings the forward's wide outputs back into [0, 4q).
__device__ __forceinline__ u64 reduce_wide(u64 x, u64 r, u64 nq) {
  u64 c, j, y;
  asm volatile("v_mad_u64_u32 v[124:125], %[j], %[rl], %[xh], 0\n\t"         // P = lo(r) hi(x) ...
      "v_mad_u64_u32 v[124:125], %[c], %[rh], %[xl], v[124:125]\n\t" // + hi(r) lo(x), carry c
      "v_mov_b32 v124, v125\n\t"
      "s_nop 0\n\t"
      "v_addc_co_u32 v125, %[j], 0, 0, %[c]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], %[rh], %[xh], v[124:125]\n\t" // ... Q'
      "v_mad_u64_u32 v[126:127], %[j], v124, %[nqh], 0\n\t"          // cross products
      "v_mad_u64_u32 v[126:127], %[j], v125, %[nql], v[126:127]\n\t"
      "v_mad_u64_u32 v[124:125], %[j], v124, %[nql], %[x]\n\t"       // x + Q'0 nq0
      "v_lshlrev_b64 v[126:127], 32, v[126:127]\n\t"
      "v_lshl_add_u64 %[y], v[124:125], 0, v[126:127]"                // x - Q' q in [0, 3q)
      : [y] "=v"(y), [c] "=&s"(c), [j] "=&s"(j)
      : [x] "v"(x), [xl] "v"(lo32(x)), [xh] "v"(hi32(x)), [rl] "s"(lo32(r)), [rh] "s"(hi32(r)),
        [nql] "s"(lo32(nq)), [nqh] "s"(hi32(nq))
      : "v124", "v125", "v126", "v127");
  return y;
}

#undef NTTAMD_CLOBBERS

// Butterfly selection for the transform templates: HAND = the hand-scheduled
// versions above, else the plain C++ ones (used where the statements would sit
// inside non-inlined device functions).
template <bool HAND>
__device__ __forceinline__ void bfly_fwd(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  if constexpr (HAND) harvey_fwd(x0, x1, w, wp, q2, nq, nq2);
  else harvey_fwd_c(x0, x1, w, wp, q2, nq);
}
template <bool HAND>
__device__ __forceinline__ void bfly_inv(u64& x0, u64& x1, u64 w, u64 wp, u64 q2, u64 nq, u64 nq2) {
  if constexpr (HAND) harvey_inv(x0, x1, w, wp, q2, nq, nq2);
  else harvey_inv_c(x0, x1, w, wp, q2, nq);
}
template <bool HAND>
__device__ __forceinline__ void bfly_inv_last(u64& x0, u64& x1, u64 ni, u64 nip, u64 wn, u64 wnp, u64 q2, u64 nq) {
  if constexpr (HAND) harvey_inv_last(x0, x1, ni, nip, wn, wnp, q2, nq);
  else harvey_inv_last_c(x0, x1, ni, nip, wn, wnp, q2, nq);
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
