// Single-pass transform of one limb held by one workgroup (N <= 2^14), as a
// device-side building block: used by the single-pass kernel and by the
// persistent batch kernel.  See ntt_onchip.hip for the design notes.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"

namespace nttamd {

// WIDE: the wide-range butterflies (moduli below 2^58); the caller brings the
// forward's outputs back into [0, 4q) and the inverse's into [0, 2q).
// TBSEL: twiddle pairs per prefetch block for this use (0: the rule below).
template <bool FWD, int LOGN, int LOGR, bool SPLIT, bool HAND = true, bool WIDE = false, int TBSEL = 0>
struct OnChip {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int NT = N >> LOGR;
  static constexpr int LDSW = N + (N >> LOGR);
  // transposed sub-tables are laid out for onchip_logr(LOGN) coefficients per thread
  static constexpr int PERM_TOP = LOGR == onchip_logr(LOGN) ? onchip_perm_top(FWD, LOGN) : -1;
  // Twiddle pairs per prefetch block.  The next block's loads are issued before
  // the current block's butterflies, so in the short-stride stages (one
  // butterfly per twiddle) a block must hold enough butterflies to cover the
  // latency of an L2 hit.  At 32 coefficients per thread, within 128 registers:
  // one pair with the paper's forward butterflies and three with the wide ones
  // (measured fastest; four spill).
  static constexpr int TB = TBSEL > 0 ? TBSEL : (HAND && FWD && LOGR >= 5 ? (WIDE ? 3 : 1) : 2);
  using G = Geo<FWD, LOGN, LOGR>;
  using W = typename std::conditional<SPLIT, u32, u64>::type;

  template <int r>
  __device__ static __forceinline__ u32 rho(u32 t, int j) {
    constexpr int lo = G::lo(r);
    return ((t >> lo) << (lo + LOGR)) | ((u32)j << lo) | (t & ((1u << lo) - 1u));
  }
  __device__ static __forceinline__ u32 row(u32 r) { return r + (r >> LOGR); }

  // Padded LDS row of element j of thread t in round r, split into a per-thread
  // base and a compile-time offset of j.  With rho = hi | (j << lo) | lp
  // (hi a multiple of 2^(lo+LOGR), lp < 2^lo), rho >> LOGR is exactly
  // (hi >> LOGR) + (lp >> LOGR) + (j << lo >> LOGR) for lo >= LOGR, and
  // (hi >> LOGR) + (j >> (LOGR - lo)) for lo < LOGR.
  template <int r>
  __device__ static __forceinline__ u32 row_base(u32 t) {
    constexpr int lo = G::lo(r);
    const u32 hi = (t >> lo) << (lo + LOGR);
    const u32 lp = t & ((1u << lo) - 1u);
    return hi + (hi >> LOGR) + lp + (lo >= LOGR ? (lp >> LOGR) : 0u);
  }
  template <int r>
  static constexpr u32 row_off(int j) {
    constexpr int lo = G::lo(r);
    return ((u32)j << lo) + (lo >= LOGR ? ((u32)j << (lo - LOGR)) : ((u32)j >> (LOGR - lo)));
  }
  // Padded LDS row of tile element j * NT + t (the coalesced memory order).
  __device__ static __forceinline__ u32 lin_row(u32 t, int j) {
    if constexpr (LOGN >= 2 * LOGR) return (u32)j * (NT + (NT >> LOGR)) + t + (t >> LOGR);
    else return row((u32)j * NT + t);
  }

  // Moves the thread's coefficients between two register layouts through LDS;
  // ROW_OUT(j) / ROW_IN(j) give the padded LDS rows written / read for element j.
  template <typename FO, typename FI>
  __device__ static __forceinline__ void shuffle(W* lds, u64 (&x)[R], FO row_out, FI row_in) {
    __syncthreads();
    if constexpr (!SPLIT) {
#pragma unroll
      for (int j = 0; j < R; ++j) lds[row_out(j)] = x[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = lds[row_in(j)];
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) lds[row_out(j)] = lo32(x[j]);
      __syncthreads();
      u32 nl[R];
#pragma unroll
      for (int j = 0; j < R; ++j) nl[j] = lds[row_in(j)];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < R; ++j) lds[row_out(j)] = hi32(x[j]);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = ((u64)lds[row_in(j)] << 32) | nl[j];
    }
  }

  // twiddle pair u of the stage on local bit `bit` in round r for thread t
  template <int r>
  __device__ static __forceinline__ ulonglong2 twiddle(const PlanView& pv, u32 t, int bit, int u) {
    constexpr int lo = G::lo(r);
    if (lo == 0 && bit <= PERM_TOP) return pv.twp[(N >> (bit + 1)) + (u32)u * NT + t];
    return pv.tw[((N + rho<r>(t, 0)) >> (bit + 1)) + (u32)u];
  }

  // number of twiddle blocks of stage s in round r
  template <int r>
  static constexpr int nblocks(int s) {
    return ((R >> ((FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s)) - G::lo(r) + 1)) + TB - 1) / TB;
  }
  // first step (global block counter) of stage s in round r
  template <int r>
  static constexpr int first_step(int s) {
    int n = 0;
    for (int i = 0; i < s; ++i) n += nblocks<r>(i);
    return n;
  }

  template <int r>
  __device__ static __forceinline__ void stages(u64 (&x)[R], u32 t, const PlanView& pv) {
    constexpr int lo = G::lo(r);
    constexpr int NS = G::nst(r);
    // two twiddle buffers used alternately by consecutive blocks (ping-pong on
    // the compile-time block counter, so no register copies are needed)
    ulonglong2 buf[2][TB];
    auto load_block = [&](ulonglong2 (&dst)[TB], int s, int blk) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int p = bit - lo;
      const int n = R >> (p + 1);
      const bool fused_last = !FWD && bit == LOGN - 1;
      if (fused_last) return;
#pragma unroll
      for (int i = 0; i < TB; ++i)
        if (blk * TB + i < n) dst[i] = twiddle<r>(pv, t, bit, blk * TB + i);
    };
    load_block(buf[0], 0, 0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int p = bit - lo;
      const int n = R >> (p + 1);
      const int nb = (n + TB - 1) / TB;
      const bool fused_last = !FWD && bit == LOGN - 1;
#pragma unroll
      for (int blk = 0; blk < nb; ++blk) {
        const int step = first_step<r>(s) + blk;
        ulonglong2 (&cur)[TB] = buf[step & 1];
        ulonglong2 (&nxt)[TB] = buf[(step + 1) & 1];
        if (blk + 1 < nb) load_block(nxt, s, blk + 1);
        else if (s + 1 < NS) load_block(nxt, s + 1, 0);
#pragma unroll
        for (int i = 0; i < TB; ++i) {
          const int u = blk * TB + i;
          if (u >= n) continue;
#pragma unroll
          for (int m = 0; m < (1 << p); ++m) {
            const int j = (u << (p + 1)) | m;
            const int j2 = j | (1 << p);
            if constexpr (WIDE) {
              if (FWD) harvey_fwd_wide(x[j], x[j2], cur[i].x, cur[i].y, pv.q3, pv.nq);
              else if (fused_last) harvey_inv_last_wide(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q4, pv.nq);
              else harvey_inv_wide(x[j], x[j2], cur[i].x, cur[i].y, pv.q4, pv.nq, pv.nq4);
            } else {
              if (FWD) bfly_fwd<HAND>(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq, pv.nq2);
              else if (fused_last) bfly_inv_last<HAND>(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q2, pv.nq);
              else bfly_inv<HAND>(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq, pv.nq2);
            }
          }
        }
        stage_fence();
      }
    }
  }

  template <int r>
  __device__ static __forceinline__ void run(W* lds, u64 (&x)[R], u32 t, const PlanView& pv) {
    stages<r>(x, t, pv);
    if constexpr (r + 1 < G::NR) {
      const u32 bo = row_base<r>(t), bi = row_base<r + 1>(t);
      shuffle(lds, x, [&](int j) { return bo + row_off<r>(j); }, [&](int j) { return bi + row_off<r + 1>(j); });
      run<r + 1>(lds, x, t, pv);
    }
  }
};

// A copy of v the compiler cannot see through: index arithmetic for the output
// phase is then recomputed instead of being kept (and spilled) from the input
// phase.
__device__ __forceinline__ u32 opaque(u32 v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Brings a wide-range transform output into the ranges of the paper's
// butterflies: the forward's [0, 4q) (here [0, 3q)), the inverse's [0, 2q).
template <bool FWD, bool WIDE>
__device__ __forceinline__ u64 unwiden(u64 v, const PlanView& pv) {
  if constexpr (!WIDE) return v;
  else if constexpr (FWD) return reduce_wide(v, pv.rq, pv.nq);
  else return csub(v, pv.q2);
}

// Transforms one limb: reads `in` (N coefficients), writes `out`; the output
// step applies MODE with the per-item multiplier / accumulator `mul`.  t is the
// thread's index among the N / 2^LOGR threads that hold the limb; with active
// false the threads run every step and barrier but store nothing (a sub-group
// without a limb of its own, reading another's input).  FRESH: the twiddle and
// output indices start from fresh views of t, so the compiler recomputes them
// instead of keeping the input phase's (which spills inside a loop over limbs).
template <bool FWD, int LOGN, int LOGR, bool SPLIT, int MODE, bool HAND = true, bool WIDE = false, bool FRESH = false>
__device__ __forceinline__ void onchip_body(const PlanView& pv, const u64* in, u64* out, const u64* mul,
                                            typename OnChip<FWD, LOGN, LOGR, SPLIT, HAND, WIDE>::W* lds,
                                            bool nt_load, u32 t, bool active) {
  using K = OnChip<FWD, LOGN, LOGR, SPLIT, HAND, WIDE>;
  constexpr int R = K::R;
  constexpr int NT = K::NT;
  constexpr int RL = K::G::NR - 1;
  constexpr bool direct_in = K::G::lo(0) >= 4 || LOGN - LOGR < 4;
  constexpr bool direct_out = K::G::lo(RL) >= 4 || LOGN - LOGR < 4;
  u64 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &in[K::template rho<0>(t, j)];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &in[(u32)j * NT + t];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
    const u32 bi = K::template row_base<0>(t);
    K::shuffle(lds, x, [&](int j) { return K::lin_row(t, j); }, [&](int j) { return bi + K::template row_off<0>(j); });
  }

  K::template run<0>(lds, x, FRESH ? opaque(t) : t, pv);
  if constexpr (WIDE && FWD) {
    // before the output loop, so that its loads (fused multiply) can be grouped:
    // the compiler does not move memory accesses across these statements
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = unwiden<true, true>(x[j], pv);
  }

  const u32 to = FRESH ? opaque(t) : t;
  if constexpr (!direct_out) {
    const u32 bo = K::template row_base<RL>(to);
    K::shuffle(lds, x, [&](int j) { return bo + K::template row_off<RL>(j); }, [&](int j) { return K::lin_row(to, j); });
  }
  if (!active) return;                            // past the last barrier: nothing left but the stores
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u32 i = direct_out ? K::template rho<RL>(to, j) : (u32)j * NT + to;
    out[i] = finish_item<FWD, MODE>(FWD ? x[j] : unwiden<false, WIDE>(x[j], pv), mul, i, pv);
    if ((j & 7) == 7) stage_fence();
  }
}

// The negacyclic product of one limb kept on chip (the product listing of
// Section 4, fused): forward(b) lazy in [0, 4q), element-wise multiply by m =
// NTT(a) (lazy, [0, 4q)) with Algorithm 8, inverse, then the output step MODE
// (canonical, or accumulated into out).  With 2^LOGR coefficients per thread
// the forward's last round and the inverse's first round both give thread t
// the coefficients t R .. t R + R - 1, so the product and the inverse start
// in registers.  Every thread reads its multipliers before the inverse's
// first LDS barrier, so out may equal m.  With WIDE, the forward's outputs are
// first brought into [0, 3q), and the multiply leaves its remainder in [0, 3q)
// (no final corrections), which the wide inverse accepts.
template <int LOGN, int LOGR, bool SPLIT, int MODE, bool HAND = true, bool WIDE = false, bool FRESH = false>
__device__ __forceinline__ void onchip_product_body(const PlanView& pf, const PlanView& pi, const u64* b,
                                                    const u64* m, u64* out,
                                                    typename OnChip<true, LOGN, LOGR, SPLIT, HAND, WIDE>::W* lds,
                                                    bool nt_load, u32 t, bool active) {
  // The forward half names its block size explicitly: the same three pairs as the
  // rule gives, but as its own instantiation the compiler schedules the fused
  // kernel's registers better (measured 0.829 against 0.865 ms at N = 2^14 x 4096).
  using KF = OnChip<true, LOGN, LOGR, SPLIT, HAND, WIDE, (WIDE && LOGR >= 5) ? 3 : 0>;
  using KI = OnChip<false, LOGN, LOGR, SPLIT, HAND, WIDE>;
  constexpr int R = KF::R;
  constexpr int NT = KF::NT;
  constexpr int RLF = KF::G::NR - 1;
  constexpr int RLI = KI::G::NR - 1;
  static_assert(KF::G::lo(RLF) == 0 && KI::G::lo(0) == 0, "forward output and inverse input layouts must coincide");
  constexpr bool direct_in = KF::G::lo(0) >= 4 || LOGN - LOGR < 4;
  constexpr bool direct_out = KI::G::lo(RLI) >= 4 || LOGN - LOGR < 4;
  u64 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &b[KF::template rho<0>(t, j)];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &b[(u32)j * NT + t];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
    const u32 bi = KF::template row_base<0>(t);
    KF::shuffle(lds, x, [&](int j) { return KF::lin_row(t, j); }, [&](int j) { return bi + KF::template row_off<0>(j); });
  }
  KF::template run<0>(lds, x, FRESH ? opaque(t) : t, pf);
  if constexpr (WIDE) {
    // all reductions first: the compiler does not move the multiplier loads across
    // these statements, and grouped loads hide their latency
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = unwiden<true, true>(x[j], pf);
  }
  const u64* mt = m + ((u64)opaque(t) << LOGR);  // KF::rho<RLF>(t, j) = t R + j
#pragma unroll
  for (int j = 0; j < R; ++j) {
    // the wide inverse takes inputs in [0, 4q): Algorithm 8's remainder in [0, 3q) suffices
    x[j] = barrett_mulmod<4, !WIDE>(x[j], mt[j], pf.q, pf.q2, pf.bk, pf.qbits);
    if ((j & 7) == 7) stage_fence();
  }
  __syncthreads();                                // the forward's last LDS reads precede the inverse's writes
  KI::template run<0>(lds, x, t, pi);
  const u32 to = opaque(t);
  if constexpr (!direct_out) {
    const u32 bo = KI::template row_base<RLI>(to);
    KI::shuffle(lds, x, [&](int j) { return bo + KI::template row_off<RLI>(j); }, [&](int j) { return KI::lin_row(to, j); });
  }
  if (!active) return;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u32 i = direct_out ? KI::template rho<RLI>(to, j) : (u32)j * NT + to;
    out[i] = finish_item<false, MODE>(unwiden<false, WIDE>(x[j], pi), out, i, pi);
    if ((j & 7) == 7) stage_fence();
  }
}

}  // namespace nttamd
