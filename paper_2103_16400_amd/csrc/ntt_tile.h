// One tile of a two-pass transform (2^15 <= N <= 2^17), as a device-side
// building block: used by the two-pass kernels and by the persistent batch
// kernel.  See ntt_kernels.hip for the design notes.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"

namespace nttamd {

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, bool HAND = true>
struct TileNtt {
  static constexpr int R = 1 << LOGR;
  static constexpr int C = 1 << LOGC;
  static constexpr int RB = LOGT + LOGH;              // row bits of the tile (block bits on top)
  static constexpr int ROWS = 1 << RB;
  static constexpr int NT = (ROWS * C) >> LOGR;        // threads
  static constexpr int NO = NT >> LOGC;                // threads per column
  static constexpr int LDSW = (ROWS + (ROWS >> LOGR)) * C;
  static constexpr int TB = 2;                         // twiddle pairs per prefetch block
  static constexpr bool LOWPASS = LOGC == 0;
  using G = Geo<FWD, LOGT, LOGR>;

  template <int r>
  __device__ static __forceinline__ u32 rho(u32 o, int j) {
    constexpr int lo = G::lo(r);
    return ((o >> lo) << (lo + LOGR)) | ((u32)j << lo) | (o & ((1u << lo) - 1u));
  }
  // padded LDS row of element j of row-thread o in round r = row_base + row_off(j)
  template <int r>
  __device__ static __forceinline__ u32 row_base(u32 o) {
    constexpr int lo = G::lo(r);
    const u32 hi = (o >> lo) << (lo + LOGR);
    const u32 lp = o & ((1u << lo) - 1u);
    return hi + (hi >> LOGR) + lp + (lo >= LOGR ? (lp >> LOGR) : 0u);
  }
  template <int r>
  static constexpr u32 row_off(int j) {
    constexpr int lo = G::lo(r);
    return ((u32)j << lo) + (lo >= LOGR ? ((u32)j << (lo - LOGR)) : ((u32)j >> (LOGR - lo)));
  }
  __device__ static __forceinline__ u32 prow(u32 r) { return r + (r >> LOGR); }
  // low pass, coalesced order: element e = j * NT + t of the tile
  __device__ static __forceinline__ u32 lin_row(u32 t, int j) {
    if constexpr (RB >= 2 * LOGR) return (u32)j * (NT + (NT >> LOGR)) + t + (t >> LOGR);
    else return prow((u32)j * NT + t);
  }

  template <typename FO, typename FI>
  __device__ static __forceinline__ void shuffle(u64* lds, u64 (&x)[R], u32 c, FO row_out, FI row_in) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) lds[row_out(j) * C + c] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = lds[row_in(j) * C + c];
  }

  template <int r>
  __device__ static __forceinline__ ulonglong2 twiddle(const PlanView& pv, u64 N, u32 b0, u64 g_tile, u32 o,
                                                       u32 c, int bit, int u, int logr_perm_top) {
    constexpr int lo = G::lo(r);
    if (LOWPASS && lo == 0 && bit <= logr_perm_top) {
      const u64 tg = (g_tile >> LOGR) + o;
      return pv.twp[(N >> (bit + 1)) + (u64)u * (N >> LOGR) + tg];
    }
    const u64 g_base = g_tile + ((u64)rho<r>(o, 0) << b0) + c;
    return pv.tw[((N + g_base) >> (b0 + bit + 1)) + (u64)u];
  }

  template <int r>
  static constexpr int nblocks(int s) {
    return ((R >> ((FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s)) - G::lo(r) + 1)) + TB - 1) / TB;
  }
  template <int r>
  static constexpr int first_step(int s) {
    int n = 0;
    for (int i = 0; i < s; ++i) n += nblocks<r>(i);
    return n;
  }

  template <int r, bool LASTPASS, int PTOP>
  __device__ static __forceinline__ void stages(u64 (&x)[R], const PlanView& pv, u64 N, u32 b0, u64 g_tile, u32 o,
                                                u32 c) {
    constexpr int lo = G::lo(r);
    constexpr int NS = G::nst(r);
    ulonglong2 buf[2][TB];
    auto load_block = [&](ulonglong2 (&dst)[TB], int s, int blk) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int p = bit - lo;
      const int n = R >> (p + 1);
      const bool fused_last = !FWD && LASTPASS && bit == LOGT - 1;
      if (fused_last) return;
#pragma unroll
      for (int i = 0; i < TB; ++i)
        if (blk * TB + i < n) dst[i] = twiddle<r>(pv, N, b0, g_tile, o, c, bit, blk * TB + i, PTOP);
    };
    load_block(buf[0], 0, 0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int p = bit - lo;
      const int n = R >> (p + 1);
      const int nb = (n + TB - 1) / TB;
      const bool fused_last = !FWD && LASTPASS && bit == LOGT - 1;
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
            if (FWD) bfly_fwd<HAND>(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq, pv.nq2);
            else if (fused_last) bfly_inv_last<HAND>(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q2, pv.nq);
            else bfly_inv<HAND>(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq, pv.nq2);
          }
        }
        stage_fence();
      }
    }
  }

  template <int r, bool LASTPASS, int PTOP>
  __device__ static __forceinline__ void run(u64* lds, u64 (&x)[R], const PlanView& pv, u64 N, u32 b0, u64 g_tile,
                                             u32 o, u32 c) {
    stages<r, LASTPASS, PTOP>(x, pv, N, b0, g_tile, o, c);
    if constexpr (r + 1 < G::NR) {
      const u32 bo = row_base<r>(o), bi = row_base<r + 1>(o);
      shuffle(lds, x, c, [&](int j) { return bo + row_off<r>(j); }, [&](int j) { return bi + row_off<r + 1>(j); });
      run<r + 1, LASTPASS, PTOP>(lds, x, pv, N, b0, g_tile, o, c);
    }
  }
};

// Runs one tile of one pass.  in/out/mul point at the limb's first coefficient;
// `tile` selects the tile inside the limb; b0 = lowest index bit of the pass;
// t = the thread's index among the tile's threads; with active false nothing is
// stored.
template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int MODE, bool LASTPASS, int PTOP, bool HAND = true>
__device__ __forceinline__ void tile_body(const PlanView& pv, u32 logN, u32 b0, u32 tile, const u64* in_item,
                                          u64* out_item, const u64* mul, u64* lds, bool nt_load, u32 t,
                                          bool active) {
  using K = TileNtt<FWD, LOGT, LOGR, LOGC, LOGH, HAND>;
  constexpr int R = K::R;
  constexpr int C = K::C;
  constexpr int NT = K::NT;
  constexpr int RL = K::G::NR - 1;
  constexpr bool direct_in = !K::LOWPASS || K::G::lo(0) >= 4 || NT < 16;
  constexpr bool direct_out = !K::LOWPASS || K::G::lo(RL) >= 4 || NT < 16;
  const u64 N = 1ull << logN;
  u64 g_tile;
  if constexpr (!K::LOWPASS) {
    const u32 ncg = (1u << b0) >> LOGC;
    const u32 cg = tile % ncg, hb = tile / ncg;
    g_tile = ((u64)hb << (b0 + LOGT)) | ((u64)cg << LOGC);
  } else {
    g_tile = (u64)tile << (LOGT + LOGH);
  }
  const u32 c = t & (C - 1);
  const u32 o = t >> LOGC;
  const u64* in = in_item + g_tile;
  u64* out = out_item + g_tile;

  u64 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &in[((u64)K::template rho<0>(o, j) << b0) + c];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64* p = &in[(u32)j * NT + t];
      x[j] = nt_load ? __builtin_nontemporal_load(p) : *p;
    }
    const u32 bi = K::template row_base<0>(o);
    K::shuffle(lds, x, 0, [&](int j) { return K::lin_row(t, j); }, [&](int j) { return bi + K::template row_off<0>(j); });
  }

  K::template run<0, LASTPASS, PTOP>(lds, x, pv, N, b0, g_tile, o, c);

  if constexpr (!direct_out) {
    const u32 bo = K::template row_base<RL>(o);
    K::shuffle(lds, x, 0, [&](int j) { return bo + K::template row_off<RL>(j); }, [&](int j) { return K::lin_row(t, j); });
  }
  if (!active) return;                            // past the last barrier: nothing left but the stores
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u64 i = direct_out ? (((u64)K::template rho<RL>(o, j) << b0) + c) : (u64)((u32)j * NT + t);
    out[i] = LASTPASS ? finish_item<FWD, MODE>(x[j], mul, g_tile + i, pv) : x[j];
    if ((j & 7) == 7) stage_fence();
  }
}

}  // namespace nttamd
