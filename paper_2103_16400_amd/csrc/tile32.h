// One tile of a two-pass transform at word size beta = 2^32 (moduli below
// 2^30, N = 2^16 and 2^17): the Cooley-Tukey split N = N1 N2 of Section 2.2
// with the butterflies of Algorithms 4 and 5 at beta = 2^32 (ntt_small.hip).
// Tile geometry, twiddle indexing and LDS layout are those of the 64-bit tile
// (ntt_tile.h); only the word, the butterflies and the output step differ.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ntt_common.h"
#include "small32.h"

namespace nttamd {

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH>
struct Tile32 {
  static constexpr int R = 1 << LOGR;
  static constexpr int C = 1 << LOGC;
  static constexpr int RB = LOGT + LOGH;              // row bits of the tile (block bits on top)
  static constexpr int ROWS = 1 << RB;
  static constexpr int NT = (ROWS * C) >> LOGR;        // threads
  static constexpr int LDSW = (ROWS + (ROWS >> LOGR)) * C;
  static constexpr int TB = 2;                         // twiddle pairs per prefetch block
  static constexpr bool LOWPASS = LOGC == 0;
  using G = Geo<FWD, LOGT, LOGR>;

  template <int r>
  __device__ static __forceinline__ u32 rho(u32 o, int j) {
    constexpr int lo = G::lo(r);
    return ((o >> lo) << (lo + LOGR)) | ((u32)j << lo) | (o & ((1u << lo) - 1u));
  }
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
  __device__ static __forceinline__ u32 lin_row(u32 t, int j) {
    if constexpr (RB >= 2 * LOGR) return (u32)j * (NT + (NT >> LOGR)) + t + (t >> LOGR);
    else return prow((u32)j * NT + t);
  }

  template <typename FO, typename FI>
  __device__ static __forceinline__ void shuffle(u32* lds, u32 (&x)[R], u32 c, FO row_out, FI row_in) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) lds[row_out(j) * C + c] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = lds[row_in(j) * C + c];
  }

  // (W, W') at beta = 2^32 of twiddle pair u of the stage on tile bit `bit`
  template <int r>
  __device__ static __forceinline__ uint2 twiddle(const View32& v, u64 N, u32 b0, u64 g_tile, u32 o, u32 c, int bit,
                                                  int u, int perm_top) {
    constexpr int lo = G::lo(r);
    ulonglong2 p;
    if (LOWPASS && lo == 0 && bit <= perm_top) {
      const u64 tg = (g_tile >> LOGR) + o;
      p = v.twp[(N >> (bit + 1)) + (u64)u * (N >> LOGR) + tg];
    } else {
      const u64 g_base = g_tile + ((u64)rho<r>(o, 0) << b0) + c;
      p = v.tw[((N + g_base) >> (b0 + bit + 1)) + (u64)u];
    }
    return make_uint2((u32)p.x, (u32)(p.y >> 32));
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
  __device__ static __forceinline__ void stages(u32 (&x)[R], const View32& v, u64 N, u32 b0, u64 g_tile, u32 o,
                                                u32 c) {
    constexpr int lo = G::lo(r);
    constexpr int NS = G::nst(r);
    uint2 buf[2][TB];
    auto load_block = [&](uint2 (&dst)[TB], int s, int blk) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int n = R >> (bit - lo + 1);
      if (!FWD && LASTPASS && bit == LOGT - 1) return;    // fused last stage: constants from the header
#pragma unroll
      for (int i = 0; i < TB; ++i)
        if (blk * TB + i < n) dst[i] = twiddle<r>(v, N, b0, g_tile, o, c, bit, blk * TB + i, PTOP);
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
        uint2 (&cur)[TB] = buf[step & 1];
        uint2 (&nxt)[TB] = buf[(step + 1) & 1];
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
            if (FWD) fwd_bfly32(x[j], x[j2], cur[i].x, cur[i].y, v.q, v.q2);
            else if (fused_last) inv_last32(x[j], x[j2], v);
            else inv_bfly32(x[j], x[j2], cur[i].x, cur[i].y, v.q, v.q2);
          }
        }
        stage_fence();
      }
    }
  }

  template <int r, bool LASTPASS, int PTOP>
  __device__ static __forceinline__ void run(u32* lds, u32 (&x)[R], const View32& v, u64 N, u32 b0, u64 g_tile,
                                             u32 o, u32 c) {
    stages<r, LASTPASS, PTOP>(x, v, N, b0, g_tile, o, c);
    if constexpr (r + 1 < G::NR) {
      const u32 bo = row_base<r>(o), bi = row_base<r + 1>(o);
      shuffle(lds, x, c, [&](int j) { return bo + row_off<r>(j); }, [&](int j) { return bi + row_off<r + 1>(j); });
      run<r + 1, LASTPASS, PTOP>(lds, x, v, N, b0, g_tile, o, c);
    }
  }
};

// One tile of one pass at word size 2^32; in/out/mul point at the limb's first
// coefficient, b0 is the lowest index bit of the pass.
template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int MODE, bool LASTPASS, int PTOP>
__device__ __forceinline__ void tile32_body(const View32& v, u32 logN, u32 b0, u32 tile, const u32* in_item,
                                            u32* out_item, const u32* mul, u32* lds) {
  using K = Tile32<FWD, LOGT, LOGR, LOGC, LOGH>;
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
  const u32 t = threadIdx.x;
  const u32 c = t & (C - 1);
  const u32 o = t >> LOGC;
  const u32* in = in_item + g_tile;
  u32* out = out_item + g_tile;

  u32 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[((u64)K::template rho<0>(o, j) << b0) + c]);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[(u32)j * NT + t]);
    const u32 bi = K::template row_base<0>(o);
    K::shuffle(lds, x, 0, [&](int j) { return K::lin_row(t, j); }, [&](int j) { return bi + K::template row_off<0>(j); });
  }

  K::template run<0, LASTPASS, PTOP>(lds, x, v, N, b0, g_tile, o, c);

  if constexpr (!direct_out) {
    const u32 bo = K::template row_base<RL>(o);
    K::shuffle(lds, x, 0, [&](int j) { return bo + K::template row_off<RL>(j); }, [&](int j) { return K::lin_row(t, j); });
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u64 i = direct_out ? (((u64)K::template rho<RL>(o, j) << b0) + c) : (u64)((u32)j * NT + t);
    out[i] = LASTPASS ? finish32<FWD, MODE>(x[j], mul ? mul + g_tile : nullptr, (u32)i, v) : x[j];
    if ((j & 7) == 7) stage_fence();
  }
}

}  // namespace nttamd
