// Two-pass negacyclic NTT for 2^15 <= N <= 2^17.
//
// The forward transform is Algorithm 2 (Cooley-Tukey, merged psi twiddles,
// bit-reversed output) with the Harvey butterfly of Algorithm 4; the inverse is
// Algorithm 3 (Gentleman-Sande) with the butterfly of Algorithm 5 and the
// scaling by N^{-1} fused into its last stage.  Every butterfly performs
// exactly the arithmetic of Algorithm 4 / 5; only the order in which
// independent butterflies run differs from the radix-2 loops.
//
// Decomposition.  The stage that pairs indices differing in bit b uses the
// twiddle with table index (N + g) >> (b + 1), g the lower index (this is
// psi_rev[m + i] of Algorithm 2 and psi^{-1}_rev[h + i] of Algorithm 3).  A
// pass handles the stages of a contiguous range of index bits
// [b0, b0 + LOGT): the elements that share all other bits form independent
// sub-transforms of size 2^LOGT with stride 2^b0 (the split N = N1 N2 of
// Section 2.2).  The "high" pass (b0 > 0) gives each workgroup a tile of
// C = 2^LOGC adjacent columns, lanes running along the columns so every HBM
// access covers C contiguous words; the "low" pass (b0 = 0) gives it H = 2^LOGH
// adjacent contiguous blocks.  Forward passes run high then low, inverse
// passes low then high.
//
// Inside a tile each thread holds R = 2^LOGR coefficients and runs up to
// LOGR stages per round in registers; rounds exchange through LDS (rows
// padded by one word every R rows).  As in the single-pass kernel, twiddles
// are prefetched one block ahead, the low pass's finest stages read the
// plan's transposed sub-tables, rounds whose threads own consecutive
// coefficients go through LDS to and from HBM, and coefficient loads are
// non-temporal.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"

namespace nttamd {

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH>
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
            if (FWD) harvey_fwd(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq);
            else if (fused_last) harvey_inv_last(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q2, pv.nq);
            else harvey_inv(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq);
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

// LASTPASS: this pass produces the transform's output (output mode MODE and,
// for the inverse, the fused N^{-1} stage); PTOP: highest stage bit read from
// the transposed sub-tables in the low pass (-1: none).
template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int MINW, int MODE, bool LASTPASS, int PTOP>
__global__ void __launch_bounds__((1 << (LOGT + LOGH + LOGC)) >> LOGR, MINW) ntt_tile_kernel(const PassArgs a) {
  using K = TileNtt<FWD, LOGT, LOGR, LOGC, LOGH>;
  constexpr int R = K::R;
  constexpr int C = K::C;
  constexpr int NT = K::NT;
  constexpr int RL = K::G::NR - 1;
  constexpr bool direct_in = !K::LOWPASS || K::G::lo(0) >= 4 || NT < 16;
  constexpr bool direct_out = !K::LOWPASS || K::G::lo(RL) >= 4 || NT < 16;
  __shared__ u64 lds[K::LDSW];

  const u32 item = a.item0 + blockIdx.y;
  const u32 logN = a.logN;
  const u64 N = 1ull << logN;
  const PlanView pv = load_plan(a.plan[item % a.num_limbs], FWD, N);
  const u32 b0 = a.b0;
  const u64 base = (u64)item << logN;

  u64 g_tile;
  if constexpr (!K::LOWPASS) {
    const u32 ncg = (1u << b0) >> LOGC;
    const u32 cg = blockIdx.x % ncg, hb = blockIdx.x / ncg;
    g_tile = ((u64)hb << (b0 + LOGT)) | ((u64)cg << LOGC);
  } else {
    g_tile = (u64)blockIdx.x << (LOGT + LOGH);
  }
  const u32 t = threadIdx.x;
  const u32 c = t & (C - 1);
  const u32 o = t >> LOGC;
  const u64* in = a.in + base + g_tile;
  u64* out = a.out + base + g_tile;

  u64 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[((u64)K::template rho<0>(o, j) << b0) + c]);
  } else {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[(u32)j * NT + t]);
    const u32 bi = K::template row_base<0>(o);
    K::shuffle(lds, x, 0, [&](int j) { return K::lin_row(t, j); }, [&](int j) { return bi + K::template row_off<0>(j); });
  }

  K::template run<0, LASTPASS, PTOP>(lds, x, pv, N, b0, g_tile, o, c);

  if constexpr (!direct_out) {
    const u32 bo = K::template row_base<RL>(o);
    K::shuffle(lds, x, 0, [&](int j) { return bo + K::template row_off<RL>(j); }, [&](int j) { return K::lin_row(t, j); });
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u64 i = direct_out ? (((u64)K::template rho<RL>(o, j) << b0) + c) : (u64)((u32)j * NT + t);
    const u64 v = LASTPASS ? finish_mode<FWD, MODE>(x[j], base + g_tile + i, a, pv) : x[j];
    out[i] = v;
    if ((j & 7) == 7) stage_fence();
  }
}

// ---- schedules ---------------------------------------------------------------

typedef void (*PassKernel)(const PassArgs);

// Variants of the high (strided) pass: coefficients per thread, 2^3 or 2^4.
constexpr int kHiVariants = 2;
static int hi_logr(int variant) { return variant == 0 ? 4 : 3; }

template <bool FWD, int LOGN, int MODE, bool LAST>
static PassKernel pick_hi(int variant) {
  constexpr int LT = mp_logt_hi(LOGN);
  constexpr int MW = LT >= 9 ? 2 : 4;
  if (variant == 0) return ntt_tile_kernel<FWD, LT, 4, 4, 0, MW, MODE, LAST, -1>;
  return ntt_tile_kernel<FWD, LT, 3, 4, 0, MW, MODE, LAST, -1>;
}
template <bool FWD, int LOGN, int MODE, bool LAST>
static PassKernel pick_lo() {
  constexpr int LT = mp_logt_lo(LOGN);
  constexpr int LH = 12 - LT;                          // 4096-coefficient tiles
  return ntt_tile_kernel<FWD, LT, kMpLogrLo, 0, LH, 4, MODE, LAST, mp_perm_top(FWD, LOGN)>;
}

template <int LOGN>
static PassKernel pick_pass(bool fwd, bool hi, u32 flags, int variant) {
  if (fwd) {
    if (hi) return pick_hi<true, LOGN, kOutLazy, false>(variant);           // forward: high pass first
    if (flags & kFlagMul) return pick_lo<true, LOGN, kOutMul, true>();
    if (flags & kFlagCanon) return pick_lo<true, LOGN, kOutCanon, true>();
    return pick_lo<true, LOGN, kOutLazy, true>();
  }
  if (!hi) return pick_lo<false, LOGN, kOutLazy, false>();                   // inverse: low pass first
  if (flags & kFlagAcc) return pick_hi<false, LOGN, kOutAcc, true>(variant);
  if (flags & kFlagCanon) return pick_hi<false, LOGN, kOutCanon, true>(variant);
  return pick_hi<false, LOGN, kOutLazy, true>(variant);
}

static PassKernel pick_pass_n(int logN, bool fwd, bool hi, u32 flags, int variant) {
  switch (logN) {
    case 15: return pick_pass<15>(fwd, hi, flags, variant);
    case 16: return pick_pass<16>(fwd, hi, flags, variant);
    case 17: return pick_pass<17>(fwd, hi, flags, variant);
    default: return nullptr;
  }
}

// Number of passes the schedule for 2^logN uses (1 = the whole transform on chip).
int pass_count(int logN) { return logN <= kMaxOnchipLog ? 1 : 2; }

// High-pass variant per (direction, logN, batch size); set by the autotuner.
static int g_hi_variant[2][NTT_MAX_LOG_DEGREE + 1][2];
static int batch_bucket(uint64_t items) { return items <= 64 ? 0 : 1; }

void set_hi_variant(bool fwd, int logN, uint64_t items, int variant) {
  g_hi_variant[fwd ? 1 : 0][logN][batch_bucket(items)] = variant;
}
int get_hi_variant(bool fwd, int logN, uint64_t items) { return g_hi_variant[fwd ? 1 : 0][logN][batch_bucket(items)]; }
int hi_variant_count() { return kHiVariants; }

static ntt_status launch_passes(const NttLaunch& l, bool fwd, int force_variant) {
  const ntt_plan* p0 = l.plans[0];
  const int logN = p0->logN;
  if (l.num_limbs == 0 || l.num_limbs > (uint32_t)kMaxPlansPerLaunch) return NTT_EINVAL_COUNT;
  PassArgs a{};
  for (uint32_t i = 0; i < l.num_limbs; ++i) a.plan[i] = l.plans[i]->dev;
  a.num_limbs = l.num_limbs;
  a.logN = (u32)logN;
  a.mul = l.mul_into;
  const uint64_t items = l.num_polys * l.num_limbs;
  u32 last_flags = kFlagLast;
  if (l.out_f == 1) last_flags |= kFlagCanon;
  if (fwd && l.mul_into) last_flags |= kFlagMul;
  if (!fwd && l.mul_into) last_flags |= kFlagAcc;
  if (logN <= kMaxOnchipLog) {
    a.in = l.in;
    a.out = l.out;
    a.b0 = 0;
    a.flags = last_flags;
    ntt_status st = launch_onchip(a, items, fwd, l.stream);
    if (st) return st;
    return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
  }
  if (logN > NTT_MAX_LOG_DEGREE) return NTT_EINVAL_DEGREE;
  const int variant = force_variant >= 0 ? force_variant : get_hi_variant(fwd, logN, items);
  const int lt_lo = mp_logt_lo(logN), lt_hi = mp_logt_hi(logN);
  uint64_t* mid = l.tmp ? l.tmp : l.out;
  const uint64_t kMaxY = 65535;
  for (int step = 0; step < 2; ++step) {
    const bool hi = fwd ? (step == 0) : (step == 1);
    const bool last = step == 1;
    a.in = step == 0 ? l.in : mid;
    a.out = last ? l.out : mid;
    a.flags = last ? last_flags : 0u;
    PassKernel k = pick_pass_n(logN, fwd, hi, a.flags, variant);
    if (!k) return NTT_EINVAL_DEGREE;
    int nt;
    uint64_t tiles;
    if (hi) {
      a.b0 = (u32)lt_lo;
      const int logr = hi_logr(variant);
      nt = 1 << (lt_hi + 4 - logr);
      tiles = ((1ull << lt_lo) >> 4) * (1ull << (logN - lt_lo - lt_hi));
    } else {
      a.b0 = 0;
      nt = 1 << (12 - kMpLogrLo);
      tiles = 1ull << (logN - 12);
    }
    for (uint64_t it0 = 0; it0 < items; it0 += kMaxY) {
      const uint64_t ny = (items - it0) < kMaxY ? (items - it0) : kMaxY;
      a.item0 = (u32)it0;
      hipLaunchKernelGGL(k, dim3((unsigned)tiles, (unsigned)ny), dim3(nt), 0, l.stream, a);
    }
  }
  if (hipGetLastError() != hipSuccess) return NTT_EDEVICE;
  return NTT_OK;
}

ntt_status launch_forward(const NttLaunch& l) { return launch_passes(l, true, -1); }
ntt_status launch_inverse(const NttLaunch& l) { return launch_passes(l, false, -1); }
ntt_status launch_variant(const NttLaunch& l, bool fwd, int variant) { return launch_passes(l, fwd, variant); }

}  // namespace nttamd
