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

namespace nttamd {

template <bool FWD, int LOGN, int LOGR, bool SPLIT>
struct OnChip {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int NT = N >> LOGR;
  static constexpr int LDSW = N + (N >> LOGR);
  static constexpr int PERM_TOP = onchip_perm_top(FWD, LOGN);
  static constexpr int TB = 2;                      // twiddle pairs per prefetch block
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
            if (FWD) harvey_fwd(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq);
            else if (fused_last) harvey_inv_last(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q2, pv.nq);
            else harvey_inv(x[j], x[j2], cur[i].x, cur[i].y, pv.q2, pv.nq);
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

// MINW: waves per SIMD the register allocation must allow (occupancy target).
template <bool FWD, int LOGN, int LOGR, bool SPLIT, int MINW, int MODE>
__global__ void __launch_bounds__(1 << (LOGN - LOGR), MINW) ntt_onchip_kernel(const PassArgs a) {
  using K = OnChip<FWD, LOGN, LOGR, SPLIT>;
  constexpr int R = K::R;
  constexpr int NT = K::NT;
  constexpr int RL = K::G::NR - 1;
  // rounds whose thread layout is lane-contiguous in memory go straight to HBM
  constexpr bool direct_in = K::G::lo(0) >= 4 || LOGN - LOGR < 4;
  constexpr bool direct_out = K::G::lo(RL) >= 4 || LOGN - LOGR < 4;
  __shared__ typename K::W lds[K::LDSW];

  const u32 item = a.item0 + blockIdx.x;
  const PlanView pv = load_plan(a.plan[item % a.num_limbs], FWD, (u64)K::N);
  const u64 base = (u64)item << LOGN;
  const u64* in = a.in + base;
  u64* out = a.out + base;
  const u32 t = threadIdx.x;

  u64 x[R];
  if constexpr (direct_in) {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[K::template rho<0>(t, j)]);
  } else {
    // coalesced: element j*NT + t, then regrouped through LDS
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[(u32)j * NT + t]);
    const u32 bi = K::template row_base<0>(t);
    K::shuffle(lds, x, [&](int j) { return K::lin_row(t, j); }, [&](int j) { return bi + K::template row_off<0>(j); });
  }

  K::template run<0>(lds, x, t, pv);

  if constexpr (!direct_out) {
    const u32 bo = K::template row_base<RL>(t);
    K::shuffle(lds, x, [&](int j) { return bo + K::template row_off<RL>(j); }, [&](int j) { return K::lin_row(t, j); });
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const u32 i = direct_out ? K::template rho<RL>(t, j) : (u32)j * NT + t;
    out[i] = finish_mode<FWD, MODE>(x[j], base + i, a, pv);
    if ((j & 7) == 7) stage_fence();
  }
}

typedef void (*OnchipKernel)(const PassArgs);

template <bool FWD, int MODE>
static OnchipKernel pick_onchip_mode(int logN) {
  switch (logN) {
    case 1: return ntt_onchip_kernel<FWD, 1, onchip_logr(1), false, 1, MODE>;
    case 2: return ntt_onchip_kernel<FWD, 2, onchip_logr(2), false, 1, MODE>;
    case 3: return ntt_onchip_kernel<FWD, 3, onchip_logr(3), false, 1, MODE>;
    case 4: return ntt_onchip_kernel<FWD, 4, onchip_logr(4), false, 1, MODE>;
    case 5: return ntt_onchip_kernel<FWD, 5, onchip_logr(5), false, 1, MODE>;
    case 6: return ntt_onchip_kernel<FWD, 6, onchip_logr(6), false, 1, MODE>;
    case 7: return ntt_onchip_kernel<FWD, 7, onchip_logr(7), false, 1, MODE>;
    case 8: return ntt_onchip_kernel<FWD, 8, onchip_logr(8), false, 1, MODE>;
    case 9: return ntt_onchip_kernel<FWD, 9, onchip_logr(9), false, 2, MODE>;
    case 10: return ntt_onchip_kernel<FWD, 10, onchip_logr(10), false, 2, MODE>;
    case 11: return ntt_onchip_kernel<FWD, 11, onchip_logr(11), false, 2, MODE>;
    case 12: return ntt_onchip_kernel<FWD, 12, onchip_logr(12), false, 4, MODE>;
    case 13: return ntt_onchip_kernel<FWD, 13, onchip_logr(13), true, 4, MODE>;
    case 14: return ntt_onchip_kernel<FWD, 14, onchip_logr(14), true, 4, MODE>;
    default: return nullptr;
  }
}

static OnchipKernel pick_onchip(bool fwd, int logN, u32 flags) {
  if (fwd) {
    if (flags & kFlagMul) return pick_onchip_mode<true, kOutMul>(logN);
    if (flags & kFlagCanon) return pick_onchip_mode<true, kOutCanon>(logN);
    return pick_onchip_mode<true, kOutLazy>(logN);
  }
  if (flags & kFlagAcc) return pick_onchip_mode<false, kOutAcc>(logN);
  if (flags & kFlagCanon) return pick_onchip_mode<false, kOutCanon>(logN);
  return pick_onchip_mode<false, kOutLazy>(logN);
}

ntt_status launch_onchip(const PassArgs& base_args, uint64_t items, bool fwd, hipStream_t stream) {
  const int logN = (int)base_args.logN;
  OnchipKernel k = pick_onchip(fwd, logN, base_args.flags);
  if (!k) return NTT_EINVAL_DEGREE;
  PassArgs a = base_args;
  const uint64_t kMaxX = 1u << 30;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxX) {
    const uint64_t nx = (items - it0) < kMaxX ? (items - it0) : kMaxX;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(k, dim3((unsigned)nx), dim3(1 << (logN - onchip_logr(logN))), 0, stream, a);
  }
  return NTT_OK;
}

}  // namespace nttamd
