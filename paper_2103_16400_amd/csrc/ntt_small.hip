// Single-pass negacyclic NTT at word size beta = 2^32, for moduli below 2^30
// and N <= 2^15: the small-prime specialisation of the transforms, the
// counterpart of the paper's size-specialised IFMA52 path (Algorithms 6 and 7
// run Algorithms 4 and 5 at beta = 2^52 for moduli below 2^50).
//
// Algorithms 4 and 5 are exact at any word size beta with 4q <= beta: the
// Shoup quotient Q = floor(W' X / beta) with W' = floor(W beta / q) leaves
// W X - Q q in [0, 2q).  At beta = 2^32 every product is one native 32-bit
// multiply (mul_lo or mul_hi) instead of the four to six partial products of
// a 64-bit word, and every coefficient is 4 bytes instead of 8.
//   - W' at beta = 2^32 is the high word of the stored 64-bit companion:
//     floor(floor(W 2^64 / q) / 2^32) = floor(W 2^32 / q); the plan tables of
//     the 64-bit path serve unchanged.
//   - x mod 2q for x < 4q is min(x, x - 2q) in 32-bit arithmetic: when x < 2q
//     the difference wraps above 2^32 - 2q > 4q.  The same holds for every
//     conditional subtraction here, because 4q < 2^32.
//
// Schedule, LDS layout and twiddle order are those of the 64-bit single-pass
// kernel (ntt_onchip.h): each thread keeps 2^LOGR coefficients in registers
// and runs up to LOGR stages per round, rounds exchange through LDS (one
// 32-bit word per coefficient, rows padded every 2^LOGR words), the round in
// which a thread owns consecutive coefficients reads the plan's transposed
// sub-tables, and HBM is read and written once per coefficient.  At 4 bytes
// per coefficient a limb of N = 2^15 (128 KiB) still fits the LDS of one
// workgroup (1024 threads, one workgroup per CU); the plan's transposed copy
// at that size is laid out for the two-pass kernels, so that size reads the
// natural tables throughout.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "ntt_common.h"
#include "small32.h"
#include "tile32.h"

namespace nttamd {

template <bool FWD, int LOGN, int LOGR>
struct OnChip32 {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = 1 << LOGR;
  static constexpr int NT = N >> LOGR;
  static constexpr int LDSW = N + (N >> LOGR);
  // the transposed sub-tables are laid out for onchip_logr(LOGN) coefficients per thread, for N <= 2^14
  static constexpr int PERM_TOP =
      LOGN <= kMaxOnchipLog && LOGR == onchip_logr(LOGN) ? onchip_perm_top(FWD, LOGN) : -1;
  static constexpr int TB = 2;                    // twiddle pairs per prefetch block
  using G = Geo<FWD, LOGN, LOGR>;

  template <int r>
  __device__ static __forceinline__ u32 rho(u32 t, int j) {
    constexpr int lo = G::lo(r);
    return ((t >> lo) << (lo + LOGR)) | ((u32)j << lo) | (t & ((1u << lo) - 1u));
  }
  __device__ static __forceinline__ u32 row(u32 r) { return r + (r >> LOGR); }
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
  __device__ static __forceinline__ u32 lin_row(u32 t, int j) {
    if constexpr (LOGN >= 2 * LOGR) return (u32)j * (NT + (NT >> LOGR)) + t + (t >> LOGR);
    else return row((u32)j * NT + t);
  }

  template <typename FO, typename FI>
  __device__ static __forceinline__ void shuffle(u32* lds, u32 (&x)[R], FO row_out, FI row_in) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) lds[row_out(j)] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = lds[row_in(j)];
  }

  // (W, W') at beta = 2^32 of twiddle pair u of the stage on local bit `bit` in round r
  template <int r>
  __device__ static __forceinline__ uint2 twiddle(const View32& v, u32 t, int bit, int u) {
    constexpr int lo = G::lo(r);
    const ulonglong2 p = (lo == 0 && bit <= PERM_TOP) ? v.twp[(N >> (bit + 1)) + (u32)u * NT + t]
                                                      : v.tw[((N + rho<r>(t, 0)) >> (bit + 1)) + (u32)u];
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

  template <int r>
  __device__ static __forceinline__ void stages(u32 (&x)[R], u32 t, const View32& v) {
    constexpr int lo = G::lo(r);
    constexpr int NS = G::nst(r);
    uint2 buf[2][TB];
    auto load_block = [&](uint2 (&dst)[TB], int s, int blk) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);
      const int n = R >> (bit - lo + 1);
      if (!FWD && bit == LOGN - 1) return;        // fused last stage: constants from the header
#pragma unroll
      for (int i = 0; i < TB; ++i)
        if (blk * TB + i < n) dst[i] = twiddle<r>(v, t, bit, blk * TB + i);
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

  template <int r>
  __device__ static __forceinline__ void run(u32* lds, u32 (&x)[R], u32 t, const View32& v) {
    stages<r>(x, t, v);
    if constexpr (r + 1 < G::NR) {
      const u32 bo = row_base<r>(t), bi = row_base<r + 1>(t);
      shuffle(lds, x, [&](int j) { return bo + row_off<r>(j); }, [&](int j) { return bi + row_off<r + 1>(j); });
      run<r + 1>(lds, x, t, v);
    }
  }

  // Coefficients of this thread for round 0, from HBM (through LDS where the
  // round's layout would not coalesce).
  __device__ static __forceinline__ void load(u32* lds, u32 (&x)[R], const u32* in, u32 t) {
    constexpr bool direct = G::lo(0) >= 4 || LOGN - LOGR < 4;
    if constexpr (direct) {
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[rho<0>(t, j)]);
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = __builtin_nontemporal_load(&in[(u32)j * NT + t]);
      const u32 bi = row_base<0>(t);
      shuffle(lds, x, [&](int j) { return lin_row(t, j); }, [&](int j) { return bi + row_off<0>(j); });
    }
  }

  // Writes the last round's coefficients with output step MODE.
  template <int MODE>
  __device__ static __forceinline__ void store(u32* lds, u32 (&x)[R], u32* out, const u32* mul, u32 t,
                                               const View32& v) {
    constexpr int RL = G::NR - 1;
    constexpr bool direct = G::lo(RL) >= 4 || LOGN - LOGR < 4;
    if constexpr (!direct) {
      const u32 bo = row_base<RL>(t);
      shuffle(lds, x, [&](int j) { return bo + row_off<RL>(j); }, [&](int j) { return lin_row(t, j); });
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u32 i = direct ? rho<RL>(t, j) : (u32)j * NT + t;
      out[i] = finish32<FWD, MODE>(x[j], mul, i, v);
    }
  }
};

struct Pass32Args {
  u32* out;
  const u32* in;
  const u32* mul;                          // product: the transformed multiplier; accumulate: acc (== out)
  const u64* plan[kMaxPlansPerLaunch];     // item y uses plan[y % num_limbs]
  u32 num_limbs;
  u32 item0;
};

// One limb per workgroup: forward or inverse transform with output step MODE.
template <bool FWD, int LOGN, int MODE>
__global__ void __launch_bounds__(1 << (LOGN - onchip_logr(LOGN))) ntt32_kernel(const Pass32Args a) {
  constexpr int LOGR = onchip_logr(LOGN);
  using K = OnChip32<FWD, LOGN, LOGR>;
  __shared__ u32 lds[K::LDSW];
  const u32 item = a.item0 + blockIdx.x;
  const View32 v = view32(a.plan[item % a.num_limbs], FWD, (u64)K::N);
  const u64 base = (u64)item << LOGN;
  const u32 t = threadIdx.x;
  u32 x[K::R];
  K::load(lds, x, a.in + base, t);
  K::template run<0>(lds, x, t, v);
  K::template store<MODE>(lds, x, a.out + base, a.mul ? a.mul + base : nullptr, t, v);
}

// The negacyclic product of one limb kept on chip: forward(b) in [0, 4q),
// Algorithm 8 multiply by m (the transformed a, in [0, 4q)), inverse, then the
// canonical result or the add into out (MODE).  The forward's last round and
// the inverse's first round give thread t the same consecutive coefficients,
// so the multiply and the start of the inverse run in registers.
template <int LOGN, int MODE>
__global__ void __launch_bounds__(1 << (LOGN - onchip_logr(LOGN))) ntt32_product_kernel(const Pass32Args a) {
  constexpr int LOGR = onchip_logr(LOGN);
  using KF = OnChip32<true, LOGN, LOGR>;
  using KI = OnChip32<false, LOGN, LOGR>;
  static_assert(KF::G::lo(KF::G::NR - 1) == 0 && KI::G::lo(0) == 0, "forward output and inverse input layouts");
  __shared__ u32 lds[KF::LDSW];
  const u32 item = a.item0 + blockIdx.x;
  const u64* plan = a.plan[item % a.num_limbs];
  const View32 vf = view32(plan, true, (u64)KF::N);
  const View32 vi = view32(plan, false, (u64)KF::N);
  const u64 base = (u64)item << LOGN;
  const u32 t = threadIdx.x;
  u32 x[KF::R];
  KF::load(lds, x, a.in + base, t);
  KF::template run<0>(lds, x, t, vf);
  const u32* mt = a.mul + base + ((u64)t << LOGR);  // rho of the forward's last round: t R + j
#pragma unroll
  for (int j = 0; j < KF::R; ++j) x[j] = mulmod32_f4(x[j], mt[j], vf);
  __syncthreads();                                  // the forward's last LDS reads precede the inverse's writes
  KI::template run<0>(lds, x, t, vi);
  KI::template store<MODE>(lds, x, a.out + base, a.out + base, t, vi);
}

typedef void (*Kernel32)(const Pass32Args);

template <bool FWD, int MODE>
static Kernel32 pick32(int logN) {
  switch (logN) {
    case 1: return ntt32_kernel<FWD, 1, MODE>;
    case 2: return ntt32_kernel<FWD, 2, MODE>;
    case 3: return ntt32_kernel<FWD, 3, MODE>;
    case 4: return ntt32_kernel<FWD, 4, MODE>;
    case 5: return ntt32_kernel<FWD, 5, MODE>;
    case 6: return ntt32_kernel<FWD, 6, MODE>;
    case 7: return ntt32_kernel<FWD, 7, MODE>;
    case 8: return ntt32_kernel<FWD, 8, MODE>;
    case 9: return ntt32_kernel<FWD, 9, MODE>;
    case 10: return ntt32_kernel<FWD, 10, MODE>;
    case 11: return ntt32_kernel<FWD, 11, MODE>;
    case 12: return ntt32_kernel<FWD, 12, MODE>;
    case 13: return ntt32_kernel<FWD, 13, MODE>;
    case 14: return ntt32_kernel<FWD, 14, MODE>;
    case 15: return ntt32_kernel<FWD, 15, MODE>;
    default: return nullptr;
  }
}

template <int MODE>
static Kernel32 pick32_product(int logN) {
  switch (logN) {
    case 1: return ntt32_product_kernel<1, MODE>;
    case 2: return ntt32_product_kernel<2, MODE>;
    case 3: return ntt32_product_kernel<3, MODE>;
    case 4: return ntt32_product_kernel<4, MODE>;
    case 5: return ntt32_product_kernel<5, MODE>;
    case 6: return ntt32_product_kernel<6, MODE>;
    case 7: return ntt32_product_kernel<7, MODE>;
    case 8: return ntt32_product_kernel<8, MODE>;
    case 9: return ntt32_product_kernel<9, MODE>;
    case 10: return ntt32_product_kernel<10, MODE>;
    case 11: return ntt32_product_kernel<11, MODE>;
    case 12: return ntt32_product_kernel<12, MODE>;
    case 13: return ntt32_product_kernel<13, MODE>;
    case 14: return ntt32_product_kernel<14, MODE>;
    case 15: return ntt32_product_kernel<15, MODE>;
    default: return nullptr;
  }
}

// ---- two passes (N = 2^16, 2^17) -----------------------------------------------
// The split N = N1 N2 of the 64-bit two-pass kernels: a high (strided) pass over
// tiles of 16 adjacent columns with 8 coefficients per thread, and a low pass
// over 4096 contiguous coefficients with 16 per thread, which reads the plan's
// transposed sub-tables (laid out for that shape).  The forward runs high then
// low, the inverse low then high (its fused N^{-1} stage is the high pass's
// top bit).

struct Tile32Args {
  u32* out;
  const u32* in;
  const u32* mul;                          // kOutMul: multiplier; kOutAcc: accumulator (== out)
  const u64* plan[kMaxPlansPerLaunch];     // item y uses plan[y % num_limbs]
  u32 num_limbs;
  u32 logN;
  u32 b0;                                  // lowest index bit of this pass
  u32 item0;
};

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int MODE, bool LASTPASS, int PTOP>
__global__ void __launch_bounds__((1 << (LOGT + LOGH + LOGC)) >> LOGR) ntt32_tile_kernel(const Tile32Args a) {
  using K = Tile32<FWD, LOGT, LOGR, LOGC, LOGH>;
  __shared__ u32 lds[K::LDSW];
  // every tile of an item on one XCD (linear workgroup id mod 8) when the item count allows
  u32 yi = blockIdx.y, tile = blockIdx.x;
  if ((gridDim.y & 7u) == 0) {
    const u32 lin = blockIdx.x + blockIdx.y * gridDim.x;
    const u32 k = lin >> 3;
    yi = (lin & 7u) + 8u * (k / gridDim.x);
    tile = k % gridDim.x;
  }
  const u32 item = a.item0 + yi;
  const View32 v = view32(a.plan[item % a.num_limbs], FWD, 1ull << a.logN);
  const u64 base = (u64)item << a.logN;
  tile32_body<FWD, LOGT, LOGR, LOGC, LOGH, MODE, LASTPASS, PTOP>(v, a.logN, a.b0, tile, a.in + base, a.out + base,
                                                                a.mul ? a.mul + base : nullptr, lds);
}

typedef void (*Tile32Kernel)(const Tile32Args);

template <int LOGN>
struct TwoPass32 {
  static constexpr int LT_LO = mp_logt_lo(LOGN), LT_HI = LOGN - LT_LO;
  static constexpr int LH = 12 - LT_LO;               // low-pass tiles of 4096 coefficients
  template <bool FWD, int MODE, bool LAST>
  static Tile32Kernel hi() { return ntt32_tile_kernel<FWD, LT_HI, 3, 4, 0, MODE, LAST, -1>; }
  template <bool FWD, int MODE, bool LAST>
  static Tile32Kernel lo() { return ntt32_tile_kernel<FWD, LT_LO, kMpLogrLo, 0, LH, MODE, LAST, mp_perm_top(FWD, LOGN)>; }
  static unsigned hi_threads() { return 1u << (LT_HI + 4 - 3); }
  static unsigned lo_threads() { return 1u << (12 - kMpLogrLo); }
  static unsigned hi_tiles() { return (1u << LT_LO) >> 4; }
  static unsigned lo_tiles() { return 1u << (LOGN - 12); }
};

// One pass over `items` limbs (y of the grid), launched in chunks of at most 65535.
static void pass32(Tile32Kernel k, unsigned tiles, unsigned threads, Tile32Args a, uint64_t items, hipStream_t s) {
  const uint64_t kMaxY = 65535;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxY) {
    const uint64_t ny = (items - it0) < kMaxY ? (items - it0) : kMaxY;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(k, dim3(tiles, (unsigned)ny), dim3(threads), 0, s, a);
  }
}

template <int LOGN>
static ntt_status launch_small_twopass(const Small32Launch& l, Tile32Args a, uint64_t items) {
  using T = TwoPass32<LOGN>;
  const hipStream_t s = l.stream;
  auto fwd_hi = [&](const u32* in, u32* out) {
    Tile32Args h = a;
    h.in = in;
    h.out = out;
    h.mul = nullptr;
    h.b0 = T::LT_LO;
    pass32(T::template hi<true, kOutLazy, false>(), T::hi_tiles(), T::hi_threads(), h, items, s);
  };
  auto fwd_lo = [&](Tile32Kernel k, const u32* in, u32* out, const u32* mul) {
    Tile32Args h = a;
    h.in = in;
    h.out = out;
    h.mul = mul;
    h.b0 = 0;
    pass32(k, T::lo_tiles(), T::lo_threads(), h, items, s);
  };
  auto inv_lo = [&](const u32* in, u32* out) {
    Tile32Args h = a;
    h.in = in;
    h.out = out;
    h.mul = nullptr;
    h.b0 = 0;
    pass32(T::template lo<false, kOutLazy, false>(), T::lo_tiles(), T::lo_threads(), h, items, s);
  };
  auto inv_hi = [&](Tile32Kernel k, const u32* in, u32* out, const u32* mul) {
    Tile32Args h = a;
    h.in = in;
    h.out = out;
    h.mul = mul;
    h.b0 = T::LT_LO;
    pass32(k, T::hi_tiles(), T::hi_threads(), h, items, s);
  };
  switch (l.op) {
    case kSmallForwardLazy:
    case kSmallForwardCanon:
      fwd_hi(l.in, l.out);
      fwd_lo(l.op == kSmallForwardLazy ? T::template lo<true, kOutLazy, true>() : T::template lo<true, kOutCanon, true>(),
             l.out, l.out, nullptr);
      break;
    case kSmallInverseLazy:
    case kSmallInverseCanon:
      inv_lo(l.in, l.out);
      inv_hi(l.op == kSmallInverseLazy ? T::template hi<false, kOutLazy, true>() : T::template hi<false, kOutCanon, true>(),
             l.out, l.out, nullptr);
      break;
    case kSmallProduct:                            // out <- InvNTT(NTT(in) (.) mul), mul = NTT(a) (may be out)
      if (!l.tmp) return NTT_EINVAL_POINTER;
      fwd_hi(l.in, l.tmp);
      fwd_lo(T::template lo<true, kOutMul, true>(), l.tmp, l.out, l.mul);
      inv_lo(l.out, l.out);
      inv_hi(T::template hi<false, kOutCanon, true>(), l.out, l.out, nullptr);
      break;
    case kSmallProductAcc:                         // out += InvNTT(NTT(in) (.) mul)
      if (!l.tmp) return NTT_EINVAL_POINTER;
      fwd_hi(l.in, l.tmp);
      fwd_lo(T::template lo<true, kOutMul, true>(), l.tmp, l.tmp, l.mul);
      inv_lo(l.tmp, l.tmp);
      inv_hi(T::template hi<false, kOutAcc, true>(), l.tmp, l.out, l.out);
      break;
    default:
      return NTT_EINVAL_FACTOR;
  }
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

ntt_status launch_small(const Small32Launch& l) {
  if (l.logN < 1 || l.logN > kMaxSmallLog) return NTT_EINVAL_DEGREE;
  if (l.logN > kMaxSmallOnePassLog) {
    if (l.num_limbs == 0 || l.num_limbs > (uint32_t)kMaxPlansPerLaunch) return NTT_EINVAL_COUNT;
    Tile32Args a{};
    for (uint32_t i = 0; i < l.num_limbs; ++i) a.plan[i] = l.plans[i]->dev;
    a.num_limbs = l.num_limbs;
    a.logN = (u32)l.logN;
    const uint64_t items = l.num_polys * l.num_limbs;
    return l.logN == 16 ? launch_small_twopass<16>(l, a, items) : launch_small_twopass<17>(l, a, items);
  }
  if (l.num_limbs == 0 || l.num_limbs > (uint32_t)kMaxPlansPerLaunch) return NTT_EINVAL_COUNT;
  Kernel32 k = nullptr;
  switch (l.op) {
    case kSmallForwardLazy: k = pick32<true, kOutLazy>(l.logN); break;
    case kSmallForwardCanon: k = pick32<true, kOutCanon>(l.logN); break;
    case kSmallInverseLazy: k = pick32<false, kOutLazy>(l.logN); break;
    case kSmallInverseCanon: k = pick32<false, kOutCanon>(l.logN); break;
    case kSmallProduct: k = pick32_product<kOutCanon>(l.logN); break;
    case kSmallProductAcc: k = pick32_product<kOutAcc>(l.logN); break;
    default: return NTT_EINVAL_FACTOR;
  }
  if (!k) return NTT_EINVAL_DEGREE;
  Pass32Args a{};
  a.out = l.out;
  a.in = l.in;
  a.mul = l.mul;
  for (uint32_t i = 0; i < l.num_limbs; ++i) a.plan[i] = l.plans[i]->dev;
  a.num_limbs = l.num_limbs;
  const uint64_t items = l.num_polys * l.num_limbs;
  const unsigned threads = 1u << (l.logN - onchip_logr(l.logN));
  const uint64_t kMaxX = 1u << 30;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxX) {
    const uint64_t nx = (items - it0) < kMaxX ? (items - it0) : kMaxX;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(k, dim3((unsigned)nx), dim3(threads), 0, l.stream, a);
  }
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

}  // namespace nttamd
