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
// passes low then high.  A three-pass schedule (N = N1 N2 N3) adds a middle
// pass: strided like the high pass, with the bits above its range selecting
// independent blocks of sub-transforms.
//
// Inside a tile each thread holds R = 2^LOGR coefficients and runs up to
// LOGR stages per round in registers; rounds exchange through LDS (rows
// padded by one word every R rows).  As in the single-pass kernel, twiddles
// are prefetched one block ahead, the low pass's finest stages read the
// plan's transposed sub-tables, rounds whose threads own consecutive
// coefficients go through LDS to and from HBM, and coefficient loads are
// non-temporal.
#include <hip/hip_runtime.h>

#include <atomic>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"
#include "ntt_tile.h"

namespace nttamd {

// LASTPASS: this pass produces the transform's output (output mode MODE and,
// for the inverse, the fused N^{-1} stage); PTOP: highest stage bit read from
// the transposed sub-tables in the low pass (-1: none); HAND: false for the
// 64-VGPR schedule (twice the waves per SIMD).
template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int MINW, int MODE, bool LASTPASS, int PTOP,
          bool HAND = true>
__global__ void __launch_bounds__((1 << (LOGT + LOGH + LOGC)) >> LOGR, MINW) ntt_tile_kernel(const PassArgs a) {
  using K = TileNtt<FWD, LOGT, LOGR, LOGC, LOGH, HAND>;
  __shared__ u64 lds[K::LDSW];
  // Workgroups are dispatched to the 8 XCDs in turn (linear id mod 8).  When the
  // item count allows, every tile of an item goes to one XCD, in both passes, so
  // the intermediate the first pass writes is read back through the same L2.
  u32 yi = blockIdx.y, tile = blockIdx.x;
  if ((gridDim.y & 7u) == 0) {
    const u32 lin = blockIdx.x + blockIdx.y * gridDim.x;
    const u32 k = lin >> 3;
    yi = (lin & 7u) + 8u * (k / gridDim.x);
    tile = k % gridDim.x;
  }
  const u32 item = a.item0 + yi;
  const u32 logN = a.logN;
  const PlanView pv = load_plan(a.plan[item % a.num_limbs], FWD, 1ull << logN);
  const u64 base = (u64)item << logN;
  tile_body<FWD, LOGT, LOGR, LOGC, LOGH, MODE, LASTPASS, PTOP, HAND>(pv, logN, a.b0, tile, a.in + base,
                                                                    a.out + base, a.mul ? a.mul + base : nullptr, lds,
                                                                    true, threadIdx.x, true);
}

// ---- schedules ---------------------------------------------------------------

typedef void (*PassKernel)(const PassArgs);

// Schedule variants: (log2 coefficients per thread of the high pass, of the
// low pass, butterflies).  Fewer coefficients per thread means more waves per
// tile, which hides more latency when the batch is small, at the price of more
// LDS rounds.  The low pass reads the plan's transposed sub-tables only with
// 2^kMpLogrLo coefficients per thread (the layout they are built for);
// otherwise it reads the natural table.  Variant 5 holds 4 coefficients per
// thread within 64 VGPRs, so twice as many waves share a CU (more latency
// hidden, at the price of more LDS rounds).  Variants 6 and 7 move the split
// N = N1 N2 (Section 2.2) one index bit either way: the low pass covers one
// bit fewer or one more than the default (reading the natural table), the
// high pass the rest, with 8 columns per tile where its tile would otherwise
// exceed 1024 threads of 8 coefficients.  Variants 8 and 9 halve both passes'
// tiles (half the columns per high-pass tile, half the blocks per low-pass
// tile): twice the workgroups, for batches too small to fill the chip.
// Variant 10 splits N three ways (see three_pass_split) at 8 coefficients per
// thread: one more pass over HBM, fewer stages per pass.
constexpr int kVariants = 11;
struct VariantShape { int hi, lo; bool hand; int dlo; int half; int passes = 2; };
static constexpr VariantShape kVariantShape[kVariants] = {
    {4, 4, true, 0, 0}, {3, 4, true, 0, 0}, {2, 4, true, 0, 0}, {3, 3, true, 0, 0},
    {2, 3, true, 0, 0}, {2, 2, false, 0, 0}, {3, 4, true, -1, 0}, {3, 4, true, 1, 0},
    {3, 4, true, 0, 1}, {2, 4, true, 0, 1}, {3, 3, true, 0, 0, 3}};
// Index bits of the low pass for a variant, and columns per high-pass tile.
static int variant_lt_lo(int logN, int variant) { return mp_logt_lo(logN) + kVariantShape[variant].dlo; }
__host__ __device__ constexpr int hi_logc(int lt_hi) { return lt_hi >= 10 ? 3 : 4; }
// At most 1024 threads per workgroup: 2^(tile bits + column bits - log2 R).
__host__ __device__ constexpr int hi_logr_clamped(int lt_hi, int logr) {
  return lt_hi + hi_logc(lt_hi) - logr > 10 ? lt_hi + hi_logc(lt_hi) - 10 : logr;
}
static int hi_logr(int logN, int variant) {
  return hi_logr_clamped(logN - variant_lt_lo(logN, variant), kVariantShape[variant].hi);
}
static int lo_logr(int variant) { return kVariantShape[variant].lo; }
static int variant_half(int variant) { return kVariantShape[variant].half; }

template <bool FWD, int LOGN, int MODE, bool LAST, int LOGR0, bool HAND = true, int LTLO = mp_logt_lo(LOGN),
          int HALF = 0>
static PassKernel pick_hi_r() {
  constexpr int LT = LOGN - LTLO;
  constexpr int LC = hi_logc(LT) - HALF;
  constexpr int LOGR = hi_logr_clamped(LT, LOGR0);
  // register budget: 64 VGPRs for the 64-VGPR schedule, else 128 (256 for the widest tiles)
  constexpr int MW = !HAND ? 8 : (LOGR >= 4 && LT >= 9 ? 2 : 4);
  return ntt_tile_kernel<FWD, LT, LOGR, LC, 0, MW, MODE, LAST, -1, HAND>;
}
template <bool FWD, int LOGN, int MODE, bool LAST>
static PassKernel pick_hi(int variant) {
  if (kVariantShape[variant].dlo < 0) return pick_hi_r<FWD, LOGN, MODE, LAST, 3, true, mp_logt_lo(LOGN) - 1>();
  if (kVariantShape[variant].dlo > 0) return pick_hi_r<FWD, LOGN, MODE, LAST, 3, true, mp_logt_lo(LOGN) + 1>();
  if (!kVariantShape[variant].hand) return pick_hi_r<FWD, LOGN, MODE, LAST, 2, false>();
  if (kVariantShape[variant].half) {
    if (kVariantShape[variant].hi == 3) return pick_hi_r<FWD, LOGN, MODE, LAST, 3, true, mp_logt_lo(LOGN), 1>();
    return pick_hi_r<FWD, LOGN, MODE, LAST, 2, true, mp_logt_lo(LOGN), 1>();
  }
  switch (kVariantShape[variant].hi) {
    case 4: return pick_hi_r<FWD, LOGN, MODE, LAST, 4>();
    case 3: return pick_hi_r<FWD, LOGN, MODE, LAST, 3>();
    default: return pick_hi_r<FWD, LOGN, MODE, LAST, 2>();
  }
}
template <bool FWD, int LOGN, int MODE, bool LAST>
static PassKernel pick_lo(int variant) {
  constexpr int LT = mp_logt_lo(LOGN);
  constexpr int LH = 12 - LT;                          // 4096-coefficient tiles
  if (kVariantShape[variant].dlo < 0) return ntt_tile_kernel<FWD, LT - 1, kMpLogrLo, 0, LH + 1, 4, MODE, LAST, -1>;
  if (kVariantShape[variant].dlo > 0) return ntt_tile_kernel<FWD, LT + 1, kMpLogrLo, 0, LH - 1, 4, MODE, LAST, -1>;
  if (kVariantShape[variant].half)
    return ntt_tile_kernel<FWD, LT, kMpLogrLo, 0, LH - 1, 4, MODE, LAST, mp_perm_top(FWD, LOGN)>;
  if (lo_logr(variant) == kMpLogrLo) return ntt_tile_kernel<FWD, LT, kMpLogrLo, 0, LH, 4, MODE, LAST, mp_perm_top(FWD, LOGN)>;
  if (!kVariantShape[variant].hand) return ntt_tile_kernel<FWD, LT, 2, 0, LH, 8, MODE, LAST, -1, false>;
  return ntt_tile_kernel<FWD, LT, 3, 0, LH, 4, MODE, LAST, -1>;
}

template <int LOGN>
static PassKernel pick_pass(bool fwd, bool hi, u32 flags, int variant) {
  if (fwd) {
    if (hi) return pick_hi<true, LOGN, kOutLazy, false>(variant);           // forward: high pass first
    if (flags & kFlagMul) return pick_lo<true, LOGN, kOutMul, true>(variant);
    if (flags & kFlagCanon) return pick_lo<true, LOGN, kOutCanon, true>(variant);
    return pick_lo<true, LOGN, kOutLazy, true>(variant);
  }
  if (!hi) return pick_lo<false, LOGN, kOutLazy, false>(variant);            // inverse: low pass first
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

// Three-pass split N = 2^LT_HIGH * 2^lt_mid * 2^lt_low: index bits [0, low) in
// the low pass, [low, low + mid) in the middle pass, the top LT_HIGH bits in
// the high pass (2^15: 5 + 5 + 5, 2^16: 6 + 5 + 5, 2^17: 6 + 6 + 5).  Tiles hold
// 4096 coefficients, except the middle pass's columns, which stay inside the
// low pass's bits (2048 coefficients at 2^16, 1024 at 2^15).
constexpr int kThreeHigh = 5;
__host__ __device__ constexpr int three_low(int logN) { return logN == 15 ? 5 : 6; }
__host__ __device__ constexpr int three_mid(int logN) { return logN - kThreeHigh - three_low(logN); }
__host__ __device__ constexpr int three_mid_logc(int logN) {
  return 12 - three_mid(logN) < three_low(logN) ? 12 - three_mid(logN) : three_low(logN);
}
constexpr int kThreeLogr = 3;

// Kernel of pass `which` (0 high, 1 middle, 2 low) of the three-pass schedule.
template <bool FWD, int LOGN, int WHICH, int MODE, bool LAST>
static PassKernel pick_three_r() {
  if constexpr (WHICH == 0)
    return ntt_tile_kernel<FWD, kThreeHigh, kThreeLogr, 12 - kThreeHigh, 0, 4, MODE, LAST, -1>;
  else if constexpr (WHICH == 1)
    return ntt_tile_kernel<FWD, three_mid(LOGN), kThreeLogr, three_mid_logc(LOGN), 0, 4, MODE, LAST, -1>;
  else
    return ntt_tile_kernel<FWD, three_low(LOGN), kThreeLogr, 0, 12 - three_low(LOGN), 4, MODE, LAST, -1>;
}
// Forward: high, middle, low (the low pass last); inverse: low, middle, high.
template <int LOGN>
static PassKernel pick_three(bool fwd, int which, u32 flags) {
  if (fwd) {
    if (which == 0) return pick_three_r<true, LOGN, 0, kOutLazy, false>();
    if (which == 1) return pick_three_r<true, LOGN, 1, kOutLazy, false>();
    if (flags & kFlagMul) return pick_three_r<true, LOGN, 2, kOutMul, true>();
    if (flags & kFlagCanon) return pick_three_r<true, LOGN, 2, kOutCanon, true>();
    return pick_three_r<true, LOGN, 2, kOutLazy, true>();
  }
  if (which == 2) return pick_three_r<false, LOGN, 2, kOutLazy, false>();
  if (which == 1) return pick_three_r<false, LOGN, 1, kOutLazy, false>();
  if (flags & kFlagAcc) return pick_three_r<false, LOGN, 0, kOutAcc, true>();
  if (flags & kFlagCanon) return pick_three_r<false, LOGN, 0, kOutCanon, true>();
  return pick_three_r<false, LOGN, 0, kOutLazy, true>();
}
static PassKernel pick_three_n(int logN, bool fwd, int which, u32 flags) {
  switch (logN) {
    case 15: return pick_three<15>(fwd, which, flags);
    case 16: return pick_three<16>(fwd, which, flags);
    case 17: return pick_three<17>(fwd, which, flags);
    default: return nullptr;
  }
}

// Number of passes the schedule for 2^logN uses (1 = the whole transform on chip).
int pass_count(int logN) { return logN <= kMaxOnchipLog ? 1 : 2; }

// Schedule variant per (device, direction, logN, batch size); set by the autotuner
// on the device it ran on, read by every launch there (atomics: calls may come
// from several host threads).
constexpr int kVariantDevices = 64;
static std::atomic<int> g_hi_variant[kVariantDevices][2][NTT_MAX_LOG_DEGREE + 1][2];
static int batch_bucket(uint64_t items) { return items <= 64 ? 0 : 1; }
static int variant_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kVariantDevices) dev = 0;
  return dev;
}

void set_hi_variant(bool fwd, int logN, uint64_t items, int variant) {
  g_hi_variant[variant_device()][fwd ? 1 : 0][logN][batch_bucket(items)].store(variant, std::memory_order_relaxed);
}
int get_hi_variant(bool fwd, int logN, uint64_t items) {
  return g_hi_variant[variant_device()][fwd ? 1 : 0][logN][batch_bucket(items)].load(std::memory_order_relaxed);
}
int variant_count(int logN) { return logN > kMaxOnchipLog ? kVariants : (logN >= 10 ? 2 : 1); }

static std::atomic<int> g_wide_range{1};
bool wide_range_enabled() { return g_wide_range.load(std::memory_order_relaxed) != 0; }
void set_wide_range(bool on) { g_wide_range.store(on ? 1 : 0); }

// The single-pass kernels take the wide-range butterflies when every modulus of
// the launch is below kWideModulusBound: from inputs below 4q, 14 forward stages
// keep every value below 46 q < 2^64.
static bool use_wide(const NttLaunch& l) {
  if (!wide_range_enabled()) return false;
  for (uint32_t i = 0; i < l.num_limbs; ++i)
    if (l.plans[i]->q >= kWideModulusBound) return false;
  return true;
}

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
    const int variant = force_variant >= 0 ? force_variant : get_hi_variant(fwd, logN, items);
    if (variant < 0 || variant >= variant_count(logN)) return NTT_EINVAL_COUNT;
    ntt_status st = launch_onchip(a, items, fwd, use_wide(l), l.stream, variant);
    if (st) return st;
    return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
  }
  if (logN > NTT_MAX_LOG_DEGREE) return NTT_EINVAL_DEGREE;
  const int variant = force_variant >= 0 ? force_variant : get_hi_variant(fwd, logN, items);
  if (variant < 0 || variant >= kVariants) return NTT_EINVAL_COUNT;
  uint64_t* mid = l.tmp ? l.tmp : l.out;
  const uint64_t kMaxY = 65535;
  if (kVariantShape[variant].passes == 3) {
    // bit ranges (b0, bits, columns or blocks) of the high, middle and low passes
    const int low = three_low(logN), midb = three_mid(logN);
    for (int step = 0; step < 3; ++step) {
      const int which = fwd ? step : 2 - step;
      const bool last = step == 2;
      a.in = step == 0 ? l.in : mid;
      a.out = last ? l.out : mid;
      a.flags = last ? last_flags : 0u;
      PassKernel k = pick_three_n(logN, fwd, which, a.flags);
      if (!k) return NTT_EINVAL_DEGREE;
      int bits, logc, logh;
      if (which == 0) { a.b0 = (u32)(low + midb); bits = kThreeHigh; logc = 12 - kThreeHigh; logh = 0; }
      else if (which == 1) { a.b0 = (u32)low; bits = midb; logc = three_mid_logc(logN); logh = 0; }
      else { a.b0 = 0; bits = low; logc = 0; logh = 12 - low; }
      const int nt = 1 << (bits + logc + logh - kThreeLogr);
      const uint64_t tiles = 1ull << (logN - bits - logc - logh);
      for (uint64_t it0 = 0; it0 < items; it0 += kMaxY) {
        const uint64_t ny = (items - it0) < kMaxY ? (items - it0) : kMaxY;
        a.item0 = (u32)it0;
        hipLaunchKernelGGL(k, dim3((unsigned)tiles, (unsigned)ny), dim3(nt), 0, l.stream, a);
      }
    }
    return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
  }
  const int lt_lo = variant_lt_lo(logN, variant), lt_hi = logN - lt_lo;
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
      const int logr = hi_logr(logN, variant), logc = hi_logc(lt_hi) - variant_half(variant);
      nt = 1 << (lt_hi + logc - logr);
      tiles = (1ull << lt_lo) >> logc;
    } else {
      a.b0 = 0;
      nt = 1 << (12 - variant_half(variant) - lo_logr(variant));
      tiles = 1ull << (logN - 12 + variant_half(variant));
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

// Fused product per limb (N <= 2^14): in = b, mul_into = NTT(a) lazy, out =
// canonical product or accumulator.
ntt_status launch_product(const NttLaunch& l, bool acc) {
  const int logN = l.plans[0]->logN;
  if (logN > kMaxOnchipLog) return NTT_EINVAL_DEGREE;
  if (l.num_limbs == 0 || l.num_limbs > (uint32_t)kMaxPlansPerLaunch) return NTT_EINVAL_COUNT;
  PassArgs a{};
  for (uint32_t i = 0; i < l.num_limbs; ++i) a.plan[i] = l.plans[i]->dev;
  a.num_limbs = l.num_limbs;
  a.logN = (u32)logN;
  a.in = l.in;
  a.out = l.out;
  a.mul = l.mul_into;
  return launch_onchip_product(a, l.num_polys * l.num_limbs, acc, use_wide(l), l.stream);
}

ntt_status launch_forward(const NttLaunch& l) { return launch_passes(l, true, -1); }
ntt_status launch_inverse(const NttLaunch& l) { return launch_passes(l, false, -1); }
ntt_status launch_variant(const NttLaunch& l, bool fwd, int variant) { return launch_passes(l, fwd, variant); }

}  // namespace nttamd
