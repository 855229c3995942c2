// Negacyclic NTT kernels for gfx950.
//
// The forward transform is Algorithm 2 (Cooley-Tukey, merged psi twiddles,
// bit-reversed output) with the Harvey butterfly of Algorithm 4; the inverse is
// Algorithm 3 (Gentleman-Sande) with the butterfly of Algorithm 5 and the
// scaling by N^{-1} fused into its last stage.  Every butterfly performs
// exactly the arithmetic of Algorithm 4 / 5, so only the order in which
// independent butterflies run differs from the radix-2 loops.
//
// Decomposition.  The stage that pairs indices differing in bit b uses the
// twiddle with table index (N + g) >> (b + 1), g the lower index (this is
// psi_rev[m + i] of Algorithm 2 and psi^{-1}_rev[h + i] of Algorithm 3).  A
// "pass" handles the stages of a contiguous range of index bits
// [b0, b0 + LOGT): the elements that share all other bits form independent
// sub-transforms of size 2^LOGT with stride 2^b0 (the Cooley-Tukey split
// N = N1 N2 of Section 2.2).  A workgroup owns a tile of C = 2^LOGC adjacent
// columns (strided passes, b0 > 0) or H = 2^LOGH adjacent blocks (contiguous
// passes, b0 = 0), loads it once, runs all of the pass's stages on chip and
// stores it once.  Forward passes run from the top bits down, inverse passes
// from the bottom bits up.
//
// Inside a tile, each thread holds R = 2^LOGR elements in registers and runs
// up to LOGR stages on them ("round"); rounds exchange data through LDS.  LDS
// rows are padded by one word every R rows so that the strided exchanges are
// free of bank conflicts.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"
#include "ntt_common.h"

namespace nttamd {

template <int LOGR>
__device__ __forceinline__ u32 lds_row(u32 rho) { return rho + (rho >> LOGR); }

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH, int R>
struct Tile {
  static constexpr int RB = LOGT + LOGH;                 // row bits of the tile
  static constexpr int C = 1 << LOGC;
  static constexpr int NT = 1 << (RB + LOGC - LOGR);
  static constexpr int ROWS = 1 << RB;
  static constexpr int LDS_WORDS = (ROWS + (ROWS >> LOGR)) * C;
  using G = Geo<FWD, LOGT, LOGR>;

  // row index of element j of thread `o` (row part of the thread id) in round r
  template <int r>
  __device__ static __forceinline__ u32 rho(u32 o, int j) {
    constexpr int lo = G::lo(r);
    const u32 lo_part = o & ((1u << lo) - 1u);
    const u32 hi_part = o >> lo;
    return (hi_part << (lo + LOGR)) | ((u32)j << lo) | lo_part;
  }
  // are 16 consecutive lanes consecutive in memory in round r?
  template <int r>
  static constexpr bool coalesced() { return LOGC >= 4 || G::lo(r) >= 4; }

  template <int r>
  __device__ static __forceinline__ void to_lds(u64* lds, const u64 (&x)[R], u32 o, u32 c) {
#pragma unroll
    for (int j = 0; j < R; ++j) lds[lds_row<LOGR>(rho<r>(o, j)) * C + c] = x[j];
  }
  template <int r>
  __device__ static __forceinline__ void from_lds(const u64* lds, u64 (&x)[R], u32 o, u32 c) {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = lds[lds_row<LOGR>(rho<r>(o, j)) * C + c];
  }

  // stages of round r on the thread's registers
  template <int r>
  __device__ static __forceinline__ void stages(u64 (&x)[R], u64 g_base, const PlanView& pv, u32 b0, u64 N,
                                                bool last_pass) {
    constexpr int lo = G::lo(r);
#pragma unroll
    for (int s = 0; s < G::nst(r); ++s) {
      const int bit = FWD ? (G::first_bit(r) - s) : (G::first_bit(r) + s);   // local stage bit
      const int p = bit - lo;                                                 // bit inside j
      const u32 b = b0 + (u32)bit;                                            // global stage bit
      const u64 tbase = (N + g_base) >> (b + 1);
      const bool fused_last = !FWD && last_pass && bit == LOGT - 1;
#pragma unroll
      for (int k = 0; k < R / 2; ++k) {
        const int j = ((k >> p) << (p + 1)) | (k & ((1 << p) - 1));
        const int j2 = j | (1 << p);
        if (FWD) {
          const ulonglong2 w = pv.tw[tbase + (u64)(j >> (p + 1))];
          harvey_fwd(x[j], x[j2], w.x, w.y, pv.q2, pv.nq);
        } else if (fused_last) {
          harvey_inv_last(x[j], x[j2], pv.ninv, pv.ninv_p, pv.wn, pv.wn_p, pv.q2, pv.nq);
        } else {
          const ulonglong2 w = pv.tw[tbase + (u64)(j >> (p + 1))];
          harvey_inv(x[j], x[j2], w.x, w.y, pv.q2, pv.nq);
        }
      }
    }
  }

  template <int r>
  __device__ static __forceinline__ void run_rounds(u64* lds, u64 (&x)[R], u32 o, u32 c, u64 g_tile,
                                                    const PlanView& pv, u32 b0, u64 N, bool last_pass) {
    const u64 g_base = g_tile + ((u64)rho<r>(o, 0) << b0) + c;
    stages<r>(x, g_base, pv, b0, N, last_pass);
    if constexpr (r + 1 < G::NR) {
      __syncthreads();
      to_lds<r>(lds, x, o, c);
      __syncthreads();
      from_lds<r + 1>(lds, x, o, c);
      run_rounds<r + 1>(lds, x, o, c, g_tile, pv, b0, N, last_pass);
    }
  }
};

template <bool FWD, int LOGT, int LOGR, int LOGC, int LOGH>
__global__ void __launch_bounds__(1 << (LOGT + LOGC + LOGH - LOGR))
ntt_pass_kernel(const PassArgs a) {
  constexpr int R = 1 << LOGR;
  using TL = Tile<FWD, LOGT, LOGR, LOGC, LOGH, R>;
  using G = typename TL::G;
  constexpr int C = TL::C;
  constexpr int NT = TL::NT;
  constexpr int TILE = TL::ROWS * C;
  __shared__ u64 lds[TL::LDS_WORDS];

  const u32 item = a.item0 + blockIdx.y;
  const u32 logN = a.logN;
  const u64 N = 1ull << logN;
  const PlanView pv = load_plan(a.plan[item % a.num_limbs], FWD, N);
  const u32 b0 = a.b0;
  const bool last_pass = (a.flags & kFlagLast) != 0;
  const u64 base = (u64)item << logN;

  u64 g_tile;
  if (LOGC > 0) {
    const u32 ncg = (1u << b0) >> LOGC;
    const u32 cg = blockIdx.x % ncg, hb = blockIdx.x / ncg;
    g_tile = ((u64)hb << (b0 + LOGT)) | ((u64)cg << LOGC);
  } else {
    g_tile = (u64)blockIdx.x << (LOGT + LOGH + b0);
  }
  const u32 tid = threadIdx.x;
  const u32 c = tid & (C - 1);
  const u32 o = tid >> LOGC;

  u64 x[R];
  // ---- load
  if constexpr (TL::template coalesced<0>()) {
#pragma unroll
    for (int j = 0; j < R; ++j) x[j] = a.in[base + g_tile + ((u64)TL::template rho<0>(o, j) << b0) + c];
  } else {
#pragma unroll
    for (int e0 = 0; e0 < TILE; e0 += NT) {
      const u32 e = e0 + tid;
      const u32 rr = e >> LOGC, cc = e & (C - 1);
      lds[lds_row<LOGR>(rr) * C + cc] = a.in[base + g_tile + ((u64)rr << b0) + cc];
    }
    __syncthreads();
    TL::template from_lds<0>(lds, x, o, c);
  }

  // ---- stages
  TL::template run_rounds<0>(lds, x, o, c, g_tile, pv, b0, N, last_pass);

  // ---- store
  constexpr int RL = G::NR - 1;
  if constexpr (TL::template coalesced<RL>()) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const u64 idx = base + g_tile + ((u64)TL::template rho<RL>(o, j) << b0) + c;
      a.out[idx] = finish<FWD>(x[j], idx, a, pv);
    }
  } else {
    __syncthreads();
    TL::template to_lds<RL>(lds, x, o, c);
    __syncthreads();
#pragma unroll
    for (int e0 = 0; e0 < TILE; e0 += NT) {
      const u32 e = e0 + tid;
      const u32 rr = e >> LOGC, cc = e & (C - 1);
      const u64 idx = base + g_tile + ((u64)rr << b0) + cc;
      a.out[idx] = finish<FWD>(lds[lds_row<LOGR>(rr) * C + cc], idx, a, pv);
    }
  }
}

// ---- schedules ---------------------------------------------------------------

struct PassShape {
  int logt, logr, logc, logh;
};
struct Schedule {
  int npass;
  PassShape pass[3];  // in execution order for the FORWARD transform (top bits first)
};

// Forward passes run from the high bits down; the inverse runs the same
// passes in reverse order (low bits first).
static Schedule schedule_for(int logN) {
  switch (logN) {
    case 1: return {1, {{1, 1, 0, 0}}};
    case 2: return {1, {{2, 2, 0, 0}}};
    case 3: return {1, {{3, 3, 0, 0}}};
    case 4: return {1, {{4, 4, 0, 0}}};
    case 5: return {1, {{5, 4, 0, 0}}};
    case 6: return {1, {{6, 4, 0, 0}}};
    case 7: return {1, {{7, 4, 0, 0}}};
    case 8: return {1, {{8, 4, 0, 0}}};
    case 9: return {1, {{9, 4, 0, 0}}};
    case 10: return {1, {{10, 4, 0, 0}}};
    case 11: return {1, {{11, 4, 0, 0}}};
    case 12: return {1, {{12, 4, 0, 0}}};
    case 13: return {1, {{13, 4, 0, 0}}};
    case 14: return {1, {{14, 5, 0, 0}}};
    case 15: return {2, {{8, 4, 4, 0}, {7, 4, 0, 5}}};
    case 16: return {2, {{8, 4, 4, 0}, {8, 4, 0, 4}}};
    case 17: return {2, {{9, 4, 4, 0}, {8, 4, 0, 4}}};
    default: return {0, {}};
  }
}

typedef void (*PassKernel)(const PassArgs);

template <bool FWD>
static PassKernel pick_kernel(const PassShape& s) {
#define NTT_CASE(T, R, C, H) \
  if (s.logt == T && s.logr == R && s.logc == C && s.logh == H) return ntt_pass_kernel<FWD, T, R, C, H>;
  NTT_CASE(7, 4, 0, 5) NTT_CASE(8, 4, 4, 0) NTT_CASE(8, 4, 0, 4) NTT_CASE(9, 4, 4, 0)
#undef NTT_CASE
  return nullptr;
}

// Number of passes the schedule for 2^logN uses (1 = the whole transform on chip).
int pass_count(int logN) { return schedule_for(logN).npass; }

static ntt_status launch_passes(const NttLaunch& l, bool fwd) {
  const ntt_plan* p0 = l.plans[0];
  const int logN = p0->logN;
  const Schedule sch = schedule_for(logN);
  if (sch.npass == 0) return NTT_EINVAL_DEGREE;
  if (l.num_limbs == 0 || l.num_limbs > (uint32_t)kMaxPlansPerLaunch) return NTT_EINVAL_COUNT;
  PassArgs a{};
  for (uint32_t i = 0; i < l.num_limbs; ++i) a.plan[i] = l.plans[i]->dev;
  a.num_limbs = l.num_limbs;
  a.logN = (u32)logN;
  a.mul = l.mul_into;
  const uint64_t items = l.num_polys * l.num_limbs;
  const uint64_t kMaxY = 65535;
  // bit offsets of the forward passes: pass 0 covers the top bits
  int b0s[3];
  {
    int top = logN;
    for (int i = 0; i < sch.npass; ++i) { top -= sch.pass[i].logt; b0s[i] = top; }
  }
  if (sch.npass == 1) {
    a.in = l.in;
    a.out = l.out;
    a.b0 = 0;
    a.flags = kFlagLast;
    if (l.out_f == 1) a.flags |= kFlagCanon;
    if (fwd && l.mul_into) a.flags |= kFlagMul;
    if (!fwd && l.mul_into) a.flags |= kFlagAcc;
    ntt_status st = launch_onchip(a, items, fwd, l.stream);
    if (st) return st;
    return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
  }
  for (int step = 0; step < sch.npass; ++step) {
    const int i = fwd ? step : (sch.npass - 1 - step);
    const PassShape& s = sch.pass[i];
    PassKernel k = fwd ? pick_kernel<true>(s) : pick_kernel<false>(s);
    if (!k) return NTT_EINVAL_DEGREE;
    a.b0 = (u32)b0s[i];
    const bool last = (step == sch.npass - 1);
    uint64_t* mid = l.tmp ? l.tmp : l.out;
    a.in = (step == 0) ? l.in : mid;
    a.out = last ? l.out : mid;
    a.flags = 0;
    if (last) {
      a.flags |= kFlagLast;
      if (l.out_f == 1) a.flags |= kFlagCanon;
      if (fwd && l.mul_into) a.flags |= kFlagMul;
      if (!fwd && l.mul_into) a.flags |= kFlagAcc;
    }
    const int nt = 1 << (s.logt + s.logc + s.logh - s.logr);
    uint64_t tiles;
    if (s.logc > 0) tiles = ((1ull << a.b0) >> s.logc) * (1ull << (logN - a.b0 - s.logt));
    else tiles = 1ull << (logN - s.logt - s.logh);
    for (uint64_t it0 = 0; it0 < items; it0 += kMaxY) {
      const uint64_t ny = (items - it0) < kMaxY ? (items - it0) : kMaxY;
      a.item0 = (u32)it0;
      hipLaunchKernelGGL(k, dim3((unsigned)tiles, (unsigned)ny), dim3(nt), 0, l.stream, a);
    }
  }
  if (hipGetLastError() != hipSuccess) return NTT_EDEVICE;
  return NTT_OK;
}

ntt_status launch_forward(const NttLaunch& l) { return launch_passes(l, true); }
ntt_status launch_inverse(const NttLaunch& l) { return launch_passes(l, false); }

}  // namespace nttamd
