// Element-wise modular kernels on RNS limbs (Section 2 ring operations; the
// EltwiseMultMod / EltwiseAddMod / EltwiseFMAMod free functions of Section 4;
// Algorithms 8 and 10; subtraction and negation).  All are bound by HBM
// traffic (16-24 bytes per element), so the kernels stream 16-byte vectors
// with a grid-stride loop; blockIdx.y selects the limb, whose modulus
// constants come from the kernel arguments.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "modarith.h"

namespace nttamd {

struct LimbConst {
  u64 q, q2, k;
  u32 qbits, pad;
  u64 y, yp;         // EltwiseFMAMod: scalar in [0, q) and its Shoup companion floor(y 2^64 / q)
};

struct EltArgs {
  u64* out;
  const u64* a;
  const u64* b;
  u64 n;             // elements per limb
  u32 num_limbs;     // item y uses limb[y % num_limbs]
  u32 item0;
  LimbConst limb[NTT_MAX_LIMBS];
};

template <int F, bool VEC>
__global__ void __launch_bounds__(256) eltwise_mult_kernel(const EltArgs a) {
  const u32 item = a.item0 + blockIdx.y;
  const LimbConst L = a.limb[item % a.num_limbs];
  const u64 off = (u64)item * a.n;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const ulonglong2* A = reinterpret_cast<const ulonglong2*>(a.a + off);
    const ulonglong2* B = reinterpret_cast<const ulonglong2*>(a.b + off);
    ulonglong2* O = reinterpret_cast<ulonglong2*>(a.out + off);
    for (; i < a.n / 2; i += stride) {
      const ulonglong2 x = A[i], y = B[i];
      ulonglong2 r;
      r.x = barrett_mulmod<F>(x.x, y.x, L.q, L.q2, L.k, L.qbits);
      r.y = barrett_mulmod<F>(x.y, y.y, L.q, L.q2, L.k, L.qbits);
      O[i] = r;
    }
  } else {
    for (; i < a.n; i += stride)
      a.out[off + i] = barrett_mulmod<F>(a.a[off + i], a.b[off + i], L.q, L.q2, L.k, L.qbits);
  }
}

template <bool VEC>
__global__ void __launch_bounds__(256) eltwise_add_kernel(const EltArgs a) {
  const u32 item = a.item0 + blockIdx.y;
  const u64 q = a.limb[item % a.num_limbs].q;
  const u64 off = (u64)item * a.n;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const ulonglong2* A = reinterpret_cast<const ulonglong2*>(a.a + off);
    const ulonglong2* B = reinterpret_cast<const ulonglong2*>(a.b + off);
    ulonglong2* O = reinterpret_cast<ulonglong2*>(a.out + off);
    for (; i < a.n / 2; i += stride) {
      const ulonglong2 x = A[i], y = B[i];
      ulonglong2 r;
      r.x = csub(x.x + y.x, q);
      r.y = csub(x.y + y.y, q);
      O[i] = r;
    }
  } else {
    for (; i < a.n; i += stride) a.out[off + i] = csub(a.a[off + i] + a.b[off + i], q);
  }
}

// x mod q for x in [0, F q), F in {1, 2, 4, 8}: conditional subtractions of
// 4q, 2q and q as needed (the small_mod steps of Algorithm 10).
template <int F>
__device__ __forceinline__ u64 reduce_f(u64 x, u64 q, u64 q2) {
  if (F >= 8) x = csub(x, 2 * q2);
  if (F >= 4) x = csub(x, q2);
  if (F >= 2) x = csub(x, q);
  return x;
}

// Algorithm 10: (X Y + Z) mod q with the scalar Y's Shoup companion; inputs
// first reduced to [0, q); the product in [0, 2q) and the sum each take one
// conditional subtraction.
template <int F, bool ADD>
__device__ __forceinline__ u64 fma_one(u64 x, u64 z, const LimbConst& L) {
  x = reduce_f<F>(x, L.q, L.q2);
  u64 r = csub(shoup_mul(x, L.y, L.yp, 0 - L.q), L.q);
  if (ADD) r = csub(r + reduce_f<F>(z, L.q, L.q2), L.q);
  return r;
}

template <int F, bool ADD, bool VEC>
__global__ void __launch_bounds__(256) eltwise_fma_kernel(const EltArgs a) {
  const u32 item = a.item0 + blockIdx.y;
  const LimbConst L = a.limb[item % a.num_limbs];
  const u64 off = (u64)item * a.n;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const ulonglong2* A = reinterpret_cast<const ulonglong2*>(a.a + off);
    const ulonglong2* Z = reinterpret_cast<const ulonglong2*>(ADD ? a.b + off : a.a + off);
    ulonglong2* O = reinterpret_cast<ulonglong2*>(a.out + off);
    for (; i < a.n / 2; i += stride) {
      const ulonglong2 x = A[i];
      ulonglong2 z = {0, 0};
      if (ADD) z = Z[i];
      ulonglong2 r;
      r.x = fma_one<F, ADD>(x.x, z.x, L);
      r.y = fma_one<F, ADD>(x.y, z.y, L);
      O[i] = r;
    }
  } else {
    for (; i < a.n; i += stride) a.out[off + i] = fma_one<F, ADD>(a.a[off + i], ADD ? a.b[off + i] : 0, L);
  }
}

// (a - b) mod q for a, b in [0, q): a + (q - b) in [1, 2q), then one
// conditional subtraction; NEG computes (0 - a) mod q the same way (so that
// the zero residue stays 0).
template <bool NEG, bool VEC>
__global__ void __launch_bounds__(256) eltwise_sub_kernel(const EltArgs a) {
  const u32 item = a.item0 + blockIdx.y;
  const u64 q = a.limb[item % a.num_limbs].q;
  const u64 off = (u64)item * a.n;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const ulonglong2* A = reinterpret_cast<const ulonglong2*>(a.a + off);
    const ulonglong2* B = reinterpret_cast<const ulonglong2*>(NEG ? a.a + off : a.b + off);
    ulonglong2* O = reinterpret_cast<ulonglong2*>(a.out + off);
    for (; i < a.n / 2; i += stride) {
      const ulonglong2 x = A[i];
      const ulonglong2 y = NEG ? x : B[i];
      ulonglong2 r;
      r.x = NEG ? csub(q - x.x, q) : csub(x.x + (q - y.x), q);
      r.y = NEG ? csub(q - x.y, q) : csub(x.y + (q - y.y), q);
      O[i] = r;
    }
  } else {
    for (; i < a.n; i += stride) {
      const u64 x = a.a[off + i];
      a.out[off + i] = NEG ? csub(q - x, q) : csub(x + (q - a.b[off + i]), q);
    }
  }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static ntt_status fill_args(const EltLaunch& l, EltArgs& a, bool& vec) {
  if (l.num_limbs == 0 || l.num_limbs > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  a.out = l.out;
  a.a = l.a;
  a.b = l.b;
  a.n = l.n;
  a.num_limbs = l.num_limbs;
  for (uint32_t i = 0; i < l.num_limbs; ++i) {
    const uint64_t q = l.moduli[i];
    a.limb[i].q = q;
    a.limb[i].q2 = 2 * q;
    a.limb[i].k = barrett_factor(q, &a.limb[i].qbits);
    a.limb[i].pad = 0;
    a.limb[i].y = 0;
    a.limb[i].yp = 0;
    if (l.scalars) {
      const uint64_t y = l.scalars[i] % q;
      a.limb[i].y = y;
      a.limb[i].yp = (uint64_t)(((unsigned __int128)y << 64) / q);
    }
  }
  vec = (l.n % 2 == 0) && aligned16(l.out) && aligned16(l.a) && (!l.b || aligned16(l.b));
  return NTT_OK;
}

template <typename K>
static void launch_items(K kernel, EltArgs& a, const EltLaunch& l, bool vec) {
  const uint64_t items = l.num_polys * l.num_limbs;
  const uint64_t units = vec ? l.n / 2 : l.n;
  uint64_t blocks_x = (units + 255) / 256;
  // enough waves to fill 256 CUs without one block per element of huge limbs
  const uint64_t max_x = items >= 64 ? 8 : (items >= 8 ? 64 : 1024);
  if (blocks_x > max_x) blocks_x = max_x;
  if (blocks_x == 0) blocks_x = 1;
  const uint64_t kMaxY = 65535;
  for (uint64_t it0 = 0; it0 < items; it0 += kMaxY) {
    const uint64_t ny = (items - it0) < kMaxY ? (items - it0) : kMaxY;
    a.item0 = (u32)it0;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks_x, (unsigned)ny), dim3(256), 0, l.stream, a);
  }
}

ntt_status launch_eltwise_mult(const EltLaunch& l) {
  EltArgs a;
  bool vec = false;
  ntt_status st = fill_args(l, a, vec);
  if (st) return st;
  switch (l.in_f) {
    case 1: vec ? launch_items(eltwise_mult_kernel<1, true>, a, l, vec) : launch_items(eltwise_mult_kernel<1, false>, a, l, vec); break;
    case 2: vec ? launch_items(eltwise_mult_kernel<2, true>, a, l, vec) : launch_items(eltwise_mult_kernel<2, false>, a, l, vec); break;
    case 4: vec ? launch_items(eltwise_mult_kernel<4, true>, a, l, vec) : launch_items(eltwise_mult_kernel<4, false>, a, l, vec); break;
    default: return NTT_EINVAL_FACTOR;
  }
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

ntt_status launch_eltwise_add(const EltLaunch& l) {
  EltArgs a;
  bool vec = false;
  ntt_status st = fill_args(l, a, vec);
  if (st) return st;
  vec ? launch_items(eltwise_add_kernel<true>, a, l, vec) : launch_items(eltwise_add_kernel<false>, a, l, vec);
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

ntt_status launch_eltwise_sub(const EltLaunch& l, bool negate) {
  EltArgs a;
  bool vec = false;
  ntt_status st = fill_args(l, a, vec);
  if (st) return st;
  if (negate) vec ? launch_items(eltwise_sub_kernel<true, true>, a, l, vec) : launch_items(eltwise_sub_kernel<true, false>, a, l, vec);
  else vec ? launch_items(eltwise_sub_kernel<false, true>, a, l, vec) : launch_items(eltwise_sub_kernel<false, false>, a, l, vec);
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

template <int F>
static void launch_fma_f(EltArgs& a, const EltLaunch& l, bool vec) {
  const bool add = l.b != nullptr;
  if (add) vec ? launch_items(eltwise_fma_kernel<F, true, true>, a, l, vec) : launch_items(eltwise_fma_kernel<F, true, false>, a, l, vec);
  else vec ? launch_items(eltwise_fma_kernel<F, false, true>, a, l, vec) : launch_items(eltwise_fma_kernel<F, false, false>, a, l, vec);
}

ntt_status launch_eltwise_fma(const EltLaunch& l) {
  if (!l.scalars) return NTT_EINVAL_POINTER;
  EltArgs a;
  bool vec = false;
  ntt_status st = fill_args(l, a, vec);
  if (st) return st;
  switch (l.in_f) {
    case 1: launch_fma_f<1>(a, l, vec); break;
    case 2: launch_fma_f<2>(a, l, vec); break;
    case 4: launch_fma_f<4>(a, l, vec); break;
    case 8: launch_fma_f<8>(a, l, vec); break;
    default: return NTT_EINVAL_FACTOR;
  }
  return hipGetLastError() == hipSuccess ? NTT_OK : NTT_EDEVICE;
}

}  // namespace nttamd
