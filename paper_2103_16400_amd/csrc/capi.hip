// extern "C" entry points: argument validation, plan lookup, launches.
#include <hip/hip_runtime.h>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace nttamd;

namespace {

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// An output may equal an input exactly (in place) but not overlap it otherwise.
ntt_status check_alias(const void* out, const void* in, size_t bytes) {
  if (out == in) return NTT_OK;
  return overlaps(out, bytes, in, bytes) ? NTT_EALIAS : NTT_OK;
}

ntt_status check_fwd_factors(uint64_t in_f, uint64_t out_f) {
  if (!(in_f == 1 || in_f == 2 || in_f == 4)) return NTT_EINVAL_FACTOR;
  if (!(out_f == 1 || out_f == 4)) return NTT_EINVAL_FACTOR;
  return NTT_OK;
}
ntt_status check_inv_factors(uint64_t in_f, uint64_t out_f) {
  if (!(in_f == 1 || in_f == 2)) return NTT_EINVAL_FACTOR;
  if (!(out_f == 1 || out_f == 2)) return NTT_EINVAL_FACTOR;
  return NTT_OK;
}

// q in [2, 2^62) and f * q < 2^63 (Algorithm 8 requirements).
ntt_status check_mult_modulus(uint64_t q, uint64_t in_f) {
  if (!(in_f == 1 || in_f == 2 || in_f == 4)) return NTT_EINVAL_FACTOR;
  if (q < 2 || q >= (1ull << 62)) return NTT_EINVAL_MODULUS;
  if ((unsigned __int128)q * in_f >= ((unsigned __int128)1 << 63)) return NTT_EINVAL_MODULUS;
  return NTT_OK;
}
// q in [2, 2^63 - 1] (EltwiseAddMod contract).
ntt_status check_add_modulus(uint64_t q) {
  if (q < 2 || q > (1ull << 63) - 1) return NTT_EINVAL_MODULUS;
  return NTT_OK;
}

ntt_status rns_plans(uint64_t N, const uint64_t* moduli, uint64_t L, std::vector<const ntt_plan*>& plans) {
  if (!moduli) return NTT_EINVAL_POINTER;
  if (L == 0 || L > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  plans.resize(L);
  for (uint64_t i = 0; i < L; ++i) {
    st = cached_plan(N, moduli[i], &plans[i]);
    if (st) return st;
  }
  return NTT_OK;
}

ntt_status ntt_rns(bool fwd, uint64_t* result, const uint64_t* operand, const uint64_t* mul, uint64_t* tmp,
                   uint64_t N, const uint64_t* moduli, uint64_t L, uint64_t B, uint64_t in_f, uint64_t out_f,
                   ntt_stream_t stream) {
  if (!result || !operand) return NTT_EINVAL_POINTER;
  ntt_status st = fwd ? check_fwd_factors(in_f, out_f) : check_inv_factors(in_f, out_f);
  if (st) return st;
  if (B == 0 || L == 0) return NTT_EINVAL_COUNT;
  st = validate_degree(N);
  if (st) return st;
  if (B > (1ull << 40) / (L * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(B * L * N * sizeof(uint64_t));
  st = check_alias(result, operand, bytes);
  if (st) return st;
  std::vector<const ntt_plan*> plans;
  st = rns_plans(N, moduli, L, plans);
  if (st) return st;
  if (validate_enabled()) {
    st = check_range(operand, 64, N, moduli, L, B, in_f, (hipStream_t)stream);
    if (!st && mul) st = check_range(mul, 64, N, moduli, L, B, fwd ? 4 : 1, (hipStream_t)stream);
    if (st) return st;
  }
  NttLaunch l{result, operand, mul, tmp, plans.data(), (uint32_t)L, B, (uint32_t)in_f, (uint32_t)out_f,
              (hipStream_t)stream};
  return fwd ? launch_forward(l) : launch_inverse(l);
}

// Word-size-2^32 path: moduli below 2^30 (4q < 2^32), N in [2, 2^17]; tmp: the
// products' workspace at N >= 2^16.
ntt_status small_call(uint32_t op, uint32_t* out, const uint32_t* in, const uint32_t* mul, uint64_t N,
                      const uint64_t* moduli, uint64_t L, uint64_t B, uint64_t in_f, ntt_stream_t stream,
                      uint32_t* tmp = nullptr) {
  if (!out || !in || !moduli) return NTT_EINVAL_POINTER;
  if (B == 0 || L == 0 || L > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  int logN = 0;
  while ((1ull << logN) < N) ++logN;
  if (logN > kMaxSmallLog) return NTT_EINVAL_DEGREE;
  for (uint64_t i = 0; i < L; ++i)
    if (moduli[i] >= (1ull << 30)) return NTT_EINVAL_MODULUS;
  if (B > (1ull << 40) / (L * N)) return NTT_EINVAL_COUNT;
  std::vector<const ntt_plan*> plans;
  st = rns_plans(N, moduli, L, plans);
  if (st) return st;
  if (validate_enabled()) {
    st = check_range(in, 32, N, moduli, L, B, in_f, (hipStream_t)stream);
    if (!st && mul) st = check_range(mul, 32, N, moduli, L, B, 4, (hipStream_t)stream);
    if (!st && op == kSmallProductAcc) st = check_range(out, 32, N, moduli, L, B, 1, (hipStream_t)stream);
    if (st) return st;
  }
  Small32Launch l{out, in, mul, tmp, plans.data(), (uint32_t)L, B, logN, op, (hipStream_t)stream};
  return launch_small(l);
}

// Second half of a fused product for N <= 2^14 (one launch): out = InvNTT(NTT(b) (.) m),
// or out += it; m = NTT(a), lazy.
ntt_status product_rns(bool acc, uint64_t* out, const uint64_t* b, const uint64_t* m, uint64_t N,
                       const uint64_t* moduli, uint64_t L, uint64_t B, ntt_stream_t stream) {
  std::vector<const ntt_plan*> plans;
  ntt_status st = rns_plans(N, moduli, L, plans);
  if (st) return st;
  if (validate_enabled()) {
    st = check_range(b, 64, N, moduli, L, B, 1, (hipStream_t)stream);
    if (!st) st = check_range(m, 64, N, moduli, L, B, 4, (hipStream_t)stream);
    if (!st && acc) st = check_range(out, 64, N, moduli, L, B, 1, (hipStream_t)stream);
    if (st) return st;
  }
  NttLaunch l{out, b, m, nullptr, plans.data(), (uint32_t)L, B, 1, 1, (hipStream_t)stream};
  return launch_product(l, acc);
}

ntt_status elt_rns(bool mult, uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                   const uint64_t* moduli, uint64_t L, uint64_t B, uint64_t in_f, ntt_stream_t stream) {
  if (!result || !a || !b || !moduli) return NTT_EINVAL_POINTER;
  if (N == 0 || B == 0 || L == 0 || L > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  if (B > (1ull << 40) / (L * N)) return NTT_EINVAL_COUNT;
  for (uint64_t i = 0; i < L; ++i) {
    ntt_status st = mult ? check_mult_modulus(moduli[i], in_f) : check_add_modulus(moduli[i]);
    if (st) return st;
  }
  const size_t bytes = (size_t)(B * L * N * sizeof(uint64_t));
  ntt_status st = check_alias(result, a, bytes);
  if (st) return st;
  st = check_alias(result, b, bytes);
  if (st) return st;
  if (validate_enabled()) {
    st = check_range(a, 64, N, moduli, L, B, mult ? in_f : 1, (hipStream_t)stream);
    if (!st) st = check_range(b, 64, N, moduli, L, B, mult ? in_f : 1, (hipStream_t)stream);
    if (st) return st;
  }
  EltLaunch l{result, a, b, N, moduli, (uint32_t)L, B, (uint32_t)in_f, (hipStream_t)stream};
  return mult ? launch_eltwise_mult(l) : launch_eltwise_add(l);
}

ntt_status fma_rns(uint64_t* result, const uint64_t* a, const uint64_t* scalars, const uint64_t* z, uint64_t N,
                   const uint64_t* moduli, uint64_t L, uint64_t B, uint64_t in_f, ntt_stream_t stream) {
  if (!result || !a || !scalars || !moduli) return NTT_EINVAL_POINTER;
  if (N == 0 || B == 0 || L == 0 || L > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  if (B > (1ull << 40) / (L * N)) return NTT_EINVAL_COUNT;
  if (in_f != 1 && in_f != 2 && in_f != 4 && in_f != 8) return NTT_EINVAL_FACTOR;
  for (uint64_t i = 0; i < L; ++i)
    if (moduli[i] < 2 || moduli[i] > (1ull << 61) - 1) return NTT_EINVAL_MODULUS;
  const size_t bytes = (size_t)(B * L * N * sizeof(uint64_t));
  ntt_status st = check_alias(result, a, bytes);
  if (st) return st;
  if (z) {
    st = check_alias(result, z, bytes);
    if (st) return st;
  }
  if (validate_enabled()) {
    st = check_range(a, 64, N, moduli, L, B, in_f, (hipStream_t)stream);
    if (!st && z) st = check_range(z, 64, N, moduli, L, B, in_f, (hipStream_t)stream);
    if (st) return st;
  }
  EltLaunch l{result, a, z, N, moduli, (uint32_t)L, B, (uint32_t)in_f, (hipStream_t)stream, scalars};
  return launch_eltwise_fma(l);
}

ntt_status sub_rns(bool negate, uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                   const uint64_t* moduli, uint64_t L, uint64_t B, ntt_stream_t stream) {
  if (!result || !a || (!negate && !b) || !moduli) return NTT_EINVAL_POINTER;
  if (N == 0 || B == 0 || L == 0 || L > NTT_MAX_LIMBS) return NTT_EINVAL_COUNT;
  if (B > (1ull << 40) / (L * N)) return NTT_EINVAL_COUNT;
  for (uint64_t i = 0; i < L; ++i) {
    ntt_status st = check_add_modulus(moduli[i]);
    if (st) return st;
  }
  const size_t bytes = (size_t)(B * L * N * sizeof(uint64_t));
  ntt_status st = check_alias(result, a, bytes);
  if (st) return st;
  if (!negate) {
    st = check_alias(result, b, bytes);
    if (st) return st;
  }
  if (validate_enabled()) {
    st = check_range(a, 64, N, moduli, L, B, 1, (hipStream_t)stream);
    if (!st && !negate) st = check_range(b, 64, N, moduli, L, B, 1, (hipStream_t)stream);
    if (st) return st;
  }
  EltLaunch l{result, a, negate ? nullptr : b, N, moduli, (uint32_t)L, B, 1, (hipStream_t)stream, nullptr};
  return launch_eltwise_sub(l, negate);
}

}  // namespace

extern "C" {

const char* ntt_status_string(ntt_status s) {
  switch (s) {
    case NTT_OK: return "ok";
    case NTT_EINVAL_DEGREE: return "invalid degree: N must be a power of two in [2, 2^17]";
    case NTT_EINVAL_MODULUS: return "invalid modulus: q must be prime, q = 1 mod 2N and within the call's range";
    case NTT_EINVAL_ROOT: return "invalid root of unity: psi^N must be -1 mod q";
    case NTT_EINVAL_FACTOR: return "invalid input/output modulus factor";
    case NTT_EINVAL_POINTER: return "null pointer argument";
    case NTT_EALIAS: return "output partially overlaps an input";
    case NTT_EINVAL_COUNT: return "invalid length, limb count or polynomial count";
    case NTT_EDEVICE: return "HIP runtime error";
    case NTT_ENOMEM: return "out of memory";
    case NTT_ENOTFOUND: return "not found";
    case NTT_EBUSY: return "busy: admission refused";
    case NTT_ETIMEDOUT: return "timed out";
    case NTT_ERANGE: return "an operand value is outside [0, f q) (validation mode)";
    default: return "unknown status";
  }
}

ntt_status ntt_shutdown(void) {
  free_oneshot_batches();
  clear_plan_cache();
  free_validate_buffers();
  return NTT_OK;
}

ntt_status ntt_set_validate(int on) {
  set_validate(on != 0);
  return NTT_OK;
}

int ntt_get_validate(void) { return validate_enabled() ? 1 : 0; }

ntt_status ntt_set_wide_range(int on) {
  set_wide_range(on != 0);
  return NTT_OK;
}

int ntt_get_wide_range(void) { return wide_range_enabled() ? 1 : 0; }

ntt_status ntt_plan_create(ntt_plan** plan, uint64_t N, uint64_t q, uint64_t root_of_unity) {
  return build_plan(plan, N, q, root_of_unity);
}

ntt_status ntt_plan_destroy(ntt_plan* plan) {
  if (!plan) return NTT_EINVAL_POINTER;
  (void)hipFree(plan->dev);
  delete plan;
  return NTT_OK;
}

uint64_t ntt_plan_root(const ntt_plan* plan) { return plan ? plan->psi : 0; }

static ntt_status single_plan_call(bool fwd, const ntt_plan* plan, uint64_t* result, const uint64_t* operand,
                                   uint64_t in_f, uint64_t out_f, ntt_stream_t stream) {
  if (!plan || !result || !operand) return NTT_EINVAL_POINTER;
  ntt_status st = fwd ? check_fwd_factors(in_f, out_f) : check_inv_factors(in_f, out_f);
  if (st) return st;
  st = check_alias(result, operand, plan->N * sizeof(uint64_t));
  if (st) return st;
  st = check_range(operand, 64, plan->N, &plan->q, 1, 1, in_f, (hipStream_t)stream);
  if (st) return st;
  const ntt_plan* plans[1] = {plan};
  NttLaunch l{result, operand, nullptr, nullptr, plans, 1, 1, (uint32_t)in_f, (uint32_t)out_f, (hipStream_t)stream};
  return fwd ? launch_forward(l) : launch_inverse(l);
}

ntt_status ntt_forward_plan(const ntt_plan* plan, uint64_t* result, const uint64_t* operand,
                            uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream) {
  return single_plan_call(true, plan, result, operand, input_mod_factor, output_mod_factor, stream);
}

ntt_status ntt_inverse_plan(const ntt_plan* plan, uint64_t* result, const uint64_t* operand,
                            uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream) {
  return single_plan_call(false, plan, result, operand, input_mod_factor, output_mod_factor, stream);
}

ntt_status ntt_forward(uint64_t* result, const uint64_t* operand, uint64_t N, uint64_t q,
                       uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream) {
  return ntt_rns(true, result, operand, nullptr, nullptr, N, &q, 1, 1, input_mod_factor, output_mod_factor, stream);
}

ntt_status ntt_inverse(uint64_t* result, const uint64_t* operand, uint64_t N, uint64_t q,
                       uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream) {
  return ntt_rns(false, result, operand, nullptr, nullptr, N, &q, 1, 1, input_mod_factor, output_mod_factor, stream);
}

ntt_status eltwise_mult_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t n,
                            uint64_t modulus, uint64_t input_mod_factor, ntt_stream_t stream) {
  return elt_rns(true, result, operand1, operand2, n, &modulus, 1, 1, input_mod_factor, stream);
}

ntt_status eltwise_add_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t n,
                           uint64_t modulus, ntt_stream_t stream) {
  return elt_rns(false, result, operand1, operand2, n, &modulus, 1, 1, 1, stream);
}

ntt_status eltwise_fma_mod(uint64_t* result, const uint64_t* arg1, uint64_t arg2, const uint64_t* arg3, uint64_t n,
                           uint64_t modulus, uint64_t input_mod_factor, ntt_stream_t stream) {
  return fma_rns(result, arg1, &arg2, arg3, n, &modulus, 1, 1, input_mod_factor, stream);
}

ntt_status eltwise_fma_mod_rns(uint64_t* result, const uint64_t* arg1, const uint64_t* arg2, const uint64_t* arg3,
                               uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               uint64_t input_mod_factor, ntt_stream_t stream) {
  return fma_rns(result, arg1, arg2, arg3, N, moduli, num_limbs, num_polys, input_mod_factor, stream);
}

ntt_status eltwise_sub_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t n,
                           uint64_t modulus, ntt_stream_t stream) {
  return sub_rns(false, result, operand1, operand2, n, &modulus, 1, 1, stream);
}

ntt_status eltwise_negate_mod(uint64_t* result, const uint64_t* operand, uint64_t n, uint64_t modulus,
                              ntt_stream_t stream) {
  return sub_rns(true, result, operand, nullptr, n, &modulus, 1, 1, stream);
}

ntt_status ntt_forward_rns(uint64_t* result, const uint64_t* operand, uint64_t N, const uint64_t* moduli,
                           uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                           uint64_t output_mod_factor, ntt_stream_t stream) {
  return ntt_rns(true, result, operand, nullptr, nullptr, N, moduli, num_limbs, num_polys, input_mod_factor,
                 output_mod_factor, stream);
}

ntt_status ntt_inverse_rns(uint64_t* result, const uint64_t* operand, uint64_t N, const uint64_t* moduli,
                           uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                           uint64_t output_mod_factor, ntt_stream_t stream) {
  return ntt_rns(false, result, operand, nullptr, nullptr, N, moduli, num_limbs, num_polys, input_mod_factor,
                 output_mod_factor, stream);
}

ntt_status eltwise_mult_mod_rns(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t N,
                                const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                uint64_t input_mod_factor, ntt_stream_t stream) {
  return elt_rns(true, result, operand1, operand2, N, moduli, num_limbs, num_polys, input_mod_factor, stream);
}

ntt_status eltwise_add_mod_rns(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t N,
                               const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               ntt_stream_t stream) {
  return elt_rns(false, result, operand1, operand2, N, moduli, num_limbs, num_polys, 1, stream);
}

static bool is_one_pass(uint64_t N) {
  int logN = 0;
  while ((1ull << logN) < N) ++logN;
  return pass_count(logN) == 1;
}

ntt_status ntt_forward_mul_rns(uint64_t* result, const uint64_t* operand, const uint64_t* multiplier, uint64_t N,
                               const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               uint64_t input_mod_factor, uint64_t* workspace, ntt_stream_t stream) {
  if (!result || !operand || !multiplier) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 40) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  st = check_alias(result, multiplier, bytes);
  if (st) return st;
  st = check_alias(result, operand, bytes);
  if (st) return st;
  const bool one_pass = is_one_pass(N);
  if (!one_pass) {
    if (!workspace) return NTT_EINVAL_POINTER;
    if (overlaps(workspace, bytes, result, bytes) || overlaps(workspace, bytes, operand, bytes) ||
        overlaps(workspace, bytes, multiplier, bytes))
      return NTT_EALIAS;
  }
  return ntt_rns(true, result, operand, multiplier, one_pass ? nullptr : workspace, N, moduli, num_limbs, num_polys,
                 input_mod_factor, 4, stream);
}

ntt_status ntt_inverse_acc_rns(uint64_t* acc, const uint64_t* operand, uint64_t N, const uint64_t* moduli,
                               uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor, uint64_t* workspace,
                               ntt_stream_t stream) {
  if (!acc || !operand) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 40) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  if (overlaps(acc, bytes, operand, bytes)) return NTT_EALIAS;
  const bool one_pass = is_one_pass(N);
  if (!one_pass) {
    if (!workspace) return NTT_EINVAL_POINTER;
    if (overlaps(workspace, bytes, acc, bytes) || overlaps(workspace, bytes, operand, bytes)) return NTT_EALIAS;
  }
  return ntt_rns(false, acc, operand, acc, one_pass ? nullptr : workspace, N, moduli, num_limbs, num_polys,
                 input_mod_factor, 1, stream);
}

ntt_status poly_mul_rns(uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                        const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys, uint64_t* workspace,
                        ntt_stream_t stream) {
  if (!result || !a || !b) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 40) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  if (overlaps(result, bytes, b, bytes)) return NTT_EALIAS;
  st = check_alias(result, a, bytes);
  if (st) return st;
  const bool one_pass = is_one_pass(N);
  if (!one_pass) {
    if (!workspace) return NTT_EINVAL_POINTER;
    if (overlaps(workspace, bytes, a, bytes) || overlaps(workspace, bytes, b, bytes) ||
        overlaps(workspace, bytes, result, bytes))
      return NTT_EALIAS;
  }
  // result <- NTT(a) in [0, 4q)
  st = ntt_rns(true, result, a, nullptr, nullptr, N, moduli, num_limbs, num_polys, 1, 4, stream);
  if (st) return st;
  // on chip: result <- InvNTT(NTT(b) (.) result) in one launch
  if (one_pass) return product_rns(false, result, b, result, N, moduli, num_limbs, num_polys, stream);
  // result <- NTT(b) (.) result, canonical (last pass of forward(b) fused with the multiply, factor 4)
  st = ntt_rns(true, result, b, result, one_pass ? nullptr : workspace, N, moduli, num_limbs, num_polys, 1, 4,
               stream);
  if (st) return st;
  // result <- InvNTT(result), canonical
  return ntt_rns(false, result, result, nullptr, nullptr, N, moduli, num_limbs, num_polys, 1, 1, stream);
}

}  // extern "C"

// ---- poly_mul_rns without allocation -----------------------------------------
// The workspace of N > 2^14 products (the first pass of forward(b)) lives in a
// file-scope device array instead of a caller's buffer.  Its device address is
// taken once per device (hipGetSymbolAddress with that device current) and
// kept; the array's name is only a host-side stand-in for it.
namespace nttamd {
constexpr uint64_t kScratchWords = 4ull << 20;            // 32 MiB per GPU
__device__ __align__(256) uint64_t scratch[kScratchWords];
}  // namespace nttamd

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_dev[kScratchDevices];                 // device address of `scratch`, per device

ntt_status scratch_address(uint64_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return NTT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(nttamd::scratch)) != hipSuccess || !p) return NTT_EDEVICE;
    g_scratch_dev[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_scratch_dev[dev];
  return NTT_OK;
}
}  // namespace

extern "C" {

ntt_status poly_mul_rns_noalloc(uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                                const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                ntt_stream_t stream) {
  if (!result || !a || !b || !moduli) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_limbs > NTT_MAX_LIMBS || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 40) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  if (overlaps(result, bytes, b, bytes)) return NTT_EALIAS;
  st = check_alias(result, a, bytes);
  if (st) return st;
  const bool one_pass = is_one_pass(N);
  if (!one_pass && bytes > kScratchWords * sizeof(uint64_t)) return NTT_EINVAL_COUNT;   // beyond the scratch
  const ntt_plan* plans[NTT_MAX_LIMBS];
  for (uint64_t l = 0; l < num_limbs; ++l) {
    st = find_cached_plan(N, moduli[l], &plans[l]);
    if (st) return st;
  }
  uint64_t* ws = nullptr;
  if (!one_pass) {
    st = scratch_address(&ws);
    if (st) return st;
  }
  const hipStream_t s = (hipStream_t)stream;
  // the same launches as poly_mul_rns
  NttLaunch l{result, a, nullptr, nullptr, plans, (uint32_t)num_limbs, num_polys, 1, 4, s};
  st = launch_forward(l);                                  // result <- NTT(a), [0, 4q)
  if (st) return st;
  if (one_pass) {
    NttLaunch p{result, b, result, nullptr, plans, (uint32_t)num_limbs, num_polys, 1, 1, s};
    return launch_product(p, false);                       // result <- InvNTT(NTT(b) (.) result) on chip
  }
  l.in = b;
  l.mul_into = result;
  l.tmp = ws;
  st = launch_forward(l);                                  // result <- NTT(b) (.) result, canonical
  if (st) return st;
  l.in = result;
  l.mul_into = nullptr;
  l.tmp = nullptr;
  l.out_f = 1;
  return launch_inverse(l);                                // result <- InvNTT(result)
}

ntt_status poly_mul_acc_rns(uint64_t* acc, const uint64_t* a, const uint64_t* b, uint64_t N,
                            const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys, uint64_t* workspace,
                            ntt_stream_t stream) {
  if (!acc || !a || !b || !workspace) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 39) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  const bool one_pass = is_one_pass(N);
  const size_t wbytes = one_pass ? bytes : 2 * bytes;
  if (overlaps(acc, bytes, a, bytes) || overlaps(acc, bytes, b, bytes) || overlaps(workspace, wbytes, acc, bytes) ||
      overlaps(workspace, wbytes, a, bytes) || overlaps(workspace, wbytes, b, bytes))
    return NTT_EALIAS;
  uint64_t* prod = workspace;
  uint64_t* mid = one_pass ? nullptr : workspace + bytes / sizeof(uint64_t);
  // prod <- NTT(a), lazy
  st = ntt_rns(true, prod, a, nullptr, nullptr, N, moduli, num_limbs, num_polys, 1, 4, stream);
  if (st) return st;
  // on chip: acc <- acc + InvNTT(NTT(b) (.) prod) in one launch
  if (one_pass) return product_rns(true, acc, b, prod, N, moduli, num_limbs, num_polys, stream);
  // prod <- NTT(b) (.) prod, canonical
  st = ntt_rns(true, prod, b, prod, mid, N, moduli, num_limbs, num_polys, 1, 4, stream);
  if (st) return st;
  // acc <- acc + InvNTT(prod); the inverse's intermediate passes run in place on prod
  return ntt_rns(false, acc, prod, acc, one_pass ? nullptr : prod, N, moduli, num_limbs, num_polys, 1, 1, stream);
}

ntt_status poly_mul_acc_ntt_rns(uint64_t* acc, const uint64_t* a_ntt, const uint64_t* b, uint64_t N,
                                const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys, uint64_t* workspace,
                                ntt_stream_t stream) {
  if (!acc || !a_ntt || !b) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 39) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint64_t));
  if (overlaps(acc, bytes, a_ntt, bytes) || overlaps(acc, bytes, b, bytes)) return NTT_EALIAS;
  if (is_one_pass(N)) return product_rns(true, acc, b, a_ntt, N, moduli, num_limbs, num_polys, stream);
  if (!workspace) return NTT_EINVAL_POINTER;
  const size_t wbytes = 2 * bytes;
  if (overlaps(workspace, wbytes, acc, bytes) || overlaps(workspace, wbytes, a_ntt, bytes) ||
      overlaps(workspace, wbytes, b, bytes))
    return NTT_EALIAS;
  uint64_t* prod = workspace;
  uint64_t* mid = workspace + bytes / sizeof(uint64_t);
  // prod <- NTT(b) (.) a_ntt, canonical; then acc <- acc + InvNTT(prod)
  st = ntt_rns(true, prod, b, a_ntt, mid, N, moduli, num_limbs, num_polys, 1, 4, stream);
  if (st) return st;
  return ntt_rns(false, acc, prod, acc, prod, N, moduli, num_limbs, num_polys, 1, 1, stream);
}

ntt_status ntt_forward_rns32(uint32_t* result, const uint32_t* operand, uint64_t N, const uint64_t* moduli,
                             uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                             uint64_t output_mod_factor, ntt_stream_t stream) {
  ntt_status st = check_fwd_factors(input_mod_factor, output_mod_factor);
  if (st) return st;
  if (num_limbs && num_polys && N && num_polys <= (1ull << 40) / (num_limbs * N)) {
    st = check_alias(result, operand, (size_t)(num_polys * num_limbs * N * sizeof(uint32_t)));
    if (st) return st;
  }
  return small_call(output_mod_factor == 1 ? kSmallForwardCanon : kSmallForwardLazy, result, operand, nullptr, N,
                    moduli, num_limbs, num_polys, input_mod_factor, stream);
}

ntt_status ntt_inverse_rns32(uint32_t* result, const uint32_t* operand, uint64_t N, const uint64_t* moduli,
                             uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                             uint64_t output_mod_factor, ntt_stream_t stream) {
  ntt_status st = check_inv_factors(input_mod_factor, output_mod_factor);
  if (st) return st;
  if (num_limbs && num_polys && N && num_polys <= (1ull << 40) / (num_limbs * N)) {
    st = check_alias(result, operand, (size_t)(num_polys * num_limbs * N * sizeof(uint32_t)));
    if (st) return st;
  }
  return small_call(output_mod_factor == 1 ? kSmallInverseCanon : kSmallInverseLazy, result, operand, nullptr, N,
                    moduli, num_limbs, num_polys, input_mod_factor, stream);
}

// The 32-bit products' workspace: required (and checked for overlap) at N >= 2^16.
static ntt_status small_workspace(uint64_t N, const uint32_t* ws, size_t bytes, const void* x, const void* y,
                                  const void* z) {
  ntt_status st = validate_degree(N);                 // degree errors first
  if (st) return st;
  if (N <= (1ull << kMaxSmallOnePassLog)) return NTT_OK;
  if (!ws) return NTT_EINVAL_POINTER;
  if (overlaps(ws, bytes, x, bytes) || overlaps(ws, bytes, y, bytes) || overlaps(ws, bytes, z, bytes))
    return NTT_EALIAS;
  return NTT_OK;
}

ntt_status poly_mul_acc_ntt_rns32(uint32_t* acc, const uint32_t* a_ntt, const uint32_t* b, uint64_t N,
                                  const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                  uint32_t* workspace, ntt_stream_t stream) {
  if (!acc || !a_ntt || !b) return NTT_EINVAL_POINTER;
  if (num_limbs && num_polys && N && num_polys <= (1ull << 40) / (num_limbs * N)) {
    const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint32_t));
    if (overlaps(acc, bytes, a_ntt, bytes) || overlaps(acc, bytes, b, bytes)) return NTT_EALIAS;
    ntt_status st = small_workspace(N, workspace, bytes, acc, a_ntt, b);
    if (st) return st;
  }
  return small_call(kSmallProductAcc, acc, b, a_ntt, N, moduli, num_limbs, num_polys, 1, stream, workspace);
}

ntt_status poly_mul_rns32(uint32_t* result, const uint32_t* a, const uint32_t* b, uint64_t N, const uint64_t* moduli,
                          uint64_t num_limbs, uint64_t num_polys, uint32_t* workspace, ntt_stream_t stream) {
  if (!result || !a || !b) return NTT_EINVAL_POINTER;
  if (num_limbs && num_polys && N && num_polys <= (1ull << 40) / (num_limbs * N)) {
    const size_t bytes = (size_t)(num_polys * num_limbs * N * sizeof(uint32_t));
    if (overlaps(result, bytes, b, bytes)) return NTT_EALIAS;
    ntt_status st = check_alias(result, a, bytes);
    if (st) return st;
    st = small_workspace(N, workspace, bytes, result, a, b);
    if (st) return st;
  }
  // result <- NTT(a) in [0, 4q); then result <- InvNTT(NTT(b) (.) result), canonical
  ntt_status st = small_call(kSmallForwardLazy, result, a, nullptr, N, moduli, num_limbs, num_polys, 1, stream);
  if (st) return st;
  return small_call(kSmallProduct, result, b, result, N, moduli, num_limbs, num_polys, 1, stream, workspace);
}

}  // extern "C"

namespace {
// Autotuner operands: every word a hash of its index, shifted below 2^(bits - 1),
// so below every modulus of the launch (the smallest has `bits` bits): uniform
// data within the declared input range, as a real workload's.
__global__ void autotune_fill_kernel(uint64_t* buf, uint64_t words, uint32_t bits) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t z = i + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    buf[i] = (z ^ (z >> 31)) >> (65 - bits);
  }
}
}  // namespace

extern "C" {

ntt_status ntt_autotune(uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                        ntt_stream_t stream, int* choice_fwd, int* choice_inv) {
  if (!moduli) return NTT_EINVAL_POINTER;
  if (num_limbs == 0 || num_limbs > NTT_MAX_LIMBS || num_polys == 0) return NTT_EINVAL_COUNT;
  ntt_status st = validate_degree(N);
  if (st) return st;
  if (num_polys > (1ull << 36) / (num_limbs * N)) return NTT_EINVAL_COUNT;
  std::vector<const ntt_plan*> plans;
  st = rns_plans(N, moduli, num_limbs, plans);
  if (st) return st;
  const int logN = plans[0]->logN;
  const uint64_t items = num_limbs * num_polys;
  int best[2] = {0, 0};
  if (variant_count(logN) > 1) {
    // Scratch on the device for timing only (not a hot-path call): enough distinct operand
    // sets, used in turn, that the working set exceeds the 256 MB MALL as it does in a
    // streaming workload, so each variant is timed on data coming from HBM.
    const size_t bytes = (size_t)(items * N * sizeof(uint64_t));
    size_t rot = (size_t)(512ull << 20) / bytes + 1;
    rot = rot < 2 ? 2 : (rot > 32 ? 32 : rot);
    uint64_t* buf = nullptr;
    while (hipMalloc((void**)&buf, rot * bytes) != hipSuccess) {
      if (rot <= 2) return NTT_ENOMEM;
      rot /= 2;
    }
    uint32_t bits = 64;
    for (const ntt_plan* p : plans) bits = p->host_header.qbits < bits ? (uint32_t)p->host_header.qbits : bits;
    // refilled before each direction's trials: the inverse's trials need inputs below 2q
    auto fill = [&]() {
      hipLaunchKernelGGL(autotune_fill_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, buf,
                         (uint64_t)(rot * bytes / sizeof(uint64_t)), bits);
    };
    fill();
    if (hipGetLastError() != hipSuccess) { (void)hipFree(buf); return NTT_EDEVICE; }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int reps = 20;
    const int nv = variant_count(logN);
    auto run = [&](int dir, int v, int r) {
      uint64_t* x = buf + (size_t)(r % rot) * (bytes / sizeof(uint64_t));
      // operands below q, transformed in place: every value stays within the input
      // range declared here (forward inputs below 4q, inverse inputs below 2q)
      NttLaunch l{x, x, nullptr, nullptr, plans.data(), (uint32_t)num_limbs, num_polys, dir ? 4u : 2u,
                  dir ? 4u : 2u, (hipStream_t)stream};
      launch_variant(l, dir == 1, v);
    };
    // the clocks rise over the first few milliseconds of work: warm up on every variant
    // first, then take each variant's best of two rounds, so the order of the trials
    // does not favour the later ones
    for (int dir = 0; dir < 2; ++dir) {
      fill();
      for (int v = 0; v < nv; ++v)
        for (int w = 0; w < 5; ++w) run(dir, v, w);
    }
    for (int dir = 0; dir < 2; ++dir) {
      fill();
      std::vector<float> t(nv, 1e30f);
      for (int round = 0; round < 2; ++round) {
        for (int v = 0; v < nv; ++v) {
          (void)hipEventRecord(e0, (hipStream_t)stream);
          for (int r = 0; r < reps; ++r) run(dir, v, r);
          (void)hipEventRecord(e1, (hipStream_t)stream);
          (void)hipEventSynchronize(e1);
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (ms < t[v]) t[v] = ms;
        }
      }
      for (int v = 1; v < nv; ++v)
        if (t[v] < t[best[dir]]) best[dir] = v;
      set_hi_variant(dir == 1, logN, items, best[dir]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
  }
  if (choice_fwd) *choice_fwd = best[1];
  if (choice_inv) *choice_inv = best[0];
  return NTT_OK;
}

ntt_status ntt_set_variant(uint64_t N, uint64_t num_items, int forward, int variant) {
  ntt_status st = validate_degree(N);
  if (st) return st;
  int logN = 0;
  while ((1ull << logN) < N) ++logN;
  if (variant < 0 || variant >= variant_count(logN)) return NTT_EINVAL_COUNT;
  if (variant_count(logN) > 1) set_hi_variant(forward != 0, logN, num_items, variant);
  return NTT_OK;
}

}  // extern "C"
