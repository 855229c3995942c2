// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <mutex>
#include <vector>

#include "../../include/ntt_hip.h"

namespace nttamd {

// Layout of a plan's device buffer (u64 words):
//   [0, 16)                 header, see PlanHeader
//   [16, 16 + 2N)           forward pairs (W, W') at index k: W = psi^brv(k)
//   [16 + 2N, 16 + 4N)      inverse pairs at index k: W = psi^-brv(k)
struct PlanHeader {
  uint64_t q, q2, nq, N;      // q, 2q, 2^64 - q, degree
  uint64_t ninv, ninv_p;      // N^{-1} mod q and floor(N^{-1} 2^64 / q)
  uint64_t wn, wn_p;          // psi^-brv(1) * N^{-1} mod q and its companion
  uint64_t logN, qbits, barrett_k, reserved[5];
};
static_assert(sizeof(PlanHeader) == 16 * 8, "plan header is 16 words");
constexpr int kPlanHeaderWords = 16;

}  // namespace nttamd

struct ntt_plan {
  uint64_t N, q, psi;
  int logN;
  int device;
  uint64_t* dev;              // device buffer, see PlanHeader
  size_t bytes;
  nttamd::PlanHeader host_header;
};

namespace nttamd {

// Host-side helpers (plan.hip).
bool is_prime_u64(uint64_t n);
ntt_status validate_degree(uint64_t N);
ntt_status validate_ntt_modulus(uint64_t N, uint64_t q);
ntt_status build_plan(ntt_plan** out, uint64_t N, uint64_t q, uint64_t psi);
// Cached plan for (current device, N, q, smallest root); never freed before ntt_shutdown.
ntt_status cached_plan(uint64_t N, uint64_t q, const ntt_plan** out);
void clear_plan_cache();
uint64_t barrett_factor(uint64_t q, uint32_t* qbits);

// Kernel launchers (ntt_kernels.hip / eltwise.hip).
struct NttLaunch {
  uint64_t* out;
  const uint64_t* in;
  const uint64_t* mul_into;     // fused forward-and-multiply: out = Barrett(NTT(in), mul_into) (may equal out)
  uint64_t* tmp;                // buffer for the intermediate passes (nullptr: out)
  const ntt_plan* const* plans; // num_limbs plans
  uint32_t num_limbs;
  uint64_t num_polys;
  uint32_t in_f, out_f;
  hipStream_t stream;
};
ntt_status launch_forward(const NttLaunch& l);
int pass_count(int logN);
ntt_status launch_inverse(const NttLaunch& l);

struct EltLaunch {
  uint64_t* out;
  const uint64_t* a;
  const uint64_t* b;
  uint64_t n;                    // elements per limb (whole vector for single-modulus calls)
  const uint64_t* moduli;        // host array, num_limbs entries
  uint32_t num_limbs;
  uint64_t num_polys;
  uint32_t in_f;
  hipStream_t stream;
};
ntt_status launch_eltwise_mult(const EltLaunch& l);
ntt_status launch_eltwise_add(const EltLaunch& l);

}  // namespace nttamd
