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
//   [16 + 4N, 16 + 8N)      the same two tables with the sub-tables of the
//                           finest stages transposed, see table_perm()
struct PlanHeader {
  uint64_t q, q2, nq, N;      // q, 2q, 2^64 - q, degree
  uint64_t ninv, ninv_p;      // N^{-1} mod q and floor(N^{-1} 2^64 / q)
  uint64_t wn, wn_p;          // psi^-brv(1) * N^{-1} mod q and its companion
  uint64_t logN, qbits, barrett_k, reserved[5];
};
static_assert(sizeof(PlanHeader) == 16 * 8, "plan header is 16 words");
constexpr int kPlanHeaderWords = 16;

// Geometry of the single-pass (on-chip) transform, shared by the plan builder
// and the kernels.  Each thread holds 2^onchip_logr(logN) coefficients.
constexpr int kMaxOnchipLog = 14;
__host__ __device__ constexpr int onchip_logr(int logN) { return logN <= 4 ? logN : (logN <= 12 ? 4 : 5); }
// In the round where every thread owns 2^logr consecutive coefficients, the
// stage on index bit b (b <= top) reads, for thread t, the consecutive table
// entries (N >> (b+1)) + t*S + u, u < S = 2^(logr-1-b).  Those sub-tables are
// stored transposed, entry (N >> (b+1)) + u*(N >> logr) + t, so that the 64
// lanes of a wave read 1 KiB contiguous per instruction.  Returns top (-1: none).
// Same rule for a transform (or pass) over `logt` index bits with 2^logr
// coefficients per thread, whose forward runs from the top bit down.
__host__ __device__ constexpr int perm_top_for(bool fwd, int logt, int logr) {
  int top = logr - 2;
  if (top > logt - 1) top = logt - 1;
  if (fwd) {
    const int nr = (logt + logr - 1) / logr;
    const int first = logt - 1 - (nr - 1) * logr;   // highest bit handled by the last round
    if (first < top) top = first;
  }
  return top;
}
__host__ __device__ constexpr int onchip_perm_top(bool fwd, int logN) {
  return perm_top_for(fwd, logN, onchip_logr(logN));
}

// Two-pass schedule for 2^15 <= N <= 2^17 (the Cooley-Tukey split N = N1 N2):
// the "high" pass covers the top index bits as strided sub-transforms over
// tiles of adjacent columns, the "low" pass the bottom mp_logt_lo bits as
// contiguous blocks with 2^kMpLogrLo coefficients per thread.
constexpr int kMpLogrLo = 4;
__host__ __device__ constexpr int mp_logt_lo(int logN) { return logN == 15 ? 7 : 8; }
__host__ __device__ constexpr int mp_logt_hi(int logN) { return logN - mp_logt_lo(logN); }
__host__ __device__ constexpr int mp_perm_top(bool fwd, int logN) {
  return perm_top_for(fwd, mp_logt_lo(logN), kMpLogrLo);
}
// Which finest-stage sub-tables a plan stores transposed, and with what thread
// stride: bits 0..top, entry (N >> (b+1)) + t*S + u  ->  (N >> (b+1)) + u*(N >> logr) + t.
struct TablePerm {
  int logr, top_fwd, top_inv;
};
__host__ __device__ constexpr TablePerm table_perm(int logN) {
  return logN <= kMaxOnchipLog ? TablePerm{onchip_logr(logN), onchip_perm_top(true, logN), onchip_perm_top(false, logN)}
                               : TablePerm{kMpLogrLo, mp_perm_top(true, logN), mp_perm_top(false, logN)};
}

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
// The cached plan for (current device, N, q) without building one: NTT_ENOTFOUND
// when no earlier call has created it.  Allocates nothing.
ntt_status find_cached_plan(uint64_t N, uint64_t q, const ntt_plan** out);
uint64_t barrett_factor(uint64_t q, uint32_t* qbits);

// One limb task of the persistent batch kernel (ntt_batch.hip).
struct BatchTask {
  uint64_t* out;
  const uint64_t* in;
  const uint64_t* in2;      // second product factor
  uint64_t* tmp;            // product workspace (N > 2^14)
  const uint64_t* plan;
  uint32_t logN, op;
};
enum : uint32_t { kBatchFwdLazy = 0, kBatchFwdCanon = 1, kBatchInvLazy = 2, kBatchInvCanon = 3, kBatchProduct = 4 };
// Set in BatchTask::op when the task's on-chip code (N <= 2^14) takes the
// wide-range butterflies (modulus below kWideModulusBound, switch on).
constexpr uint32_t kBatchWide = 0x100u;
constexpr uint32_t kBatchOpMask = 0xffu;
uint32_t batch_wide_flag(uint32_t logN, uint64_t q);

// Kernel launchers (ntt_kernels.hip / eltwise.hip).
struct NttLaunch {
  uint64_t* out;
  const uint64_t* in;
  const uint64_t* mul_into;     // forward: out = Barrett(NTT(in), mul_into); inverse: out = mul_into + InvNTT(in)
                                //   (mul_into may equal out)
  uint64_t* tmp;                // buffer for the intermediate passes (nullptr: out)
  const ntt_plan* const* plans; // num_limbs plans
  uint32_t num_limbs;
  uint64_t num_polys;
  uint32_t in_f, out_f;
  hipStream_t stream;
};
ntt_status launch_forward(const NttLaunch& l);
// N <= 2^14: out = InvNTT(NTT(in) (.) mul_into) canonical, or out += that (acc);
// mul_into is NTT(a) with the forward's lazy output range; out may equal mul_into.
ntt_status launch_product(const NttLaunch& l, bool acc);
int pass_count(int logN);
// autotuner hooks (ntt_kernels.hip): schedule variants of the transforms (the
// thread shapes and splits of the two-pass sizes, two thread shapes of the
// single-pass sizes 2^10 .. 2^14)
ntt_status launch_variant(const NttLaunch& l, bool fwd, int variant);
void set_hi_variant(bool fwd, int logN, uint64_t items, int variant);
int get_hi_variant(bool fwd, int logN, uint64_t items);
int variant_count(int logN);
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
  const uint64_t* scalars;       // EltwiseFMAMod: host array, one scalar per limb (else nullptr)
};
ntt_status launch_eltwise_mult(const EltLaunch& l);
ntt_status launch_eltwise_sub(const EltLaunch& l, bool negate);   // b unused when negating
ntt_status launch_eltwise_fma(const EltLaunch& l);                // b = addend or nullptr
// Persistent batch launch of already-resolved tasks (ntt_batch.hip); sorts them
// into class blocks in the context's staging buffer.
ntt_status batch_launch_tasks(ntt_batch* b, const BatchTask* tasks, size_t count, hipStream_t stream, bool graph);
// Copies of the descriptors on the context's own stream (the default) or on the launch stream.
void batch_use_copy_stream(ntt_batch* b, bool on);
ntt_status launch_eltwise_add(const EltLaunch& l);

// Word-size-2^32 transforms for moduli below 2^30 (ntt_small.hip): single pass
// up to N = 2^15, two passes at 2^16 and 2^17.
constexpr int kMaxSmallOnePassLog = 15;
constexpr int kMaxSmallLog = 17;
enum SmallOp : uint32_t {
  kSmallForwardLazy, kSmallForwardCanon, kSmallInverseLazy, kSmallInverseCanon, kSmallProduct, kSmallProductAcc
};
struct Small32Launch {
  uint32_t* out;
  const uint32_t* in;
  const uint32_t* mul;          // products: the transformed multiplier (lazy, [0, 4q))
  uint32_t* tmp;                // products at N >= 2^16: workspace of num_polys * num_limbs * N words
  const ntt_plan* const* plans; // num_limbs plans
  uint32_t num_limbs;
  uint64_t num_polys;
  int logN;
  uint32_t op;                  // SmallOp
  hipStream_t stream;
};
ntt_status launch_small(const Small32Launch& l);

// Opt-in range validation (validate.hip): with validation on, check_range returns
// NTT_ERANGE when a value of limb l is not below factor * moduli[l]; it waits for
// the stream.  Off (the default), it returns NTT_OK at once.
bool validate_enabled();
void set_validate(bool on);
void free_validate_buffers();
// One-shot batch calls (ntt_batch.hip): per-thread contexts, freed by ntt_shutdown.
ntt_status oneshot_run(const ntt_batch_item* items, size_t count, ntt_stream_t stream, uint32_t op_a,
                       uint32_t op_b);
void free_oneshot_batches();
ntt_status check_range(const void* data, int bits, uint64_t n, const uint64_t* moduli, uint64_t num_limbs,
                       uint64_t num_polys, uint64_t factor, hipStream_t stream);
// Wide-range butterflies in the single-pass kernels (ntt_kernels.hip): used for
// launches whose moduli are all below kWideModulusBound while enabled (the default).
constexpr uint64_t kWideModulusBound = 1ull << 58;
bool wide_range_enabled();
void set_wide_range(bool on);

}  // namespace nttamd
