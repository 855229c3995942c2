/*
 * ntt_hip.h -- C ABI of the MI355X (gfx950) negacyclic NTT library.
 *
 * The operations are those of "Intel HEXL: Accelerating Homomorphic Encryption
 * with Intel AVX512-IFMA52" (Boemer, Kim, Seifu, de Souza, Gopal, WAHC 2021):
 * the forward and inverse negacyclic number-theoretic transform over
 * Z_q[X]/(X^N + 1) (Section 2.2, Algorithms 2-5, NTT class listing of
 * Section 4) and the element-wise modular add and multiply on RNS limbs
 * (Section 2 ring operations, free-function listing of Section 4,
 * Algorithm 8).  Every call is exact unsigned 64-bit integer arithmetic.
 *
 * Conventions shared by every entry point
 *   - Data pointers are DEVICE pointers owned by the caller, 8-byte aligned
 *     (256-byte alignment is recommended).  The library never frees them.
 *   - Calls are asynchronous: work is enqueued on `stream` (NULL = the
 *     device's default stream) on the device that is current for the calling
 *     host thread, and the call returns.  The status reports argument errors
 *     and launch failures only; execution completes at the caller's next
 *     synchronisation with the stream.
 *   - result == operand (exactly the same pointer) runs in place, as the
 *     paper's product listing does.  Any other overlap of an output with an
 *     input is rejected with NTT_EALIAS.
 *   - Operand values must lie in [0, input_mod_factor * q).  This is a
 *     precondition and is not checked on the hot path; values outside the
 *     range give unspecified (but memory-safe) results.
 *   - Host-side twiddle tables ("plans") are built once per (device, N, q,
 *     root) and cached; the first call with a new modulus allocates and
 *     uploads them.  No call allocates memory once its plans exist.
 *   - Thread safety: every entry point may be called concurrently from
 *     several host threads; plans are immutable after creation.
 *   - Errors never throw across the ABI; they are returned as negative
 *     ntt_status values.
 */
#ifndef NTT_HIP_H
#define NTT_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int ntt_status;

#define NTT_OK 0
#define NTT_EINVAL_DEGREE (-1)   /* N not a power of two, or outside [2, 2^17]        */
#define NTT_EINVAL_MODULUS (-2)  /* q not prime, q != 1 mod 2N, or q outside its range */
#define NTT_EINVAL_ROOT (-3)     /* root_of_unity is not a primitive 2N-th root mod q  */
#define NTT_EINVAL_FACTOR (-4)   /* input/output mod factor outside the allowed set    */
#define NTT_EINVAL_POINTER (-5)  /* a required pointer is NULL                         */
#define NTT_EALIAS (-6)          /* an output partially overlaps an input              */
#define NTT_EINVAL_COUNT (-7)    /* a length, limb or polynomial count is invalid      */
#define NTT_EDEVICE (-8)         /* the HIP runtime reported an error                  */
#define NTT_ENOMEM (-9)          /* device or host allocation failed                   */
#define NTT_ENOTFOUND (-10)      /* unknown handle / nothing to report                 */
#define NTT_EBUSY (-11)          /* admission refused: budget or queue full            */
#define NTT_ETIMEDOUT (-12)      /* a wait ended before the awaited work completed     */
#define NTT_ERANGE (-13)         /* validation mode: an operand value is out of range  */

/* Largest ring degree and limb count the kernels are built for. */
#define NTT_MAX_LOG_DEGREE 17
#define NTT_MAX_LIMBS 64

/* Same type as hipStream_t, declared without the HIP headers. */
typedef struct ihipStream_t* ntt_stream_t;

/* Human-readable text for a status code (static storage, never NULL). */
const char* ntt_status_string(ntt_status status);

/* Releases every cached plan and library-owned device buffer.  Calls made
 * afterwards rebuild what they need.  Must not race with other calls. */
ntt_status ntt_shutdown(void);

/* Validation mode (a debugging aid).  Operand values outside the range a call
 * states ([0, f q) for the call's input factor f, limb by limb) are a
 * precondition violation: the output is unspecified and, by default, nothing
 * checks them.  With validation on, every call that reads operand values first
 * checks them on the device, waits for the stream, and returns NTT_ERANGE
 * without launching the operation when one is out of range.  It is on when
 * the environment variable NTT_VALIDATE is "1" at the first call, or after
 * ntt_set_validate(1); ntt_set_validate(0) turns it off.  Not for timing or
 * for calls captured into a graph (it synchronises the stream).  The batch
 * calls check each item, ntt_server_submit checks a and b. */
ntt_status ntt_set_validate(int on);
int ntt_get_validate(void);

/* Wide-range butterflies (on by default).  For N <= 2^14 and launches whose
 * moduli are all below 2^58, the transforms (and the fused products built on
 * them) use a cheaper form of the butterflies of Algorithms 4 and 5: the
 * Shoup quotient omits its lowest partial product (so it may be one short and
 * W X mod q is left in [0, 3q)), and the forward lets values grow by up to 3q
 * a stage instead of reducing them to [0, 2q), with one reduction after the
 * last stage.  Values stay below 2^64 because q < 2^58.  Canonical outputs are
 * identical either way; lazy outputs stay within the stated ranges and
 * congruent mod q but are not always the words Algorithms 4 and 5 produce.
 * ntt_set_wide_range(0) makes every kernel use the paper's butterflies (for
 * example, to reproduce its lazy words); it applies to calls enqueued
 * afterwards and must not race with them.  The batch calls, the server and
 * the multi-pass sizes (N >= 2^15) always use the paper's butterflies. */
ntt_status ntt_set_wide_range(int on);
int ntt_get_wide_range(void);

/* ---------------------------------------------------------------------------
 * Plans: the paper's NTT object (Section 4, NTT class listing).  A plan owns
 * the device-resident tables of one (N, q, psi): psi_rev[k] = psi^brv(k) and
 * psi^{-1}_rev[k] = psi^{-brv(k)} (Algorithms 2 and 3) with their Shoup
 * companions W' = floor(W * 2^64 / q) (Algorithms 4 and 5), N^{-1} mod q.
 *
 *   N              ring degree, a power of two in [2, 2^17]
 *   q              prime modulus with q = 1 mod 2N and q < 2^62 (Algorithm 4
 *                  requires q < beta/4 with beta = 2^64)
 *   root_of_unity  a primitive 2N-th root psi of unity mod q (psi^N = -1), or
 *                  0 to use the smallest such root
 * Errors: NTT_EINVAL_DEGREE, NTT_EINVAL_MODULUS, NTT_EINVAL_ROOT,
 *         NTT_EINVAL_POINTER, NTT_ENOMEM, NTT_EDEVICE.
 * The plan belongs to the device current at creation; destroy it with
 * ntt_plan_destroy once no enqueued work uses it.
 */
typedef struct ntt_plan ntt_plan;
ntt_status ntt_plan_create(ntt_plan** plan, uint64_t N, uint64_t q, uint64_t root_of_unity);
ntt_status ntt_plan_destroy(ntt_plan* plan);
/* The root of unity psi a plan uses (0 for a NULL plan). */
uint64_t ntt_plan_root(const ntt_plan* plan);

/* ---------------------------------------------------------------------------
 * Forward negacyclic NTT of one limb (Section 2.2; Algorithm 2 with the
 * Harvey butterfly of Algorithm 4; NTT::ComputeForward of the Section 4
 * listing).
 *   result[i] = sum_j operand[j] * psi^((2*brv(i)+1)*j)  (mod q), i < N,
 * i.e. the output is in bit-reversed order.
 *   input_mod_factor   1, 2 or 4: operand values lie in [0, f*q)
 *   output_mod_factor  1 -> result in [0, q);  4 -> result in [0, 4q)
 *                      (lazy: congruent to the canonical value mod q)
 * ntt_forward uses the plan of (N, q, smallest psi) from the library cache;
 * ntt_forward_plan uses an explicit plan.
 * Lazy results are the exact words of Algorithm 4 except where the wide-range
 * butterflies run (see ntt_set_wide_range): then they are other values of the
 * same residue within the same range.
 */
ntt_status ntt_forward(uint64_t* result, const uint64_t* operand, uint64_t N, uint64_t q,
                       uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);
ntt_status ntt_forward_plan(const ntt_plan* plan, uint64_t* result, const uint64_t* operand,
                            uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);

/* ---------------------------------------------------------------------------
 * Inverse negacyclic NTT of one limb (Section 2.2; Algorithm 3 with the
 * Harvey butterfly of Algorithm 5 and the final multiplication by N^{-1};
 * NTT::ComputeInverse).  The operand is in bit-reversed order, the result in
 * natural order:
 *   result[j] = N^{-1} * sum_i operand[i] * psi^(-(2*brv(i)+1)*j)  (mod q).
 *   input_mod_factor   1 or 2
 *   output_mod_factor  1 -> [0, q);  2 -> [0, 2q) (lazy)
 */
ntt_status ntt_inverse(uint64_t* result, const uint64_t* operand, uint64_t N, uint64_t q,
                       uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);
ntt_status ntt_inverse_plan(const ntt_plan* plan, uint64_t* result, const uint64_t* operand,
                            uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);

/* ---------------------------------------------------------------------------
 * Element-wise kernels (Section 2; EltwiseMultMod / EltwiseAddMod of the
 * Section 4 free-function listing).  n is any length >= 1.
 *
 * eltwise_mult_mod: result[i] = operand1[i] * operand2[i] mod q, canonical.
 *   Inputs lie in [0, input_mod_factor * q), input_mod_factor in {1, 2, 4};
 *   q in [2, 2^62) and input_mod_factor * q < 2^63 (Algorithm 8).  Barrett
 *   reduction with Q = floor(log2 q) + 1, L = 63 + Q, followed by two
 *   conditional subtractions (one is not always enough for these Q, L).
 * eltwise_add_mod: result[i] = (operand1[i] + operand2[i]) mod q, inputs in
 *   [0, q), q in [2, 2^63 - 1].
 */
ntt_status eltwise_mult_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2,
                            uint64_t n, uint64_t modulus, uint64_t input_mod_factor, ntt_stream_t stream);
ntt_status eltwise_add_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2,
                           uint64_t n, uint64_t modulus, ntt_stream_t stream);

/* ---------------------------------------------------------------------------
 * Vector-scalar fused multiply-add: the EltwiseFMAMod free function of the
 * Section 4 listing, computed as in Algorithm 10 (inputs reduced to [0, q),
 * Shoup product with the scalar's precomputed companion, then the addition):
 *   result[i] = (arg1[i] * arg2 + arg3[i]) mod q, canonical in [0, q).
 * arg3 may be NULL (no addition).  arg1 and arg3 values in
 * [0, input_mod_factor * q), input_mod_factor in {1, 2, 4, 8}
 * (NTT_EINVAL_FACTOR otherwise); modulus in [2, 2^61 - 1] (NTT_EINVAL_MODULUS);
 * the scalar is taken modulo q.  result may equal arg1 and/or arg3 exactly.
 * eltwise_fma_mod_rns: the same on num_polys x num_limbs limbs of N elements
 * ([(p L + l) N + i]); arg2 is a host array of num_limbs scalars (one per
 * limb), moduli a host array of num_limbs moduli.
 */
ntt_status eltwise_fma_mod(uint64_t* result, const uint64_t* arg1, uint64_t arg2, const uint64_t* arg3, uint64_t n,
                           uint64_t modulus, uint64_t input_mod_factor, ntt_stream_t stream);
ntt_status eltwise_fma_mod_rns(uint64_t* result, const uint64_t* arg1, const uint64_t* arg2, const uint64_t* arg3,
                               uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               uint64_t input_mod_factor, ntt_stream_t stream);

/* Element-wise subtraction and negation (Section 2 ring operations):
 *   eltwise_sub_mod:    result[i] = (operand1[i] - operand2[i]) mod q,
 *   eltwise_negate_mod: result[i] = (q - operand[i]) mod q (0 stays 0),
 * operands in [0, q), results canonical; modulus in [2, 2^63 - 1].  result may
 * equal an operand exactly. */
ntt_status eltwise_sub_mod(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2, uint64_t n,
                           uint64_t modulus, ntt_stream_t stream);
ntt_status eltwise_negate_mod(uint64_t* result, const uint64_t* operand, uint64_t n, uint64_t modulus,
                              ntt_stream_t stream);

/* ---------------------------------------------------------------------------
 * RNS batches (Section 5: a polynomial modulo Q = q_0 ... q_{L-1} is held as
 * L residue polynomials, one per word-sized prime, processed limb by limb).
 * Layout: num_polys polynomials, each num_limbs limbs of N coefficients,
 * limb-major and contiguous: element (p, l, i) is at [(p*num_limbs + l)*N + i].
 * `moduli` is a HOST array of num_limbs primes (limb l uses moduli[l]; every
 * prime must satisfy the single-limb conditions for N).  Each call is one
 * batched launch sequence over all num_polys * num_limbs limbs; semantics per
 * limb are exactly those of the single-limb calls above.
 *   num_limbs in [1, NTT_MAX_LIMBS], num_polys >= 1.
 */
ntt_status ntt_forward_rns(uint64_t* result, const uint64_t* operand, uint64_t N,
                           const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                           uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);
ntt_status ntt_inverse_rns(uint64_t* result, const uint64_t* operand, uint64_t N,
                           const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                           uint64_t input_mod_factor, uint64_t output_mod_factor, ntt_stream_t stream);
ntt_status eltwise_mult_mod_rns(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2,
                                uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                uint64_t input_mod_factor, ntt_stream_t stream);
ntt_status eltwise_add_mod_rns(uint64_t* result, const uint64_t* operand1, const uint64_t* operand2,
                               uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               ntt_stream_t stream);

/* Negacyclic product of RNS polynomials: result = a * b mod (X^N + 1, q_l)
 * per limb (Section 2 vector-vector multiplication), computed as in the
 * Section 4 input_mod_factor listing: forward(a, 1 -> 4), forward(b, 1 -> 4),
 * element-wise multiply with input factor 4, inverse (1 -> 1).  The last pass
 * of the forward transform of b is fused with the element-wise multiply.
 *   a, b       canonical inputs in [0, q_l), left unchanged
 *   result     canonical output; may equal a (in place), must not overlap b
 *   workspace  device buffer of num_polys * num_limbs * N words holding the
 *              intermediate passes of forward(b); may be NULL when N <= 2^13
 *              (one on-chip pass per transform), required otherwise
 *              (NTT_EINVAL_POINTER).  Must not overlap a, b or result. */
ntt_status poly_mul_rns(uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                        const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                        uint64_t* workspace, ntt_stream_t stream);

/* Cross-kernel fusions of the product pipeline (the paper's conclusion names
 * fusing sequences of its kernels as future work).  Same layouts and limits
 * as the RNS calls above; `workspace` is a device buffer of
 * num_polys * num_limbs * N words for the intermediate passes of a multi-pass
 * transform (N > 2^14); it may be NULL when N <= 2^14.
 *
 * ntt_forward_mul_rns: result = NTT(operand) (.) multiplier  (canonical),
 *   the forward transform (Algorithm 2/4) whose last pass multiplies by the
 *   multiplier element-wise (Algorithm 8 with input factor 4).  operand in
 *   [0, f q), f in {1, 2, 4}; multiplier in [0, 4q) (typically a forward
 *   transform left lazy).  result may equal multiplier or operand.
 * ntt_inverse_acc_rns: acc = (acc + InvNTT(operand)) mod q, the inverse
 *   transform (Algorithm 3/5) whose last pass adds into a canonical
 *   accumulator (EltwiseAddMod).  operand in [0, f q), f in {1, 2}; acc must
 *   not overlap operand.
 * poly_mul_acc_rns: acc = acc + a * b  (negacyclic product per limb), as
 *   forward(a) -> forward-multiply(b) -> inverse-accumulate.  workspace is
 *   required: num_polys * num_limbs * N words for N <= 2^14, twice that above.
 */
ntt_status ntt_forward_mul_rns(uint64_t* result, const uint64_t* operand, const uint64_t* multiplier, uint64_t N,
                               const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                               uint64_t input_mod_factor, uint64_t* workspace, ntt_stream_t stream);
ntt_status ntt_inverse_acc_rns(uint64_t* acc, const uint64_t* operand, uint64_t N, const uint64_t* moduli,
                               uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                               uint64_t* workspace, ntt_stream_t stream);
/* poly_mul_rns without any allocation, for callers that cannot allocate
 * device memory at call time (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and launches as
 * poly_mul_rns, except:
 *   - the workspace of N > 2^14 is a library-owned 32 MiB device array per
 *     GPU (held until the process ends): num_polys * num_limbs * N words must
 *     fit in 2^22 (e.g. 32 limbs at N = 2^17), else NTT_EINVAL_COUNT before
 *     anything is launched;
 *   - no plan is built: every (N, q) pair must already be in the library's
 *     plan cache (created by an earlier call with it, e.g. poly_mul_rns or
 *     ntt_forward_rns), else NTT_ENOTFOUND;
 *   - the validation mode does not check its operands.
 * All calls on one GPU share that GPU's workspace, which keeps the last
 * call's contents: calls that overlap in time on one GPU (different streams
 * or host threads) race and must be ordered by the caller. */
ntt_status poly_mul_rns_noalloc(uint64_t* result, const uint64_t* a, const uint64_t* b, uint64_t N,
                                const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                ntt_stream_t stream);
ntt_status poly_mul_acc_rns(uint64_t* acc, const uint64_t* a, const uint64_t* b, uint64_t N,
                            const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                            uint64_t* workspace, ntt_stream_t stream);
/* acc += a * b with a given in NTT form: a_ntt is the forward transform of a
 * (lazy output, values in [0, 4q), e.g. from ntt_forward_rns with
 * output_mod_factor 4), b in coefficient form in [0, q); acc canonical.  For
 * N <= 2^14 this is one launch that keeps each limb on chip (forward of b,
 * multiply, inverse, accumulate; workspace may be NULL); above, the forward
 * of b fused with the multiply and the inverse fused with the accumulate,
 * with a workspace of 2 * num_polys * num_limbs * N words.  acc must not
 * overlap a_ntt or b. */
ntt_status poly_mul_acc_ntt_rns(uint64_t* acc, const uint64_t* a_ntt, const uint64_t* b, uint64_t N,
                                const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys, uint64_t* workspace,
                                ntt_stream_t stream);

/* ---- Small moduli: word size 2^32 ---------------------------------------
 * Algorithms 2-5 (Section 3) at machine word beta = 2^32 instead of 2^64, for
 * moduli q < 2^30 (so that the lazy range 4q fits a 32-bit word), prime,
 * q = 1 mod 2N, and N a power of two in [2, 2^17]: the analogue of the
 * paper's size-specialised IFMA52 path (Algorithms 6 and 7, beta = 2^52 for
 * q < 2^50).  Coefficients are uint32_t, laid out like the 64-bit calls
 * ([num_polys][num_limbs][N], limb l under moduli[l]); every product is a
 * native 32 x 32-bit multiply and every coefficient moves 4 bytes.
 *
 * Ranges and factors are those of the 64-bit calls: the forward takes inputs
 * in [0, f q), f in {1, 2, 4}, and returns [0, 4q) (output factor 4, the words
 * Algorithm 4 produces at beta = 2^32) or [0, q) (factor 1); the inverse takes
 * [0, f q), f in {1, 2}, and returns [0, 2q) or [0, q), with N^{-1} fused into
 * its last stage.  Up to N = 2^15 each call is one launch of one workgroup per
 * limb (N = 2^15 takes 132 KiB of LDS: one workgroup per CU); N = 2^16 and
 * 2^17 take two passes over HBM (the split N = N1 N2 of Section 2.2), like
 * the 64-bit calls.
 *
 * Errors: NTT_EINVAL_MODULUS for a modulus of 2^30 or more (or one that is
 * not a valid NTT prime for N), NTT_EINVAL_DEGREE for N above 2^17,
 * NTT_EINVAL_FACTOR, NTT_EINVAL_COUNT, NTT_EINVAL_POINTER, and NTT_EALIAS when
 * an output partially overlaps an input (exact in-place is allowed where the
 * 64-bit call allows it). */
ntt_status ntt_forward_rns32(uint32_t* result, const uint32_t* operand, uint64_t N, const uint64_t* moduli,
                             uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                             uint64_t output_mod_factor, ntt_stream_t stream);
ntt_status ntt_inverse_rns32(uint32_t* result, const uint32_t* operand, uint64_t N, const uint64_t* moduli,
                             uint64_t num_limbs, uint64_t num_polys, uint64_t input_mod_factor,
                             uint64_t output_mod_factor, ntt_stream_t stream);
/* result = a * b mod (X^N + 1, q_l) per limb, canonical (the product listing of
 * Section 4): forward(a) in one launch, then, up to N = 2^15, one launch that
 * keeps each limb on chip for forward(b), the Algorithm 8 multiply and the
 * inverse; at N = 2^16 and 2^17 forward(b) fused with the multiply and the
 * inverse take two passes each.  a and b in [0, q); result may equal a, not b.
 * workspace: num_polys * num_limbs * N words for the first pass of forward(b)
 * at N >= 2^16 (NTT_EINVAL_POINTER without it), ignored (may be NULL) below;
 * it must not overlap a, b or result. */
ntt_status poly_mul_rns32(uint32_t* result, const uint32_t* a, const uint32_t* b, uint64_t N, const uint64_t* moduli,
                          uint64_t num_limbs, uint64_t num_polys, uint32_t* workspace, ntt_stream_t stream);
/* acc += a * b with a given as its forward transform (a_ntt in [0, 4q), e.g.
 * ntt_forward_rns32 with output factor 4), b in [0, q), acc canonical: one
 * launch up to N = 2^15, four passes at 2^16 and 2^17 (workspace as for
 * poly_mul_rns32).  acc must not overlap a_ntt or b. */
ntt_status poly_mul_acc_ntt_rns32(uint32_t* acc, const uint32_t* a_ntt, const uint32_t* b, uint64_t N,
                                  const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                                  uint32_t* workspace, ntt_stream_t stream);

/* ---------------------------------------------------------------------------
 * Batches of limb tasks with uneven ring degrees in one persistent launch.
 * RNS polynomials of different sizes and limb counts (Section 5) are lists of
 * independent limb transforms; a batch runs any mix of them in one persistent
 * kernel launch (workgroups claim units of work from a device-side counter),
 * plus a second launch for the last pass when the batch holds transforms with
 * N >= 2^15.
 *
 * ntt_batch_item: one limb task, N in [2^10, 2^17], q its modulus (plans come
 *   from the library cache, smallest psi), device pointers to N words each:
 *     op NTT_BATCH_FWD_LAZY   out = NTT(in) in [0, 4q), in < q   (forward 1 -> 4)
 *        NTT_BATCH_FWD        out = NTT(in) canonical           (forward 1 -> 1)
 *        NTT_BATCH_INV_LAZY   out = InvNTT(in) in [0, 2q)       (inverse 1 -> 2)
 *        NTT_BATCH_INV        out = InvNTT(in) canonical        (inverse 1 -> 1)
 *        NTT_BATCH_PRODUCT    out = in * in2 mod (X^N + 1, q), canonical (the
 *                             Section 4 product listing); tmp: N-word
 *                             workspace, required for N > 2^14, else ignored
 *   out may equal in; for products out must not overlap in2 or tmp.
 *   input_mod_factor / output_mod_factor: the NTT class's factors per item
 *   (Section 4); 0 selects the op's own (input 1 for forward and product, 2
 *   for inverse; output as listed above).
 *   Forward: input 1, 2 or 4, output 1 or 4; inverse: input 1 or 2, output
 *   1 or 2; product: input 1, 2 or 4 (both factors), output 1.  A nonzero
 *   output factor decides lazy or canonical output (the op then only gives
 *   the direction); values outside these sets: NTT_EINVAL_FACTOR.  Operand
 *   values must lie below input_mod_factor * q (checked in validation mode).
 * ntt_batch_create: a reusable batch context for up to `capacity` tasks (owns
 *   pinned and device descriptor buffers; not thread-safe: one context per
 *   host thread or external locking).
 * ntt_batch_run: copies the descriptors and launches, asynchronously on
 *   `stream`.  The context holds two staging sets used in turn, so the host
 *   prepares a run while the previous one executes; a run first waits for
 *   the run two before it.  Errors: NTT_EINVAL_* for a bad task (nothing
 *   launched).
 * ntt_batch_run_graph: same work through a hipGraph (one per staging set)
 *   captured on first use:
 *   [persistent kernel, second launch for the last passes]; the graph reads
 *   the task list and counts from device memory, so it is replayed for every
 *   later batch of up to `capacity` tasks.  Each run (plain or graph) first
 *   copies its own descriptors on a stream of the context, ordered before the
 *   kernels by an event.
 * ntt_batch_set_grid: number of persistent workgroups (0 = two per CU).
 * ntt_batch_set_shape: per-limb shape of the transform units staged from then
 *   on: 0 (default) the per-call kernels' own (16 or 32 coefficients per
 *   thread, several limbs per workgroup below 2^14, tiles of 16 per thread);
 *   1 twice the threads per limb or tile (for N <= 2^13 and for the tiles of
 *   N >= 2^15; N = 2^14 transforms and products keep shape 0); 2 twice the
 *   threads per tile only (limbs as in shape 0).  Results are the same words
 *   whichever the shape.  NTT_EINVAL_COUNT for another value.
 * ntt_batch_get_config: the context's workgroup count (0 = automatic) and
 *   unit shape, as set or chosen by ntt_batch_autotune (either pointer may be
 *   NULL).
 */
typedef struct ntt_batch ntt_batch;
#define NTT_BATCH_FWD_LAZY 0u
#define NTT_BATCH_FWD 1u
#define NTT_BATCH_INV_LAZY 2u
#define NTT_BATCH_INV 3u
#define NTT_BATCH_PRODUCT 4u
typedef struct {
  uint64_t* out;
  const uint64_t* in;
  const uint64_t* in2;
  uint64_t* tmp;
  uint64_t N;
  uint64_t q;
  uint32_t op;
  uint16_t input_mod_factor;
  uint16_t output_mod_factor;
} ntt_batch_item;
ntt_status ntt_batch_create(ntt_batch** batch, size_t capacity);
ntt_status ntt_batch_destroy(ntt_batch* batch);
ntt_status ntt_batch_set_grid(ntt_batch* batch, int workgroups);
ntt_status ntt_batch_set_shape(ntt_batch* batch, int shape);
ntt_status ntt_batch_get_config(const ntt_batch* batch, int* workgroups, int* shape);
ntt_status ntt_batch_run(ntt_batch* batch, const ntt_batch_item* items, size_t count, ntt_stream_t stream);
ntt_status ntt_batch_run_graph(ntt_batch* batch, const ntt_batch_item* items, size_t count, ntt_stream_t stream);
/* Times the persistent launch of this batch with one, one and a half and two
 * workgroups per CU, each with the three unit shapes (ntt_batch_set_shape), and
 * keeps the fastest grid and shape for the context (the chosen workgroup
 * count in *chosen, may be NULL).  Runs the batch several times, so every
 * task must have out != in (NTT_EALIAS otherwise); outputs end up holding the
 * batch's result.  Synchronises `stream`. */
/* One-shot batch calls: run a task list whose items are all forward
 * (NTT_BATCH_FWD_LAZY / NTT_BATCH_FWD), all inverse (NTT_BATCH_INV_LAZY /
 * NTT_BATCH_INV) or all products (NTT_BATCH_PRODUCT); NTT_EINVAL_FACTOR for
 * an item of another kind.  They use a library-owned batch context per host
 * thread and device (grown to the largest list seen, freed by ntt_shutdown)
 * and replay its captured graph; otherwise as ntt_batch_run_graph. */
ntt_status ntt_batch_forward(const ntt_batch_item* items, size_t count, ntt_stream_t stream);
ntt_status ntt_batch_inverse(const ntt_batch_item* items, size_t count, ntt_stream_t stream);
ntt_status ntt_batch_product(const ntt_batch_item* items, size_t count, ntt_stream_t stream);
ntt_status ntt_batch_autotune(ntt_batch* batch, const ntt_batch_item* items, size_t count, ntt_stream_t stream,
                              int* chosen);

/* ---------------------------------------------------------------------------
 * Autotuning (Section 4 notes that the best implementation can be picked by
 * trying the candidates at initialisation).  For two-pass sizes (N > 2^14) the
 * library has several kernel variants per pass (thread shapes, N1 x N2 splits
 * and a three-pass split), for N = 2^10 .. 2^14 two thread shapes of the single-pass kernel
 * (variant 1 gives each limb twice the threads); this call times each, 20
 * launches per variant, on scratch operand sets of num_limbs * num_polys * N
 * words used in turn (enough sets, up to 32, that they exceed the 256 MB MALL,
 * so the data comes from HBM as in a streaming workload; allocated and freed
 * here, so it is not a hot-path call), synchronises `stream`, and uses the
 * fastest for later calls of the same direction, N and batch-size class (up to
 * 64 limbs, or more).  choice_fwd / choice_inv (may be NULL)
 * receive the chosen variant indices.  N < 2^10 has a single variant; the
 * fused products (poly_mul_*) always take the single-pass kernel's variant 0.
 * ntt_set_variant pins a variant explicitly (forward != 0 for the forward
 * transform); NTT_EINVAL_COUNT for an unknown variant.
 */
ntt_status ntt_autotune(uint64_t N, const uint64_t* moduli, uint64_t num_limbs, uint64_t num_polys,
                        ntt_stream_t stream, int* choice_fwd, int* choice_inv);
ntt_status ntt_set_variant(uint64_t N, uint64_t num_items, int forward, int variant);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of negacyclic polynomial products.
 *
 * A request asks for c = a * b in Z_q[X]/(X^N + 1) for each of its L RNS
 * limbs (the forward / multiply / inverse sequence of the paper's Section 4
 * product listing; the limbs are independent, Section 5).  The server is a
 * native scheduler thread on the device current at creation:
 *   - arrival: a request counts from its arrival time (ntt_server_now_ns
 *     clock; 0 = when submitted).  A request submitted ahead of its arrival
 *     time stays invisible to the scheduler until that time, so a load
 *     generator can hand over a pre-drawn open-loop schedule;
 *   - admission: arrived requests are admitted strictly in arrival order
 *     while the server's device arena (hbm_budget bytes, allocated once at
 *     creation) has room for the request's footprint: its result,
 *     L * N * 8 bytes, plus for N > 2^14 (and for every N in per-limb mode) a
 *     workspace of the same size (one limb's worth, N * 8, in per-limb mode).
 *     A request that does not fit waits (backpressure) until earlier requests
 *     complete and are released;
 *   - NTT_SERVE_BATCHED: every admitted request not yet launched goes into
 *     the next persistent batch launch (one task per limb product, largest
 *     first), with up to `streams` launches in flight on separate streams, so
 *     requests that arrive while others run join the next launch and its work
 *     overlaps the tail of the running one.  Requests with N at or above
 *     2^wide_min_log_degree instead run as their own three launches of the
 *     two-pass kernels (forward, forward fused with the multiply, inverse),
 *     round robin over `streams` further streams, overlapping the rest, as
 *     long as fewer than wide_max_inflight such launches per wide stream are
 *     in flight;
 *     beyond that they join the persistent launches (which pack the chip
 *     better under load);
 *   - NTT_SERVE_FIFO: each request alone, in arrival order on one stream,
 *     as three launches over its limbs (forward, forward fused with the
 *     multiply, inverse);
 *   - NTT_SERVE_FIFO_PER_LIMB: each request alone, in arrival order on one
 *     stream, one launch per limb transform and per limb multiply (the plain
 *     per-call form);
 *   - completion: a request is done when the launch that holds its last limb
 *     has completed on the device; its result (canonical, layout [L][N]) is
 *     then readable at info.result until ntt_server_release.
 * Every mode gives bit-identical results: each limb product is computed by
 * the same exact arithmetic whatever else shares the launch.
 *
 * ntt_server_create: config may be NULL (all defaults).  hbm_budget 0 = 16 GiB;
 *   streams 0 = 2 (at most 4); max_batch_tasks 0 = 4096 (at least 64);
 *   max_queue 0 = 2^20 requests submitted but not yet admitted.
 *   release_on_completion != 0 returns a request's arena space as soon as it
 *   completes (for load generation: the result is then not kept).
 *   NTT_EINVAL_COUNT for a mode, stream count, task cap, wide_min_log_degree
 *   (10..18) or wide_max_inflight out of range.
 * ntt_server_submit: validates and queues; plans for new (N, q) are built on
 *   the calling thread, which must have the server's device current
 *   (NTT_EDEVICE otherwise).  Errors: NTT_EINVAL_POINTER (null a, b, moduli,
 *   ticket), NTT_EINVAL_DEGREE (N not a power of two in [2^10, 2^17]),
 *   NTT_EINVAL_COUNT (num_limbs outside [1, 64]), NTT_EINVAL_MODULUS (a limb
 *   modulus not prime, not 1 mod 2N, or >= 2^62), NTT_ENOMEM (the footprint
 *   exceeds the whole budget, so the request could never be admitted),
 *   NTT_EBUSY (queue full, or the server is shutting down).  a and b are
 *   device arrays [L][N] with limb l's values in [0, q_l); they are read-only
 *   and must stay valid until the request completes.
 * ntt_server_poll / ntt_server_query: state of one / several tickets
 *   (NTT_ENOTFOUND for an unknown or released ticket).
 * ntt_server_wait: blocks until the ticket completes or fails
 *   (NTT_ETIMEDOUT after timeout_ns; < 0 waits without limit).
 * ntt_server_drain: blocks until every submitted request has completed or
 *   failed (NTT_ETIMEDOUT after timeout_ns; < 0 waits without limit).
 * ntt_server_read: enqueues on `stream` a copy of a completed request's
 *   result into dst (device, L * N words); NTT_EBUSY before completion, the
 *   request's own status if it failed, NTT_ENOTFOUND without a kept result.
 *   The server records an event after the copy on `stream`.
 * ntt_server_release: drops a completed request's record and returns its
 *   result's arena range (NTT_EBUSY while it is still queued or running).  A
 *   range read with ntt_server_read goes back to the arena only once every
 *   such copy has completed on its stream, so read-then-release needs no
 *   synchronisation in between.  Uses of info.result made by the caller's own
 *   kernels are not tracked: release after they have completed.  A request
 *   whose launch failed part way keeps its ranges until the kernels already
 *   enqueued for it have drained.
 * ntt_server_destroy: requests not yet launched fail with NTT_EBUSY, launches
 *   in flight are waited for, then the arena and streams are freed.
 */
typedef struct ntt_server ntt_server;
#define NTT_SERVE_BATCHED 0u
#define NTT_SERVE_FIFO 1u
#define NTT_SERVE_FIFO_PER_LIMB 2u
typedef struct {
  uint64_t hbm_budget;
  uint32_t mode;
  uint32_t streams;
  uint32_t max_batch_tasks;
  uint32_t max_queue;
  uint32_t release_on_completion;
  uint32_t use_graph;       /* nonzero: batched launches replay a captured hipGraph */
  uint32_t wide_min_log_degree;  /* batched mode: requests with N >= 2^this run as their own
                                    launches of the two-pass kernels on `streams` extra streams;
                                    0 = 15, 18 = never (all requests in persistent launches) */
  uint32_t wide_max_inflight;    /* such launches in flight per wide stream before further large
                                    requests join the persistent launches; 0 = 2, at most 1024 */
} ntt_server_config;
typedef struct {
  uint64_t N;
  uint64_t num_limbs;
  const uint64_t* moduli;   /* host array of num_limbs primes, copied at submission */
  const uint64_t* a;
  const uint64_t* b;
  int64_t arrival_ns;
} ntt_request;
#define NTT_REQ_WAITING 0u    /* submitted, not arrived or not admitted */
#define NTT_REQ_ADMITTED 1u   /* arena space reserved, not launched */
#define NTT_REQ_RUNNING 2u
#define NTT_REQ_DONE 3u
#define NTT_REQ_FAILED 4u
typedef struct {
  uint32_t state;
  ntt_status status;        /* NTT_OK, or why the request failed */
  uint64_t* result;         /* device [L][N], valid in state DONE until release (NULL otherwise) */
  int64_t arrival_ns, admit_ns, launch_ns, done_ns;
} ntt_request_info;
typedef struct {
  uint64_t submitted, rejected, completed, failed;
  uint64_t launches, tasks;
  uint64_t waiting, in_flight;
  uint64_t arena_bytes, arena_in_use, arena_peak;
  uint64_t deferred;        /* admissions postponed for lack of arena space */
} ntt_server_stats;
ntt_status ntt_server_create(ntt_server** server, const ntt_server_config* config);
ntt_status ntt_server_submit(ntt_server* server, const ntt_request* request, uint64_t* ticket);
ntt_status ntt_server_poll(ntt_server* server, uint64_t ticket, ntt_request_info* info);
ntt_status ntt_server_query(ntt_server* server, const uint64_t* tickets, size_t count, ntt_request_info* infos);
ntt_status ntt_server_wait(ntt_server* server, uint64_t ticket, int64_t timeout_ns, ntt_request_info* info);
ntt_status ntt_server_drain(ntt_server* server, int64_t timeout_ns);
ntt_status ntt_server_read(ntt_server* server, uint64_t ticket, uint64_t* dst, ntt_stream_t stream);
ntt_status ntt_server_release(ntt_server* server, uint64_t ticket);
ntt_status ntt_server_stats_get(ntt_server* server, ntt_server_stats* stats);
int64_t ntt_server_now_ns(void);
ntt_status ntt_server_destroy(ntt_server* server);

#ifdef __cplusplus
}
#endif
#endif /* NTT_HIP_H */
