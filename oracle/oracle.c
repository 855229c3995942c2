/*
 * Plain CPU oracle for the negacyclic NTT and the RNS element-wise kernels of
 * "Intel HEXL: Accelerating Homomorphic Encryption with Intel AVX512-IFMA52"
 * (Boemer et al., WAHC 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may include, link or
 * call this file: it exists so that tests, the smoke check and the CPU-baseline
 * leg of the benchmark have an independent, obviously correct reference.  It
 * shares no code, header, table or constant with the GPU implementation.
 *
 * Arithmetic rules:
 *   - Every modular product is the naive 128-bit product followed by `%`
 *     (Section 2.1, the "native modular multiplication" listing).  No Barrett,
 *     Shoup or Montgomery reduction is used except inside the explicitly named
 *     Harvey model below, whose purpose is to replay the paper's algorithms.
 *   - Sums of products are accumulated exactly in unsigned __int128 and reduced
 *     with `%`; the result is the exact integer sum mod q, so the order of
 *     accumulation cannot change any output.
 *
 * Definitions implemented (all from Section 2 of the paper):
 *   - element-wise add / multiply / subtract / negate and the vector-scalar
 *     fused multiply-add (Section 2, list of ring operations; Section 4
 *     free-function listing);
 *   - negacyclic product c_i = sum_{j<=i} a_j b_{i-j} - sum_{j>i} a_j b_{N+i-j}
 *     (Section 2, "vector-vector multiplication");
 *   - negacyclic forward NTT with bit-reversed output (Section 2.2: cyclic NTT
 *     of the psi-weighted input with omega = psi^2, stored at bit-reversed
 *     positions): out[i] = sum_j a_j psi^{(2 brv(i) + 1) j};
 *   - inverse: out[j] = N^{-1} sum_i A_i psi^{-(2 brv(i) + 1) j}.
 *
 * The Harvey model (or_harvey_*) runs the stages of Algorithm 2 with the
 * butterfly of Algorithm 4 and those of Algorithm 3 with the butterfly of
 * Algorithm 5 at word size beta = 2^64 (or_harvey_forward / _inverse) or
 * beta = 2^32 for moduli below 2^30 (the _w variants), to pin the lazy output
 * ranges the paper states and the representatives a word-size-beta
 * implementation produces.  Its N^{-1} step is one Shoup multiplication of each
 * [0, 2q) value (the paper leaves the representative open).  The _batch forms
 * run many limbs of one modulus over threads; or_product_batch is the
 * O(N log N) negacyclic product through these transforms, used where the
 * O(N^2) schoolbook product would take too long.
 *
 * Parity status: no function here is "parity unpinned"; every one is checked
 * by the CPU tests against closed forms, brute force, an independent big-integer
 * implementation or a second algorithm (see tests/test_oracle_*.py).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef unsigned __int128 u128;

/* ---- scalar number theory ------------------------------------------------ */

/* Native modular multiplication (Section 2.1 listing): (a * b) mod q. */
uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * b) % q);
}

uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)(a % q) + (b % q)) % q);
}

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, x = a % q;
  while (e) {
    if (e & 1) r = or_mulmod(r, x, q);
    x = or_mulmod(x, x, q);
    e >>= 1;
  }
  return r;
}

/* Inverse of a modulo a prime q (Fermat). */
uint64_t or_invmod(uint64_t a, uint64_t q) { return or_powmod(a, q - 2, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases decide every
 * n < 3.3e24 (Sorenson & Webster 2015), hence every 64-bit n. */
int or_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = or_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int r = 1; r < s; ++r) {
      x = or_mulmod(x, x, n);
      if (x == n - 1) { witness = 0; break; }
    }
    if (witness) return 0;
  }
  return 1;
}

/* Reverse the low `logn` bits of i (Section 2.2, bit-reversed ordering). */
uint64_t or_brv(uint64_t i, int logn) {
  uint64_t r = 0;
  for (int b = 0; b < logn; ++b) r |= ((i >> b) & 1u) << (logn - 1 - b);
  return r;
}

static int ilog2(uint64_t n) { int l = 0; while ((1ull << l) < n) ++l; return l; }

/* The smallest primitive 2N-th root of unity modulo the prime q, or 0 when
 * none exists (q != 1 mod 2N).  A primitive 2N-th root psi is any element with
 * psi^N = -1 (N a power of two).  One such root g is found as x^{(q-1)/2N}
 * for the first x that works; all primitive 2N-th roots are then the odd
 * powers g^k, k < 2N, and the minimum over them is returned. */
uint64_t or_min_root(uint64_t N, uint64_t q) {
  if (N == 0 || (N & (N - 1)) || q < 3 || (q - 1) % (2 * N) != 0) return 0;
  uint64_t g = 0;
  for (uint64_t x = 2; x < q; ++x) {
    uint64_t c = or_powmod(x, (q - 1) / (2 * N), q);
    if (or_powmod(c, N, q) == q - 1) { g = c; break; }
  }
  if (g == 0) return 0;
  uint64_t g2 = or_mulmod(g, g, q), cur = g, best = g;
  for (uint64_t k = 1; k < N; ++k) {          /* cur runs over g^1, g^3, ... */
    cur = or_mulmod(cur, g2, q);
    if (cur < best) best = cur;
  }
  return best;
}

/* The `count` largest primes p < 2^bits with p = 1 mod m, written in
 * descending order; returns how many were found. */
uint64_t or_find_primes(int bits, uint64_t m, uint64_t count, uint64_t* out) {
  uint64_t top = (bits >= 64) ? UINT64_MAX : ((1ull << bits) - 1);
  uint64_t p = top - (top % m) + 1;           /* largest value = 1 mod m ... */
  if (p > top) p -= m;                        /* ... not above top */
  uint64_t found = 0;
  while (found < count && p > m) {
    if (or_is_prime(p)) out[found++] = p;
    p -= m;
  }
  return found;
}

/* ---- element-wise kernels (Section 2 ring operations) -------------------- */

/* c_i = (a_i + b_i) mod q; inputs are interpreted modulo q. */
void or_eltwise_add(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q) {
  for (uint64_t i = 0; i < n; ++i) c[i] = or_addmod(a[i], b[i], q);
}

/* c_i = (a_i * b_i) mod q; inputs are interpreted modulo q. */
void or_eltwise_mult(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q) {
  for (uint64_t i = 0; i < n; ++i) c[i] = or_mulmod(a[i] % q, b[i] % q, q);
}

/* c_i = (a_i * y + z_i) mod q, the fused multiply-add of the free-function
 * listing of Section 4 (vector-scalar multiplication of Section 2 plus an
 * optional vector addition: z == NULL adds nothing).  Inputs are interpreted
 * modulo q. */
void or_eltwise_fma(uint64_t* c, const uint64_t* a, uint64_t y, const uint64_t* z, uint64_t n, uint64_t q) {
  for (uint64_t i = 0; i < n; ++i) {
    u128 v = (u128)(a[i] % q) * (y % q);
    if (z) v += z[i] % q;
    c[i] = (uint64_t)(v % q);
  }
}

/* c_i = (a_i - b_i) mod q in [0, q); inputs are interpreted modulo q. */
void or_eltwise_sub(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q) {
  for (uint64_t i = 0; i < n; ++i) c[i] = (uint64_t)(((u128)(a[i] % q) + q - (b[i] % q)) % q);
}

/* c_i = -a_i mod q in [0, q) (Section 2, element-wise negation q - a_i, with
 * the zero residue kept at 0); inputs are interpreted modulo q. */
void or_eltwise_negate(uint64_t* c, const uint64_t* a, uint64_t n, uint64_t q) {
  for (uint64_t i = 0; i < n; ++i) c[i] = (uint64_t)((q - (a[i] % q)) % q);
}

/* ---- direct O(N^2) transforms (Section 2.2 definitions) ------------------ */

typedef struct {
  uint64_t* out; const uint64_t* in; const uint64_t* idx; uint64_t count;
  uint64_t N, q; int logn; const uint64_t* pw; int inverse; uint64_t ninv;
  uint64_t lo, hi;
} job_t;

/* pw[k] = psi^k for k < 2N. */
static uint64_t* power_table(uint64_t N, uint64_t q, uint64_t psi) {
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * 2 * N);
  pw[0] = 1 % q;
  for (uint64_t k = 1; k < 2 * N; ++k) pw[k] = or_mulmod(pw[k - 1], psi, q);
  return pw;
}

/* One output coefficient of the forward or inverse transform.
 * forward: sum_j a_j psi^{(2 brv(i)+1) j}
 * inverse: N^{-1} sum_i A_i psi^{-(2 brv(i)+1) j}   (here `i` is the output
 *          index j and the sum runs over the bit-reversed input positions). */
static uint64_t direct_one(const job_t* jb, uint64_t o) {
  const uint64_t N = jb->N, q = jb->q, twoN = 2 * N;
  u128 acc = 0;
  int pending = 0;
  for (uint64_t s = 0; s < N; ++s) {
    uint64_t e;
    if (!jb->inverse) {
      e = ((2 * or_brv(o, jb->logn) + 1) * s) % twoN;         /* exponent of psi */
    } else {
      e = ((2 * or_brv(s, jb->logn) + 1) * o) % twoN;
      e = (twoN - e) % twoN;                                    /* psi^{-e} = psi^{2N-e} */
    }
    acc += (u128)(jb->in[s] % q) * jb->pw[e];                   /* each term < 2^124 */
    if (++pending == 8) { acc %= q; pending = 0; }              /* keeps acc < 2^128 */
  }
  uint64_t r = (uint64_t)(acc % q);
  if (jb->inverse) r = or_mulmod(r, jb->ninv, q);
  return r;
}

static void* direct_worker(void* arg) {
  job_t* jb = (job_t*)arg;
  for (uint64_t k = jb->lo; k < jb->hi; ++k) {
    uint64_t o = jb->idx ? jb->idx[k] : k;
    jb->out[k] = direct_one(jb, o);
  }
  return NULL;
}

static void run_direct(uint64_t* out, const uint64_t* in, const uint64_t* idx, uint64_t count,
                       uint64_t N, uint64_t q, uint64_t psi, int inverse, int nthreads) {
  uint64_t* pw = power_table(N, q, psi);
  job_t base;
  memset(&base, 0, sizeof(base));
  base.out = out; base.in = in; base.idx = idx; base.count = count; base.N = N; base.q = q;
  base.logn = ilog2(N); base.pw = pw; base.inverse = inverse;
  base.ninv = or_invmod(N % q, q);
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > count) nthreads = (int)(count ? count : 1);
  job_t* jobs = (job_t*)malloc(sizeof(job_t) * nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = base;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, direct_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th); free(jobs); free(pw);
}

/* Forward negacyclic NTT, bit-reversed output, all N outputs. */
void or_ntt_forward(uint64_t* out, const uint64_t* in, uint64_t N, uint64_t q, uint64_t psi, int nthreads) {
  run_direct(out, in, NULL, N, N, q, psi, 0, nthreads);
}
/* Inverse negacyclic NTT, bit-reversed input, natural-order output. */
void or_ntt_inverse(uint64_t* out, const uint64_t* in, uint64_t N, uint64_t q, uint64_t psi, int nthreads) {
  run_direct(out, in, NULL, N, N, q, psi, 1, nthreads);
}
/* Spot checks: out[k] = transform(in)[idx[k]] for k < count, O(count * N). */
void or_ntt_forward_at(uint64_t* out, const uint64_t* in, const uint64_t* idx, uint64_t count,
                       uint64_t N, uint64_t q, uint64_t psi, int nthreads) {
  run_direct(out, in, idx, count, N, q, psi, 0, nthreads);
}
void or_ntt_inverse_at(uint64_t* out, const uint64_t* in, const uint64_t* idx, uint64_t count,
                       uint64_t N, uint64_t q, uint64_t psi, int nthreads) {
  run_direct(out, in, idx, count, N, q, psi, 1, nthreads);
}

/* ---- schoolbook negacyclic product (Section 2, vector-vector multiply) --- */

typedef struct {
  uint64_t* c; const uint64_t* a; const uint64_t* b; const uint64_t* idx;
  uint64_t N, q, lo, hi;
} mul_job_t;

/* c_k = sum_{j<=k} a_j b_{k-j} - sum_{j>k} a_j b_{N+k-j}  (mod q) */
static uint64_t schoolbook_one(const mul_job_t* jb, uint64_t k) {
  const uint64_t N = jb->N, q = jb->q;
  u128 pos = 0, neg = 0;
  int pp = 0, pn = 0;
  for (uint64_t j = 0; j <= k; ++j) {
    pos += (u128)(jb->a[j] % q) * (jb->b[k - j] % q);
    if (++pp == 8) { pos %= q; pp = 0; }
  }
  for (uint64_t j = k + 1; j < N; ++j) {
    neg += (u128)(jb->a[j] % q) * (jb->b[N + k - j] % q);
    if (++pn == 8) { neg %= q; pn = 0; }
  }
  uint64_t p = (uint64_t)(pos % q), m = (uint64_t)(neg % q);
  return p >= m ? p - m : p + (q - m);
}

static void* schoolbook_worker(void* arg) {
  mul_job_t* jb = (mul_job_t*)arg;
  for (uint64_t t = jb->lo; t < jb->hi; ++t) {
    uint64_t k = jb->idx ? jb->idx[t] : t;
    jb->c[t] = schoolbook_one(jb, k);
  }
  return NULL;
}

static void run_schoolbook(uint64_t* c, const uint64_t* a, const uint64_t* b, const uint64_t* idx,
                           uint64_t count, uint64_t N, uint64_t q, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > count) nthreads = (int)(count ? count : 1);
  mul_job_t* jobs = (mul_job_t*)malloc(sizeof(mul_job_t) * nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) {
    mul_job_t j = {c, a, b, idx, N, q, count * t / nthreads, count * (t + 1) / nthreads};
    jobs[t] = j;
    pthread_create(&th[t], NULL, schoolbook_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th); free(jobs);
}

void or_negacyclic_mul(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t N, uint64_t q, int nthreads) {
  run_schoolbook(c, a, b, NULL, N, N, q, nthreads);
}
void or_negacyclic_mul_at(uint64_t* c, const uint64_t* a, const uint64_t* b, const uint64_t* idx,
                          uint64_t count, uint64_t N, uint64_t q, int nthreads) {
  run_schoolbook(c, a, b, idx, count, N, q, nthreads);
}

/* ---- Harvey model: the lazy transforms at word size beta ----------------- */
/* Algorithms 4 and 5 are stated for a machine word of size beta (the paper's
 * scalar path uses beta = 2^64, its IFMA path beta = 2^52).  The model takes
 * beta = 2^bits with bits = 64 or 32; beta = 2^32 requires 4q < 2^32.  All
 * "mod beta" arithmetic is unsigned arithmetic masked to bits.
 *
 * Stage structure (Section 2.2; Algorithms 2 and 3).  A length-N transform is
 * log2 N stages, one per index bit b.  The stage on bit b combines every
 * position g whose bit b is clear with its partner g + 2^b, and both
 * directions take that pair's twiddle from entry k = (N + g) >> (b + 1) of a
 * table in bit-reversed order: psi^{brv(k)} for the forward, psi^{-brv(k)} for
 * the inverse.  The forward runs its stages from the top bit down (decimation
 * in time, bit-reversed output), the inverse from bit 0 up (decimation in
 * frequency, natural-order output).  Pairs of one stage are independent, so
 * the order inside a stage does not change any value. */

static uint64_t word_mask(int bits) { return bits == 64 ? ~0ull : ((1ull << bits) - 1); }

/* W' = floor(W * beta / q) (Algorithm 4/5 requirement). */
static uint64_t shoup_precon_w(uint64_t w, uint64_t q, int bits) { return (uint64_t)(((u128)w << bits) / q); }

/* Algorithm 4: lazy forward butterfly on [0, 4q). */
static void harvey_fwd_bfly(uint64_t* x0, uint64_t* x1, uint64_t w, uint64_t wp, uint64_t q, int bits) {
  const uint64_t M = word_mask(bits);
  uint64_t X0 = *x0, X1 = *x1;
  if (X0 >= 2 * q) X0 -= 2 * q;
  uint64_t Q = (uint64_t)(((u128)wp * X1) >> bits);
  uint64_t T = (w * X1 - Q * q) & M;           /* arithmetic mod beta */
  *x0 = X0 + T;
  *x1 = X0 - T + 2 * q;
}

/* Algorithm 5: lazy inverse butterfly on [0, 2q). */
static void harvey_inv_bfly(uint64_t* x0, uint64_t* x1, uint64_t w, uint64_t wp, uint64_t q, int bits) {
  const uint64_t M = word_mask(bits);
  uint64_t X0 = *x0, X1 = *x1;
  uint64_t Y0 = X0 + X1;
  if (Y0 >= 2 * q) Y0 -= 2 * q;
  uint64_t T = X0 - X1 + 2 * q;
  uint64_t Q = (uint64_t)(((u128)wp * T) >> bits);
  *x0 = Y0;
  *x1 = (w * T - Q * q) & M;                   /* arithmetic mod beta */
}

/* Twiddles of one direction for (N, q): w[k] = r^{brv(k)} with r = psi
 * (forward) or psi^{-1} (inverse), and their companions at word size 2^bits. */
typedef struct {
  uint64_t N, q;
  int logn, bits, out_f;
  uint64_t *w, *wp;
  uint64_t ninv, ninvp;
} hv_plan_t;

static void hv_plan_init(hv_plan_t* p, uint64_t N, uint64_t q, uint64_t psi, int inverse, int out_f, int bits) {
  p->N = N; p->q = q; p->logn = ilog2(N); p->bits = bits; p->out_f = out_f;
  const uint64_t r = inverse ? or_invmod(psi, q) : psi;
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * N);      /* pw[e] = r^e, e < N */
  pw[0] = 1 % q;
  for (uint64_t e = 1; e < N; ++e) pw[e] = or_mulmod(pw[e - 1], r, q);
  p->w = (uint64_t*)malloc(sizeof(uint64_t) * N);
  p->wp = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint64_t k = 0; k < N; ++k) {
    p->w[k] = pw[or_brv(k, p->logn)];
    p->wp[k] = shoup_precon_w(p->w[k], q, bits);
  }
  free(pw);
  p->ninv = or_invmod(N % q, q);
  p->ninvp = shoup_precon_w(p->ninv, q, bits);
}

static void hv_plan_free(hv_plan_t* p) { free(p->w); free(p->wp); }

/* Forward transform of one limb in place (Algorithm 2 with Algorithm 4
 * butterflies).  Input values must be < 4q.  out_f = 4 leaves [0, 4q);
 * out_f = 1 reduces to [0, q) by conditional subtraction of 2q then q. */
static void hv_forward_limb(uint64_t* a, const hv_plan_t* p) {
  const uint64_t N = p->N, q = p->q;
  for (int b = p->logn - 1; b >= 0; --b) {
    const uint64_t half = 1ull << b;
    for (uint64_t g = 0; g < N; ++g) {
      if (g & half) continue;
      const uint64_t k = (N + g) >> (b + 1);
      harvey_fwd_bfly(&a[g], &a[g + half], p->w[k], p->wp[k], q, p->bits);
    }
  }
  if (p->out_f == 1) {
    for (uint64_t j = 0; j < N; ++j) {
      if (a[j] >= 2 * q) a[j] -= 2 * q;
      if (a[j] >= q) a[j] -= q;
    }
  }
}

/* Inverse transform of one limb in place (Algorithm 3 with Algorithm 5
 * butterflies), then each value times N^{-1} by one Shoup multiplication.
 * Input values must be < 2q.  out_f = 2 leaves [0, 2q); out_f = 1 reduces to
 * [0, q). */
static void hv_inverse_limb(uint64_t* a, const hv_plan_t* p) {
  const uint64_t N = p->N, q = p->q, M = word_mask(p->bits);
  for (int b = 0; b < p->logn; ++b) {
    const uint64_t half = 1ull << b;
    for (uint64_t g = 0; g < N; ++g) {
      if (g & half) continue;
      const uint64_t k = (N + g) >> (b + 1);
      harvey_inv_bfly(&a[g], &a[g + half], p->w[k], p->wp[k], q, p->bits);
    }
  }
  for (uint64_t j = 0; j < N; ++j) {
    uint64_t Q = (uint64_t)(((u128)p->ninvp * a[j]) >> p->bits);
    a[j] = (p->ninv * a[j] - Q * q) & M;        /* [0, 2q) */
    if (p->out_f == 1 && a[j] >= q) a[j] -= q;
  }
}

/* Work over `count` limbs of one modulus, spread over threads. */
typedef struct {
  int op;                                       /* 0 forward, 1 inverse, 2 product */
  uint64_t* a; const uint64_t* b; uint64_t* c;
  const hv_plan_t* fwd; const hv_plan_t* inv;
  uint64_t lo, hi;
} hv_job_t;

/* The negacyclic product of one limb through the transforms: the product
 * listing of Section 4 (forward of both factors, element-wise product mod q,
 * inverse), c = a * b mod (X^N + 1, q), canonical. */
static void hv_product_limb(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t* tmp,
                            const hv_plan_t* fwd, const hv_plan_t* inv) {
  const uint64_t N = fwd->N, q = fwd->q;
  for (uint64_t j = 0; j < N; ++j) { c[j] = a[j] % q; tmp[j] = b[j] % q; }
  hv_forward_limb(c, fwd);
  hv_forward_limb(tmp, fwd);
  for (uint64_t j = 0; j < N; ++j) c[j] = or_mulmod(c[j] % q, tmp[j] % q, q);
  hv_inverse_limb(c, inv);
}

static void* hv_worker(void* arg) {
  hv_job_t* jb = (hv_job_t*)arg;
  const uint64_t N = jb->fwd ? jb->fwd->N : jb->inv->N;
  uint64_t* tmp = jb->op == 2 ? (uint64_t*)malloc(sizeof(uint64_t) * N) : NULL;
  for (uint64_t l = jb->lo; l < jb->hi; ++l) {
    if (jb->op == 0) hv_forward_limb(jb->a + l * N, jb->fwd);
    else if (jb->op == 1) hv_inverse_limb(jb->a + l * N, jb->inv);
    else hv_product_limb(jb->c + l * N, jb->a + l * N, jb->b + l * N, tmp, jb->fwd, jb->inv);
  }
  free(tmp);
  return NULL;
}

static void hv_run(hv_job_t base, uint64_t count, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > count) nthreads = (int)(count ? count : 1);
  hv_job_t* jobs = (hv_job_t*)malloc(sizeof(hv_job_t) * nthreads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = base;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, hv_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th); free(jobs);
}

/* `count` limbs a[count][N] of modulus q, transformed in place at word size
 * 2^bits: forward with out_f in {1, 4}, inverse with out_f in {1, 2}. */
void or_harvey_forward_batch(uint64_t* a, uint64_t count, uint64_t N, uint64_t q, uint64_t psi, int out_f,
                             int bits, int nthreads) {
  hv_plan_t p;
  hv_plan_init(&p, N, q, psi, 0, out_f, bits);
  hv_job_t jb = {0, a, NULL, NULL, &p, NULL, 0, 0};
  hv_run(jb, count, nthreads);
  hv_plan_free(&p);
}
void or_harvey_inverse_batch(uint64_t* a, uint64_t count, uint64_t N, uint64_t q, uint64_t psi, int out_f,
                             int bits, int nthreads) {
  hv_plan_t p;
  hv_plan_init(&p, N, q, psi, 1, out_f, bits);
  hv_job_t jb = {1, a, NULL, NULL, NULL, &p, 0, 0};
  hv_run(jb, count, nthreads);
  hv_plan_free(&p);
}

/* c[l] = a[l] * b[l] mod (X^N + 1, q) for each of `count` limbs [count][N],
 * through the transforms (the product listing of Section 4), canonical; inputs
 * are interpreted mod q.  O(N log N) per limb; the schoolbook product
 * (or_negacyclic_mul) is the definition it is checked against. */
void or_product_batch(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t count, uint64_t N, uint64_t q,
                      uint64_t psi, int nthreads) {
  hv_plan_t pf, pi;
  hv_plan_init(&pf, N, q, psi, 0, 4, 64);
  hv_plan_init(&pi, N, q, psi, 1, 1, 64);
  hv_job_t jb = {2, (uint64_t*)a, b, c, &pf, &pi, 0, 0};
  hv_run(jb, count, nthreads);
  hv_plan_free(&pf);
  hv_plan_free(&pi);
}

/* Single limb at word size 2^bits (forward: values < 4q in; inverse: < 2q). */
void or_harvey_forward_w(uint64_t* a, uint64_t N, uint64_t q, uint64_t psi, int out_f, int bits) {
  or_harvey_forward_batch(a, 1, N, q, psi, out_f, bits, 1);
}
void or_harvey_inverse_w(uint64_t* a, uint64_t N, uint64_t q, uint64_t psi, int out_f, int bits) {
  or_harvey_inverse_batch(a, 1, N, q, psi, out_f, bits, 1);
}

/* The scalar path of the paper: beta = 2^64. */
void or_harvey_forward(uint64_t* a, uint64_t N, uint64_t q, uint64_t psi, int out_f) {
  or_harvey_forward_w(a, N, q, psi, out_f, 64);
}
void or_harvey_inverse(uint64_t* a, uint64_t N, uint64_t q, uint64_t psi, int out_f) {
  or_harvey_inverse_w(a, N, q, psi, out_f, 64);
}

/* One Algorithm 4 butterfly at word size 2^bits on each (x0[i], x1[i]) with
 * the same (w, w'), for brute-force checks of the butterfly alone. */
void or_harvey_fwd_bfly_w(uint64_t* x0, uint64_t* x1, uint64_t n, uint64_t w, uint64_t q, int bits) {
  const uint64_t wp = shoup_precon_w(w, q, bits);
  for (uint64_t i = 0; i < n; ++i) harvey_fwd_bfly(&x0[i], &x1[i], w, wp, q, bits);
}

/* The `count` smallest primes p in [2^(bits-1), 2^bits) with p = 1 mod m,
 * ascending; returns how many were found.  Used for edge-case moduli just
 * above a power of two. */
uint64_t or_find_primes_up(int bits, uint64_t m, uint64_t count, uint64_t* out) {
  uint64_t lo = 1ull << (bits - 1);
  uint64_t top = (bits >= 64) ? UINT64_MAX : ((1ull << bits) - 1);
  uint64_t p = lo + ((m + 1 - (lo % m)) % m);   /* smallest value >= lo that is 1 mod m */
  uint64_t found = 0;
  while (found < count && p <= top && p >= lo) {
    if (or_is_prime(p)) out[found++] = p;
    if (top - p < m) break;
    p += m;
  }
  return found;
}
