// Host-side plan construction: validation of (N, q, psi), the bit-reversed
// twiddle tables of Algorithms 2 and 3 with their Shoup companions
// (Algorithms 4 and 5), N^{-1}, and a per-device cache of plans.
#include <hip/hip_runtime.h>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace nttamd {
namespace {

typedef unsigned __int128 u128;

inline uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t pow_mod(uint64_t base, uint64_t exp, uint64_t m) {
  uint64_t result = 1 % m;
  base %= m;
  for (; exp; exp >>= 1) {
    if (exp & 1) result = mul_mod(result, base, m);
    base = mul_mod(base, base, m);
  }
  return result;
}

// One strong-probable-prime round to base a for odd n = d * 2^s + 1.
bool sprp(uint64_t n, uint64_t a, uint64_t d, int s) {
  a %= n;
  if (a == 0) return true;
  uint64_t x = pow_mod(a, d, n);
  if (x == 1 || x == n - 1) return true;
  for (int i = 1; i < s; ++i) {
    x = mul_mod(x, x, n);
    if (x == n - 1) return true;
    if (x == 1) return false;
  }
  return false;
}

uint64_t bit_reverse(uint64_t v, int bits) {
  uint64_t r = 0;
  for (int i = 0; i < bits; ++i, v >>= 1) r = (r << 1) | (v & 1);
  return r;
}

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

int log2_exact(uint64_t N) {
  int l = 0;
  while ((1ull << l) < N) ++l;
  return l;
}

// Smallest r with r^N = -1 mod q: first find one such root g, then scan the
// other N - 1 (the odd powers of g).
uint64_t smallest_root(uint64_t N, uint64_t q) {
  const uint64_t e = (q - 1) / (2 * N);
  uint64_t g = 0;
  for (uint64_t x = 2; x < q && g == 0; ++x) {
    uint64_t c = pow_mod(x, e, q);
    if (pow_mod(c, N, q) == q - 1) g = c;
  }
  if (g == 0) return 0;
  const uint64_t g2 = mul_mod(g, g, q);
  uint64_t best = g, cur = g;
  for (uint64_t k = 1; k < N; ++k) {
    cur = mul_mod(cur, g2, q);
    if (cur < best) best = cur;
  }
  return best;
}

struct CacheKey {
  int device;
  uint64_t N, q;
  bool operator<(const CacheKey& o) const { return std::tie(device, N, q) < std::tie(o.device, o.N, o.q); }
};

std::mutex g_cache_mu;
std::map<CacheKey, ntt_plan*>& cache() {
  static std::map<CacheKey, ntt_plan*> m;
  return m;
}

}  // namespace

// Deterministic for 64-bit n: bases 2..37 (the first twelve primes).
bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : small)
    if (!sprp(n, a, d, s)) return false;
  return true;
}

ntt_status validate_degree(uint64_t N) {
  if (N < 2 || N > (1ull << NTT_MAX_LOG_DEGREE) || (N & (N - 1))) return NTT_EINVAL_DEGREE;
  return NTT_OK;
}

// q < 2^62 (Algorithm 4: q < beta / 4), q = 1 mod 2N, q prime.
ntt_status validate_ntt_modulus(uint64_t N, uint64_t q) {
  if (q < 3 || q >= (1ull << 62) || (q - 1) % (2 * N) != 0) return NTT_EINVAL_MODULUS;
  if (!is_prime_u64(q)) return NTT_EINVAL_MODULUS;
  return NTT_OK;
}

// k = floor(2^L / q) with Q = bit length of q and L = 63 + Q (Algorithm 8).
uint64_t barrett_factor(uint64_t q, uint32_t* qbits) {
  uint32_t Q = 64 - (uint32_t)__builtin_clzll(q);
  if (qbits) *qbits = Q;
  // 2^(63+Q) / q = (2^(63+Q-64) * 2^64) / q; the quotient fits in 64 bits because q > 2^(Q-1).
  u128 num = (u128)1 << (63 + Q);
  return (uint64_t)(num / q);
}

ntt_status build_plan(ntt_plan** out, uint64_t N, uint64_t q, uint64_t psi) {
  if (!out) return NTT_EINVAL_POINTER;
  *out = nullptr;
  ntt_status st = validate_degree(N);
  if (st) return st;
  st = validate_ntt_modulus(N, q);
  if (st) return st;
  if (psi == 0) {
    psi = smallest_root(N, q);
    if (psi == 0) return NTT_EINVAL_MODULUS;
  } else if (psi >= q || pow_mod(psi, N, q) != q - 1) {
    return NTT_EINVAL_ROOT;
  }
  const int logN = log2_exact(N);
  const uint64_t psi_inv = pow_mod(psi, 2 * N - 1, q);

  std::vector<uint64_t> host(kPlanHeaderWords + 8 * N, 0);
  // powers psi^i and psi^-i, i < N, then the bit-reversed pair tables
  std::vector<uint64_t> pw(N), pwi(N);
  pw[0] = pwi[0] = 1;
  for (uint64_t i = 1; i < N; ++i) {
    pw[i] = mul_mod(pw[i - 1], psi, q);
    pwi[i] = mul_mod(pwi[i - 1], psi_inv, q);
  }
  uint64_t* fwd = host.data() + kPlanHeaderWords;
  uint64_t* inv = fwd + 2 * N;
  for (uint64_t k = 0; k < N; ++k) {
    const uint64_t r = bit_reverse(k, logN);
    fwd[2 * k] = pw[r];
    fwd[2 * k + 1] = shoup(pw[r], q);
    inv[2 * k] = pwi[r];
    inv[2 * k + 1] = shoup(pwi[r], q);
  }
  {
    // transposed copies of the finest stages' sub-tables (see table_perm)
    const TablePerm tp = table_perm(logN);
    const int logr = tp.logr;
    const uint64_t R = 1ull << logr, NT = N >> logr;
    for (int dir = 0; dir < 2; ++dir) {
      const uint64_t* src = fwd + dir * 2 * N;
      uint64_t* dst = fwd + 4 * N + dir * 2 * N;
      std::memcpy(dst, src, 2 * N * sizeof(uint64_t));
      const int top = dir == 0 ? tp.top_fwd : tp.top_inv;
      for (int b = 0; b <= top; ++b) {
        const uint64_t base = N >> (b + 1), S = R >> (b + 1);
        for (uint64_t t = 0; t < NT; ++t)
          for (uint64_t u = 0; u < S; ++u) {
            const uint64_t from = base + t * S + u, to = base + u * NT + t;
            dst[2 * to] = src[2 * from];
            dst[2 * to + 1] = src[2 * from + 1];
          }
      }
    }
  }
  PlanHeader h{};
  h.q = q;
  h.q2 = 2 * q;
  h.nq = (uint64_t)0 - q;
  h.N = N;
  h.ninv = pow_mod(N % q, q - 2, q);
  h.ninv_p = shoup(h.ninv, q);
  h.wn = mul_mod(inv[2 * 1], h.ninv, q);
  h.wn_p = shoup(h.wn, q);
  h.logN = (uint64_t)logN;
  uint32_t qb = 0;
  h.barrett_k = barrett_factor(q, &qb);
  h.qbits = qb;
  std::memcpy(host.data(), &h, sizeof(h));

  ntt_plan* p = new (std::nothrow) ntt_plan();
  if (!p) return NTT_ENOMEM;
  p->N = N;
  p->q = q;
  p->psi = psi;
  p->logN = logN;
  p->host_header = h;
  p->bytes = host.size() * sizeof(uint64_t);
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return NTT_EDEVICE; }
  if (hipMalloc((void**)&p->dev, p->bytes) != hipSuccess) { delete p; return NTT_ENOMEM; }
  if (hipMemcpy(p->dev, host.data(), p->bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->dev);
    delete p;
    return NTT_EDEVICE;
  }
  *out = p;
  return NTT_OK;
}

ntt_status cached_plan(uint64_t N, uint64_t q, const ntt_plan** out) {
  ntt_status st0 = validate_degree(N);
  if (st0) return st0;
  if (q < 3 || q >= (1ull << 62) || (q - 1) % (2 * N) != 0) return NTT_EINVAL_MODULUS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_EDEVICE;
  CacheKey key{dev, N, q};
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = cache().find(key);
    if (it != cache().end()) { *out = it->second; return NTT_OK; }
  }
  ntt_plan* p = nullptr;
  ntt_status st = build_plan(&p, N, q, 0);   // built outside the lock: may take milliseconds
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto ins = cache().emplace(key, p);
  if (!ins.second) {                          // another thread won the race
    (void)hipFree(p->dev);
    delete p;
  }
  *out = ins.first->second;
  return NTT_OK;
}

ntt_status find_cached_plan(uint64_t N, uint64_t q, const ntt_plan** out) {
  ntt_status st0 = validate_degree(N);
  if (st0) return st0;
  if (q < 3 || q >= (1ull << 62) || (q - 1) % (2 * N) != 0) return NTT_EINVAL_MODULUS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NTT_EDEVICE;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = cache().find(CacheKey{dev, N, q});
  if (it == cache().end()) return NTT_ENOTFOUND;
  *out = it->second;
  return NTT_OK;
}

void clear_plan_cache() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : cache()) {
    (void)hipFree(kv.second->dev);
    delete kv.second;
  }
  cache().clear();
}

}  // namespace nttamd
