"""CPU checks of the arithmetic claims behind the GPU kernels' wide-range butterflies.

The wide butterflies (single-pass kernels, moduli below 2^58) take the Shoup quotient
without its lowest partial product and let forward values grow between stages.  These
tests model that arithmetic exactly with Python integers, word by word as the kernels
compute it, and check what the kernels rely on:
  - the quotient estimate is Q or Q - 1, so W X - Q' q lies in [0, 3q) for every X < 2^64;
  - the reduction by 1 (companion floor(2^64 / q)) maps any x < 2^64 into [0, 3q);
  - a whole forward transform from inputs below 4q keeps every value below 46 q < 2^64
    for q < 2^58 and N = 2^14 stages' worth of growth, and the inverse keeps [0, 4q);
  - after the final reductions both transforms equal the oracle's (Section 2.2
    definitions), so the representatives differ from Algorithms 4 and 5 only mod q.
The model is test code, not part of the oracle: it restates the kernels' arithmetic to
check the error analysis on the CPU.
"""
import numpy as np
import pytest

import oracle
from synthetic import lazy_mod, splitmix64, unit_seed

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1


def shoup_companion(w, q):
    return (w << 64) // q


def approx_quotient(wp, x):
    """MulHi(W', X) without lo(W') lo(X): the 65-bit middle sum's high part plus hi hi."""
    pl, ph = wp & M32, wp >> 32
    xl, xh = x & M32, x >> 32
    mid = pl * xh + ph * xl                      # up to 65 bits: the kernels carry bit 64 in an SGPR
    return ph * xh + (mid >> 32)


def wide_mul(w, wp, x, q):
    """T = W X - Q' q, as the low 64 bits the kernels compute; returns (T, exact value)."""
    qp = approx_quotient(wp, x)
    t_low = (w * x + qp * ((1 << 64) - q)) & M64
    return t_low, w * x - qp * q


def wide_fwd_bfly(x0, x1, w, wp, q):
    t, exact = wide_mul(w, wp, x1, q)
    assert t == exact and 0 <= exact < 3 * q
    y0, y1 = x0 + t, x0 + 3 * q - t
    assert y0 <= M64 and y1 <= M64
    return y0, y1


def wide_inv_bfly(x0, x1, w, wp, q):
    assert x0 < 4 * q and x1 < 4 * q
    s = x0 + x1
    s = s - 4 * q if s >= 4 * q else s
    d = x0 + 4 * q - x1
    t, exact = wide_mul(w, wp, d, q)
    assert t == exact and 0 <= exact < 3 * q
    return s, t


def reduce_wide(x, q):
    r = (1 << 64) // q
    qp = approx_quotient(r, x)
    y = (x + qp * ((1 << 64) - q)) & M64
    assert y == x - qp * q and 0 <= y < 3 * q
    return y


def _randint(seed, n, bound):
    w = splitmix64(seed, n).astype(object)
    return [int(v) % bound for v in w]


@pytest.mark.parametrize("bits", [2, 17, 30, 50, 57, 58])
def test_quotient_short_by_at_most_one(bits):
    """Random and extreme (W, X, q) with q below 2^bits: Q - Q' in {0, 1}, T in [0, 3q)."""
    qs = [(1 << bits) - 1 if bits > 2 else 3, (1 << (bits - 1)) + 1 if bits > 2 else 3]
    qs += [v | 1 for v in _randint(unit_seed(500, bits), 6, 1 << bits) if v > 2]
    for q in qs:
        ws = [0, 1, q - 1] + _randint(unit_seed(501, q), 40, q)
        xs = [0, 1, M64, M64 - 1, 1 << 63, (1 << 32) - 1, 1 << 32] + _randint(unit_seed(502, q), 60, 1 << 64)
        for w in ws:
            wp = shoup_companion(w, q)
            for x in xs:
                exact_q = (wp * x) >> 64
                qp = approx_quotient(wp, x)
                assert exact_q - qp in (0, 1), (q, w, x)
                t, ex = wide_mul(w, wp, x, q)
                assert t == ex and 0 <= ex < 3 * q and ex % q == (w * x) % q, (q, w, x)


def test_quotient_worst_case_brute_force_small_words():
    """Exhaustive over a small slice: every W < q for q = 97, X at the word's top and
    bottom ends and across the middle-carry boundary."""
    q = 97
    xs = [M64 - k for k in range(64)] + list(range(64)) + [(1 << 32) * k - 1 for k in range(1, 64)]
    for w in range(q):
        wp = shoup_companion(w, q)
        for x in xs:
            t, ex = wide_mul(w, wp, x, q)
            assert t == ex and 0 <= ex < 3 * q


@pytest.mark.parametrize("q", [3, 12289, (1 << 58) - 27, (1 << 50) + 1])
def test_reduce_by_one_lands_below_3q(q):
    for x in [0, 1, q - 1, q, 3 * q, 46 * q - 1, M64, M64 - q] + _randint(unit_seed(510, q), 200, 1 << 64):
        assert reduce_wide(x, q) % q == x % q


def _wide_forward_model(a, q, psi):
    """Algorithm 2's loop structure with the wide butterfly; returns the values before the
    final reduction and after it."""
    n = len(a)
    logn = n.bit_length() - 1
    tw = [pow(psi, int(oracle.brv(k, logn)), q) for k in range(n)]
    x = [int(v) for v in a]
    t, m = n, 1
    peak = 0
    while m < n:
        t //= 2
        for i in range(m):
            w = tw[m + i]
            wp = shoup_companion(w, q)
            for j in range(2 * i * t, 2 * i * t + t):
                x[j], x[j + t] = wide_fwd_bfly(x[j], x[j + t], w, wp, q)
                peak = max(peak, x[j], x[j + t])
        m *= 2
    return x, [reduce_wide(v, q) for v in x], peak


def _wide_inverse_model(A, q, psi):
    """Algorithm 3's loop structure with the wide inverse butterfly and the fused N^{-1}
    last stage; returns values in [0, 3q) and after the subtraction of 2q."""
    n = len(A)
    logn = n.bit_length() - 1
    pinv = pow(psi, q - 2, q)
    tw = [pow(pinv, int(oracle.brv(k, logn)), q) for k in range(n)]
    x = [int(v) for v in A]
    t, m = 1, n
    while m > 2:
        h = m // 2
        j1 = 0
        for i in range(h):
            w = tw[h + i]
            wp = shoup_companion(w, q)
            for j in range(j1, j1 + t):
                x[j], x[j + t] = wide_inv_bfly(x[j], x[j + t], w, wp, q)
            j1 += 2 * t
        t *= 2
        m //= 2
    ninv = pow(n, q - 2, q)
    wn = ninv * tw[1] % q
    for j in range(t):                           # last stage: both outputs times N^{-1}
        x0, x1 = x[j], x[j + t]
        assert x0 < 4 * q and x1 < 4 * q
        s, d = x0 + x1, x0 + 4 * q - x1
        y0, e0 = wide_mul(ninv, shoup_companion(ninv, q), s, q)
        y1, e1 = wide_mul(wn, shoup_companion(wn, q), d, q)
        assert y0 == e0 < 3 * q and y1 == e1 < 3 * q
        x[j], x[j + t] = y0, y1
    return x, [v - 2 * q if v >= 2 * q else v for v in x]


@pytest.mark.parametrize("logn", [1, 3, 6, 9])
def test_wide_transforms_match_the_definitions(logn):
    """Whole wide transforms at the largest prime below 2^58 that is 1 mod 2N, inputs at the
    top of their ranges and random: outputs equal the oracle's transforms mod q, the
    forward's peak stays below (4 + 3 log N) q, the final ranges are [0, 3q) and [0, 2q)."""
    n = 1 << logn
    q = oracle.find_primes(58, 2 * n, 1)[0]
    psi = oracle.min_root(n, q)
    for a in (np.full(n, 4 * q - 1, dtype=np.uint64), lazy_mod(unit_seed(520, logn), n, q, 4)):
        raw, out, peak = _wide_forward_model(a, q, psi)
        assert peak < (4 + 3 * logn) * q < (1 << 64)
        assert all(v < 3 * q for v in out)
        ref = oracle.ntt_forward(a, q, psi)
        assert [v % q for v in out] == [int(v) for v in ref]
    for A in (np.full(n, 2 * q - 1, dtype=np.uint64), lazy_mod(unit_seed(521, logn), n, q, 2)):
        _, out = _wide_inverse_model(A, q, psi)
        assert all(v < 2 * q for v in out)
        assert [v % q for v in out] == [int(v) for v in oracle.ntt_inverse(A, q, psi)]


def test_growth_bound_for_the_kernels_largest_shape():
    """The bound the kernels' host check uses: from inputs below 4q, 14 stages of growth
    below 3q each stay below 46 q, and 46 q < 2^64 for every q < 2^58 (17 stages, the
    largest transform, would give 55 q, also below 2^64)."""
    q = (1 << 58) - 1
    assert (4 + 3 * 14) * q < (1 << 64)
    assert (4 + 3 * 17) * q < (1 << 64)
    assert 8 * q < (1 << 64)                      # the inverse's S and D
