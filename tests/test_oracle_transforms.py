"""Pins the oracle's transforms and products (Section 2 definitions) to facts
other than their own formulas:

* exhaustive brute force on the smallest rings (N = 2, q = 5; N = 4, q = 17)
  against closed forms / polynomial evaluation;
* the forward transform evaluates the input polynomial at the N roots of
  X^N + 1 (Horner in Python big integers), in the bit-reversed order of the
  paper's Figure 1, i.e. as the cyclic NTT of the psi-weighted input with
  omega = psi^2 (Section 2.2);
* the round trip InvNTT(NTT(a)) = a and the convolution theorem
  InvNTT(NTT(a) . NTT(b)) = a * b stated in Section 2.2;
* the schoolbook product against full polynomial multiplication followed by
  reduction with X^N = -1, and against special products (by 1, by X, X^{N/2}^2);
* a second algorithm: the Harvey model (Algorithms 2+4 and 3+5) must agree with
  the direct O(N^2) sums, and stay inside the lazy ranges of Algorithms 4 and 5;
* its batched forms (many limbs of one modulus on threads, and the O(N log N)
  product through the transforms) limb by limb against the direct sums and the
  schoolbook product, plus the special products X^(N/2) X^(N/2) = -1 and a X.
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
from synthetic import lazy_mod, uniform_mod, unit_seed

HERE = os.path.dirname(os.path.abspath(__file__))


def _horner(coeffs, x, q):
    r = 0
    for c in reversed(coeffs):
        r = (r * x + int(c)) % q
    return r


def _brv(i, logn):
    return int(format(i, "0%db" % logn)[::-1], 2) if logn else 0


def _poly_mul_mod_xn1(a, b, q):
    N = len(a)
    full = [0] * (2 * N - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            full[i + j] += int(x) * int(y)
    out = [0] * N
    for k, v in enumerate(full):          # X^(N+k) = -X^k
        if k < N:
            out[k] += v
        else:
            out[k - N] -= v
    return [v % q for v in out]


def test_exhaustive_n2_q5_closed_form():
    q, N, psi = 5, 2, oracle.min_root(2, 5)
    assert psi == 2
    for a0, a1 in itertools.product(range(q), repeat=2):
        out = oracle.ntt_forward([a0, a1], q, psi, threads=1)
        assert list(out) == [(a0 + psi * a1) % q, (a0 - psi * a1) % q]
        back = oracle.ntt_inverse(out, q, psi, threads=1)
        assert list(back) == [a0, a1]


def test_exhaustive_n4_q17_polynomial_evaluation():
    q, N = 17, 4
    psi = oracle.min_root(N, q)
    assert psi == 2
    points = [pow(psi, 2 * _brv(i, 2) + 1, q) for i in range(N)]
    assert sorted(points) == sorted({x for x in range(q) if pow(x, N, q) == q - 1})
    allin = np.array(list(itertools.product(range(q), repeat=N)), dtype=np.uint64)
    for a in allin:
        out = oracle.ntt_forward(a, q, psi, threads=1)
        assert [int(v) for v in out] == [_horner(a, x, q) for x in points]
        assert np.array_equal(oracle.ntt_inverse(out, q, psi, threads=1), a)


def test_forward_is_evaluation_at_roots_in_figure1_order(golden_primes):
    with open(os.path.join(HERE, "golden", "fig1_output_order_n16.json")) as f:
        fig = {int(k): v for k, v in json.load(f)["row_to_output_index"].items()}
    for q in [97, 12289, 1125899906826241, golden_primes["large_65536"]["moduli"][0]]:
        N = 16
        psi = oracle.min_root(N, q)
        a = uniform_mod(unit_seed(7, q), N, q)
        out = oracle.ntt_forward(a, q, psi, threads=1)
        # cyclic NTT of the psi-weighted input, omega = psi^2, natural order
        omega = psi * psi % q
        ahat = [int(a[j]) * pow(psi, j, q) % q for j in range(N)]
        X = [sum(ahat[j] * pow(omega, k * j, q) for j in range(N)) % q for k in range(N)]
        for row, idx in fig.items():
            assert int(out[row]) == X[idx]


@pytest.mark.parametrize("logn", [1, 2, 3, 5, 8, 10])
def test_forward_evaluates_at_distinct_roots_of_xn_plus_1(logn, golden_primes):
    N = 1 << logn
    for q in [golden_primes["single_1024"]["moduli"][0], golden_primes["large_65536"]["moduli"][3],
              golden_primes["edge"]["by_bits"]["62"][0]]:
        psi = oracle.min_root(N, q)
        a = uniform_mod(unit_seed(11, logn, q), N, q)
        out = oracle.ntt_forward(a, q, psi)
        pts = [pow(psi, 2 * _brv(i, logn) + 1, q) for i in range(N)]
        assert len(set(pts)) == N and all(pow(x, N, q) == q - 1 for x in pts)
        idx = list(range(N)) if N <= 64 else random.Random(logn).sample(range(N), 64)
        for i in idx:
            assert int(out[i]) == _horner(a, pts[i], q)


def test_round_trip_and_convolution_theorem(golden_primes):
    rng = random.Random(3)
    primes = [golden_primes["single_1024"]["moduli"][0], golden_primes["large_65536"]["moduli"][1],
              golden_primes["edge"]["by_bits"]["50"][0], golden_primes["edge"]["by_bits"]["62"][1]]
    for logn in [1, 2, 4, 7, 9]:
        N = 1 << logn
        for q in primes:
            psi = oracle.min_root(N, q)
            a = uniform_mod(unit_seed(1, logn, q), N, q)
            b = uniform_mod(unit_seed(2, logn, q), N, q)
            assert np.array_equal(oracle.ntt_inverse(oracle.ntt_forward(a, q, psi), q, psi), a)
            A, B = oracle.ntt_forward(a, q, psi), oracle.ntt_forward(b, q, psi)
            c = oracle.ntt_inverse(oracle.eltwise_mult(A, B, q), q, psi)
            assert np.array_equal(c, oracle.negacyclic_mul(a, b, q))
            # any other primitive root gives another transform but the same product
            psi2 = pow(psi, 2 * rng.randrange(N) + 1, q)
            A2, B2 = oracle.ntt_forward(a, q, psi2), oracle.ntt_forward(b, q, psi2)
            assert np.array_equal(oracle.ntt_inverse(oracle.eltwise_mult(A2, B2, q), q, psi2), c)


def test_delta_inputs():
    q, N = 12289, 64
    psi = oracle.min_root(N, q)
    one = np.zeros(N, dtype=np.uint64); one[0] = 1
    assert np.all(oracle.ntt_forward(one, q, psi) == 1)
    x = np.zeros(N, dtype=np.uint64); x[1] = 1
    out = oracle.ntt_forward(x, q, psi)
    assert [int(v) for v in out] == [pow(psi, 2 * _brv(i, 6) + 1, q) for i in range(N)]


def test_schoolbook_against_polynomial_division_and_special_products(golden_primes):
    for N in [1, 2, 3, 8, 33, 64]:
        for q in [17, 12289, golden_primes["large_65536"]["moduli"][0]]:
            a = uniform_mod(unit_seed(5, N, q), N, q)
            b = uniform_mod(unit_seed(6, N, q), N, q)
            assert [int(v) for v in oracle.negacyclic_mul(a, b, q)] == _poly_mul_mod_xn1(a, b, q)
            one = np.zeros(N, dtype=np.uint64); one[0] = 1
            assert np.array_equal(oracle.negacyclic_mul(a, one, q), a)
            if N >= 2:
                x = np.zeros(N, dtype=np.uint64); x[1] = 1
                shifted = np.array([(q - int(a[-1])) % q] + [int(v) for v in a[:-1]], dtype=np.uint64)
                assert np.array_equal(oracle.negacyclic_mul(x, a, q), shifted)
            if N % 2 == 0:
                h = np.zeros(N, dtype=np.uint64); h[N // 2] = 1
                minus_one = np.zeros(N, dtype=np.uint64); minus_one[0] = q - 1
                assert np.array_equal(oracle.negacyclic_mul(h, h, q), minus_one)


def test_eltwise_against_big_integers():
    rng = random.Random(4)
    for q in [2, 17, 1125899906826241, (1 << 62) - 57, (1 << 63) - 25]:
        n = 257
        a = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
        b = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
        assert [int(v) for v in oracle.eltwise_add(a, b, q)] == [(int(x) + int(y)) % q for x, y in zip(a, b)]
        assert [int(v) for v in oracle.eltwise_mult(a, b, q)] == [int(x) * int(y) % q for x, y in zip(a, b)]
        if 4 * q < (1 << 64):
            la = np.array([rng.randrange(4 * q) for _ in range(n)], dtype=np.uint64)
            assert [int(v) for v in oracle.eltwise_mult(la, b, q)] == [int(x) * int(y) % q for x, y in zip(la, b)]


def test_spot_checks_equal_full_transforms(golden_primes):
    N = 512
    q = golden_primes["large_65536"]["moduli"][5]
    psi = oracle.min_root(N, q)
    a = uniform_mod(unit_seed(8), N, q)
    b = uniform_mod(unit_seed(9), N, q)
    idx = np.array([0, 1, 7, 255, 256, 511], dtype=np.uint64)
    assert np.array_equal(oracle.ntt_forward_at(a, idx, q, psi), oracle.ntt_forward(a, q, psi)[idx])
    assert np.array_equal(oracle.ntt_inverse_at(a, idx, q, psi), oracle.ntt_inverse(a, q, psi)[idx])
    assert np.array_equal(oracle.negacyclic_mul_at(a, b, idx, q), oracle.negacyclic_mul(a, b, q)[idx])


@pytest.mark.parametrize("logn", [1, 2, 3, 6, 10, 12])
def test_harvey_model_agrees_with_direct_and_keeps_lazy_ranges(logn, golden_primes):
    N = 1 << logn
    primes = [golden_primes["single_1024"]["moduli"][0], golden_primes["large_65536"]["moduli"][0],
              golden_primes["edge"]["by_bits"]["62"][0], golden_primes["edge"]["by_bits"]["50"][0],
              golden_primes["edge"]["by_bits"]["61"][1]]
    for q in primes:
        psi = oracle.min_root(N, q)
        for in_f in (1, 2, 4):
            a = lazy_mod(unit_seed(20, logn, q, in_f), N, q, in_f)
            ref = oracle.ntt_forward(a, q, psi)
            lazy = oracle.harvey_forward(a, q, psi, out_f=4)
            assert np.all(lazy < np.uint64(4 * q))
            assert np.array_equal(lazy % np.uint64(q), ref)
            assert np.array_equal(oracle.harvey_forward(a, q, psi, out_f=1), ref)
        for in_f in (1, 2):
            A = lazy_mod(unit_seed(21, logn, q, in_f), N, q, in_f)
            ref = oracle.ntt_inverse(A, q, psi)
            lazy = oracle.harvey_inverse(A, q, psi, out_f=2)
            assert np.all(lazy < np.uint64(2 * q))
            assert np.array_equal(lazy % np.uint64(q), ref)
            assert np.array_equal(oracle.harvey_inverse(A, q, psi, out_f=1), ref)


def test_listing_product_pipeline_matches_schoolbook(golden_primes):
    """The lazy product of the input_mod_factor listing (Section 4): forward
    (1 -> 4), forward (1 -> 4), multiply with input factor 4, inverse (1 -> 1)."""
    N = 256
    for q in golden_primes["rns_16384"]["moduli"][:3] + golden_primes["large_65536"]["moduli"][:2]:
        psi = oracle.min_root(N, q)
        a = uniform_mod(unit_seed(30, q), N, q)
        b = uniform_mod(unit_seed(31, q), N, q)
        fa = oracle.harvey_forward(a, q, psi, 4)
        fb = oracle.harvey_forward(b, q, psi, 4)
        c = oracle.harvey_inverse(oracle.eltwise_mult(fa, fb, q), q, psi, 1)
        assert np.array_equal(c, oracle.negacyclic_mul(a, b, q))


# ---- word size beta = 2^32 (moduli below 2^30) --------------------------------

def _small_moduli(golden_primes, N):
    """Moduli below 2^30 with q = 1 mod 2N: the two smallest 30-bit primes = 1 mod 2^18,
    and 12289 = 3 * 2^12 + 1 or 17 where N allows."""
    qs = list(golden_primes["edge"]["by_bits"]["30"])
    if (12289 - 1) % (2 * N) == 0:
        qs.append(12289)
    if (17 - 1) % (2 * N) == 0:
        qs.append(17)
    return qs


@pytest.mark.parametrize("logn", [1, 2, 3, 6, 10, 12])
def test_harvey_word32_model_agrees_with_direct_and_keeps_lazy_ranges(logn, golden_primes):
    """Algorithms 2-5 at beta = 2^32 give the direct definition mod q, within the
    lazy ranges of Algorithms 4 and 5, for inputs up to the largest input factor."""
    N = 1 << logn
    for q in _small_moduli(golden_primes, N):
        psi = oracle.min_root(N, q)
        for in_f in (1, 2, 4):
            a = lazy_mod(unit_seed(40, logn, q, in_f), N, q, in_f)
            if in_f == 4:
                a[-1] = np.uint64(4 * q - 1)
            ref = oracle.ntt_forward(a, q, psi)
            lazy = oracle.harvey_forward_w(a, q, psi, out_f=4, bits=32)
            assert np.all(lazy < np.uint64(4 * q))
            assert np.array_equal(lazy % np.uint64(q), ref)
            assert np.array_equal(oracle.harvey_forward_w(a, q, psi, out_f=1, bits=32), ref)
        for in_f in (1, 2):
            A = lazy_mod(unit_seed(41, logn, q, in_f), N, q, in_f)
            ref = oracle.ntt_inverse(A, q, psi)
            lazy = oracle.harvey_inverse_w(A, q, psi, out_f=2, bits=32)
            assert np.all(lazy < np.uint64(2 * q))
            assert np.array_equal(lazy % np.uint64(q), ref)
            assert np.array_equal(oracle.harvey_inverse_w(A, q, psi, out_f=1, bits=32), ref)


def test_harvey_word_size_parameter(golden_primes):
    """At beta = 2^64 the parameterised model is the scalar model; at beta = 2^32
    the representatives are the ones a 32-bit word produces, not the 64-bit ones."""
    N = 1024
    q = golden_primes["edge"]["by_bits"]["30"][0]
    psi = oracle.min_root(N, q)
    a = lazy_mod(unit_seed(42), N, q, 4)
    f64 = oracle.harvey_forward(a, q, psi, 4)
    assert np.array_equal(oracle.harvey_forward_w(a, q, psi, 4, bits=64), f64)
    f32 = oracle.harvey_forward_w(a, q, psi, 4, bits=32)
    assert np.array_equal(f32 % np.uint64(q), f64 % np.uint64(q))
    assert not np.array_equal(f32, f64)
    with pytest.raises(ValueError):
        oracle.harvey_forward_w(a, golden_primes["edge"]["by_bits"]["31"][0], psi, 4, bits=32)


@pytest.mark.parametrize("bits", [32, 64])
def test_harvey_butterfly_brute_force(bits, golden_primes):
    """One Algorithm 4 butterfly on many (X0, X1) pairs, against exact integer
    arithmetic: X0' = A + T and X1' = A + 2q - T with A = X0 mod 2q (X0 < 4q),
    T = W X1 mod q taken in [0, 2q); both outputs below 4q."""
    for q in list(golden_primes["edge"]["by_bits"]["30"]) + [12289, 17]:
        n = 4000
        x0 = lazy_mod(unit_seed(43, q, bits), n, q, 4)
        x1 = lazy_mod(unit_seed(44, q, bits), n, q, 4)
        x0[:3] = np.array([0, 2 * q, 4 * q - 1], dtype=np.uint64)
        x1[:3] = np.array([4 * q - 1, 0, 4 * q - 1], dtype=np.uint64)
        for w in [1, q - 1, int(uniform_mod(unit_seed(45, q), 1, q)[0])]:
            y0, y1 = oracle.harvey_fwd_bfly_w(x0, x1, w, q, bits)
            for i in range(0, n, 7):
                X0, X1 = int(x0[i]), int(x1[i])
                A = X0 - 2 * q if X0 >= 2 * q else X0
                T = int(y0[i]) - A
                assert 0 <= T < 2 * q and T % q == (w * X1) % q, (q, w, X0, X1)
                assert int(y1[i]) == A + 2 * q - T and int(y0[i]) < 4 * q and int(y1[i]) < 4 * q


# ---- batched forms (many limbs of one modulus, threads) ------------------------

@pytest.mark.parametrize("logn", [1, 3, 7, 9])
def test_product_batch_matches_schoolbook(logn, golden_primes):
    """The O(N log N) product through the transforms (Section 4 product listing) equals the
    schoolbook negacyclic product of Section 2 on every limb, for lazy inputs up to 4q and for
    edge moduli (the smallest 50- and 62-bit NTT primes, a 30-bit one)."""
    N = 1 << logn
    primes = [golden_primes["rns_16384"]["moduli"][0], golden_primes["large_65536"]["moduli"][3],
              golden_primes["edge"]["by_bits"]["62"][0], golden_primes["edge"]["by_bits"]["50"][1],
              golden_primes["edge"]["by_bits"]["30"][0]]
    for q in primes:
        count = 5
        a = np.concatenate([lazy_mod(unit_seed(50, logn, q, k), N, q, 4) for k in range(count)])
        b = np.concatenate([uniform_mod(unit_seed(51, logn, q, k), N, q) for k in range(count)])
        c = oracle.product_batch(a, b, N, q, threads=3)
        for k in range(count):
            s = slice(k * N, (k + 1) * N)
            assert np.array_equal(c[s], oracle.negacyclic_mul(a[s], b[s], q)), (q, k)


def test_product_batch_special_products(golden_primes):
    """X^(N/2) * X^(N/2) = -1 and a * X = the negacyclic shift of a, limb by limb."""
    N, q = 1024, golden_primes["single_1024"]["moduli"][0]
    half = np.zeros(N, dtype=np.uint64)
    half[N // 2] = 1
    x = np.zeros(N, dtype=np.uint64)
    x[1] = 1
    a = uniform_mod(unit_seed(52), N, q)
    c = oracle.product_batch(np.concatenate([half, a]), np.concatenate([half, x]), N, q)
    minus_one = np.zeros(N, dtype=np.uint64)
    minus_one[0] = q - 1
    assert np.array_equal(c[:N], minus_one)
    shifted = np.concatenate([[(q - int(a[-1])) % q], a[:-1]]).astype(np.uint64)
    assert np.array_equal(c[N:], shifted)


@pytest.mark.parametrize("logn", [2, 5, 10])
def test_harvey_batch_matches_direct(logn, golden_primes):
    """Every limb of the batched Harvey forward/inverse reduces to the direct O(N^2) sums, and
    the lazy words stay in [0, 4q) / [0, 2q); the canonical form equals the sums exactly."""
    N = 1 << logn
    for q in [golden_primes["single_1024"]["moduli"][0], golden_primes["edge"]["by_bits"]["61"][0]]:
        psi = oracle.min_root(N, q)
        count = 4
        a = np.concatenate([lazy_mod(unit_seed(53, logn, q, k), N, q, 4) for k in range(count)])
        A = np.concatenate([lazy_mod(unit_seed(54, logn, q, k), N, q, 2) for k in range(count)])
        lazy = oracle.harvey_forward_batch(a, N, q, psi, 4, threads=2)
        canon = oracle.harvey_forward_batch(a, N, q, psi, 1, threads=2)
        ilazy = oracle.harvey_inverse_batch(A, N, q, psi, 2, threads=2)
        icanon = oracle.harvey_inverse_batch(A, N, q, psi, 1, threads=2)
        assert np.all(lazy < np.uint64(4 * q)) and np.all(ilazy < np.uint64(2 * q))
        for k in range(count):
            s = slice(k * N, (k + 1) * N)
            ref = oracle.ntt_forward(a[s], q, psi)
            iref = oracle.ntt_inverse(A[s], q, psi)
            assert np.array_equal(canon[s], ref) and np.array_equal(lazy[s] % np.uint64(q), ref)
            assert np.array_equal(icanon[s], iref) and np.array_equal(ilazy[s] % np.uint64(q), iref)


def test_rns_helpers_use_each_limbs_modulus(golden_primes):
    """product_rns / forward_rns / inverse_rns / add_rns on a [B][L][N] array treat limb l of
    every polynomial modulo moduli[l] (checked limb by limb against the schoolbook product and
    the direct sums)."""
    N = 64
    moduli = golden_primes["rns_16384"]["moduli"][:3]
    B, L = 2, len(moduli)
    a = np.concatenate([uniform_mod(unit_seed(55, p, l), N, q) for p in range(B) for l, q in enumerate(moduli)])
    b = np.concatenate([uniform_mod(unit_seed(56, p, l), N, q) for p in range(B) for l, q in enumerate(moduli)])
    c = oracle.product_rns(a, b, N, moduli)
    f = oracle.forward_rns(a, N, moduli)
    i = oracle.inverse_rns(a, N, moduli)
    s_ = oracle.add_rns(a, b, N, moduli)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            psi = oracle.min_root(N, q)
            assert np.array_equal(c[s], oracle.negacyclic_mul(a[s], b[s], q))
            assert np.array_equal(f[s], oracle.ntt_forward(a[s], q, psi))
            assert np.array_equal(i[s], oracle.ntt_inverse(a[s], q, psi))
            assert np.array_equal(s_[s], oracle.eltwise_add(a[s], b[s], q))
