"""Pins the oracle's scalar number theory to independent references.

* modular products / powers / inverses: Python's arbitrary-precision integers
  (the textbook definition (a * b) mod q of the native listing in Section 2.1);
* primality: sympy.isprime, plus composites that fool weaker Miller-Rabin sets;
* minimal primitive 2N-th root: brute force over every residue for small q;
* bit reversal: the output labels of the paper's Figure 1 (N = 16);
* prime search: sympy, plus the congruence and bit-length conditions.
"""
import json
import os
import random

import pytest
import sympy

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_mulmod_powmod_invmod_match_big_integers():
    rng = random.Random(1)
    moduli = [2, 3, 17, 12289, (1 << 31) - 1, 1125899906826241, (1 << 61) - 1, (1 << 62) - 57,
              (1 << 63) - 25, (1 << 64) - 59]
    for q in moduli:
        for _ in range(300):
            a, b = rng.randrange(1 << 64), rng.randrange(1 << 64)
            assert oracle.mulmod(a % q, b % q, q) == (a % q) * (b % q) % q
            assert oracle.addmod(a, b, q) == (a + b) % q
            e = rng.randrange(1 << 64)
            assert oracle.powmod(a, e, q) == pow(a, e, q)
        if sympy.isprime(q) and q > 2:
            for _ in range(50):
                a = rng.randrange(1, q)
                assert oracle.mulmod(oracle.invmod(a, q), a, q) == 1


def test_is_prime_matches_sympy():
    rng = random.Random(2)
    cases = [0, 1, 2, 3, 4, 5, 561, 1105, 1729, 2047, 3215031751, 2152302898747, 3474749660383,
             341550071728321, 3825123056546413051, 318665857834031151167461 % (1 << 64),
             (1 << 61) - 1, (1 << 64) - 59, (1 << 64) - 1, 1000000007 ** 2, 4294967291 * 4294967279]
    cases += [rng.randrange(1 << 64) | 1 for _ in range(3000)]
    cases += [int(sympy.nextprime(rng.randrange(1 << 62))) for _ in range(200)]
    for n in cases:
        assert oracle.is_prime(n) == bool(sympy.isprime(n)), n


def test_brv_matches_figure1_labels():
    with open(os.path.join(HERE, "golden", "fig1_output_order_n16.json")) as f:
        fig = json.load(f)
    for row, idx in fig["row_to_output_index"].items():
        assert oracle.brv(int(row), 4) == idx
    for logn in range(0, 12):
        for i in range(1 << logn):
            assert oracle.brv(oracle.brv(i, logn), logn) == i


def _small_ntt_primes(limit):
    return [q for q in sympy.primerange(3, limit)]


def test_min_root_brute_force_small_primes():
    for q in _small_ntt_primes(1200):
        for logn in range(0, 9):
            N = 1 << logn
            if (q - 1) % (2 * N):
                assert oracle.min_root(N, q) == 0
                continue
            brute = next(r for r in range(2, q) if pow(r, N, q) == q - 1)
            assert oracle.min_root(N, q) == brute, (N, q)


def test_min_root_large_primes_is_primitive_and_smallest_of_the_orbit(golden_primes):
    for key in ("single_1024", "rns_16384", "large_65536"):
        N = golden_primes[key]["N"]
        for q, psi in zip(golden_primes[key]["moduli"], golden_primes[key]["psi"]):
            assert oracle.min_root(N, q) == psi
            assert pow(psi, N, q) == q - 1                    # psi^N = -1: order exactly 2N
            # every primitive 2N-th root is psi^k for odd k; none is smaller than psi
            g2, cur = psi * psi % q, psi
            for _ in range(N - 1):
                cur = cur * g2 % q
                assert cur > psi or cur == psi


def test_find_primes_against_sympy(golden_primes):
    for bits, m, count in [(50, 2048, 3), (50, 1 << 15, 8), (60, 1 << 17, 5), (40, 1 << 18, 4)]:
        got = oracle.find_primes(bits, m, count)
        ref, p = [], (1 << bits) - 1
        p -= (p - 1) % m
        while len(ref) < count:
            if sympy.isprime(p):
                ref.append(p)
            p -= m
        assert got == ref
    for key in ("single_1024", "rns_16384", "large_65536"):
        N = golden_primes[key]["N"]
        for q in golden_primes[key]["moduli"]:
            assert sympy.isprime(q) and q % (2 * N) == 1 and q < (1 << 62)
    for Q, ps in golden_primes["edge"]["by_bits"].items():
        for q in ps:
            assert sympy.isprime(q) and q.bit_length() == int(Q) and q % (1 << 18) == 1
        assert ps[0] == next(p for p in range((1 << (int(Q) - 1)) + 1, 1 << int(Q), 1 << 18) if sympy.isprime(p))
    for q in golden_primes["serving"]["moduli"]:
        assert sympy.isprime(q) and q % (1 << 18) == 1 and 50 <= q.bit_length() <= 60
