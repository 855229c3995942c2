"""Pins the oracle's element-wise ring operations (Section 2 list of ring
operations; Section 4 free-function listing) to relations they must satisfy,
so that a dropped term, a sign or an operand mix-up in any one of them fails:

* negation is an additive inverse (a + (-a) = 0), an involution, and fixes 0;
* subtraction equals adding the negation, and (a - b) + b = a;
* the fused multiply-add reduces to the element-wise product when the addend
  is absent or zero, to the element-wise sum when the scalar is 1, and is
  linear in the scalar: fma(a, y1 + y2, 0) = fma(a, y1, 0) + fma(a, y2, 0);
* every output is canonical, for inputs up to the largest input factor (8q)
  and moduli from 2 up to 2^61 - 1;
* and, for a handful of values, the plain big-integer definition.
"""
import numpy as np
import pytest

import oracle
from synthetic import uniform_int, uniform_mod, unit_seed

MODULI = [2, 3, 17, 12289, (1 << 50) - 27, (1 << 60) - 93, (1 << 61) - 1]


def _vec(seed, n, bound):
    return uniform_mod(seed, n, bound).astype(np.uint64)


@pytest.mark.parametrize("q", MODULI)
def test_negate_and_sub(q):
    n = 257
    a = _vec(unit_seed(500, q), n, q)
    b = _vec(unit_seed(501, q), n, q)
    a[0] = 0
    neg = oracle.eltwise_negate(a, q)
    assert np.all(neg < np.uint64(q)) and neg[0] == 0
    assert np.all(oracle.eltwise_add(a, neg, q) == 0)
    assert np.array_equal(oracle.eltwise_negate(neg, q), a)
    d = oracle.eltwise_sub(a, b, q)
    assert np.all(d < np.uint64(q))
    assert np.array_equal(d, oracle.eltwise_add(a, oracle.eltwise_negate(b, q), q))
    assert np.array_equal(oracle.eltwise_add(d, b, q), a)
    # inputs are taken modulo q: lazy representatives give the same result
    lazy = a + np.uint64(q) * (np.arange(n, dtype=np.uint64) % np.uint64(4)) if q < (1 << 61) else a
    assert np.array_equal(oracle.eltwise_sub(lazy, b, q), d)


@pytest.mark.parametrize("q", MODULI)
def test_fma_relations(q):
    n = 300
    f = 8 if q < (1 << 61) else 1
    a = _vec(unit_seed(510, q), n, f * q if f * q < (1 << 64) else q)
    z = _vec(unit_seed(511, q), n, f * q if f * q < (1 << 64) else q)
    ys = [0, 1, q - 1] + [int(v) for v in uniform_mod(unit_seed(512, q), 3, q)]
    am = a % np.uint64(q)
    for y in ys:
        r = oracle.eltwise_fma(a, y, z, q)
        assert np.all(r < np.uint64(q))
        r0 = oracle.eltwise_fma(a, y, None, q)
        assert np.array_equal(r0, oracle.eltwise_mult(am, np.full(n, y % q, dtype=np.uint64), q))
        assert np.array_equal(oracle.eltwise_fma(a, y, np.zeros(n, dtype=np.uint64), q), r0)
        assert np.array_equal(r, oracle.eltwise_add(r0, z, q))
    assert np.array_equal(oracle.eltwise_fma(a, 1, z, q), oracle.eltwise_add(am, z, q))
    y1, y2 = ys[-2], ys[-1]
    lhs = oracle.eltwise_fma(a, (y1 + y2) % q, None, q)
    rhs = oracle.eltwise_add(oracle.eltwise_fma(a, y1, None, q), oracle.eltwise_fma(a, y2, None, q), q)
    assert np.array_equal(lhs, rhs)


def test_fma_big_integer_spot_values():
    q = (1 << 61) - 1
    a = np.array([0, 1, q - 1, 8 * q - 1 - (1 << 63) * 0, 123456789], dtype=np.uint64)
    a[3] = np.uint64((8 * q - 1) % (1 << 64))
    z = np.array([q - 1, 0, q - 1, 5, 987654321], dtype=np.uint64)
    y = q - 2
    got = oracle.eltwise_fma(a, y, z, q)
    for i in range(a.size):
        assert int(got[i]) == (int(a[i]) * y + int(z[i])) % q
    # small modulus, exhaustive over all residues
    q = 17
    a = np.arange(17 * 8, dtype=np.uint64)
    for y in range(17):
        got = oracle.eltwise_fma(a, y, a[::-1].copy(), q)
        want = [(int(a[i]) * y + int(a[::-1][i])) % q for i in range(a.size)]
        assert [int(v) for v in got] == want
