"""GPU parity of the wide-range butterflies (single-pass kernels, N <= 2^14, every modulus
below 2^58).

They compute the same transforms as Algorithms 4 and 5 with a quotient estimate that may
be one short and without the forward's per-stage reduction, so their lazy outputs are
other representatives of the same residues.  What is unique is checked bit-exactly:
canonical outputs, fused products and accumulations equal the oracle's definitions
(Section 2.2 transforms, Section 2 negacyclic product) and the paper-butterfly path
(switched on with ntt_set_wide_range(0)), whose lazy words equal the oracle's Harvey
model.  Lazy outputs are checked for range and residue.  The worst case for the growth
bound is driven explicitly: the largest admissible modulus below 2^58 with every input at
the top of its range.
"""
import numpy as np
import pytest

import oracle
from synthetic import lazy_mod, uniform_mod, unit_seed
from gpu_util import WIDE_BOUND, empty_dev, from_dev, have_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]


@pytest.fixture(scope="module")
def nt():
    import paper_2103_16400_amd as nt
    yield nt
    nt.set_wide_range(True)


def _moduli(logN):
    """Moduli below 2^58 valid for 2^logN: 17 and 12289 where allowed, the smallest 30-
    and 50-bit primes = 1 mod 2^18 and the largest prime below 2^58 = 1 mod 2^(logN+1)."""
    m = 2 << logN
    out = [q for q in (17, 12289) if (q - 1) % m == 0]
    out += oracle.find_primes_up(30, 1 << 18, 1) + oracle.find_primes_up(50, 1 << 18, 1)
    out += oracle.find_primes(58, m, 1)
    assert all(q < WIDE_BOUND for q in out)
    return out


def _rns(tag, N, moduli, B, f, top=True):
    L = len(moduli)
    out = np.empty(B * L * N, dtype=np.uint64)
    for p in range(B):
        for l, q in enumerate(moduli):
            x = lazy_mod(unit_seed(tag, p, l, q, f), N, q, f)
            if top:
                x[-1] = np.uint64(f * q - 1)
            out[(p * L + l) * N:(p * L + l + 1) * N] = x
    return out


def _segs(N, moduli, B):
    L = len(moduli)
    for p in range(B):
        for l, q in enumerate(moduli):
            yield slice((p * L + l) * N, (p * L + l + 1) * N), q


def _idx(N, seed, k=20):
    """Every output is compared: None selects the whole array."""
    return None


def _fwd_ref(a, q, idx=None):
    """Canonical forward transform: the O(N^2) direct sums up to N = 1024, above that the
    O(N log N) Harvey model with a final correction, which CPU tests pin to the direct sums."""
    psi = oracle.min_root(a.size, q)
    if a.size <= 1024:
        return oracle.ntt_forward(a, q, psi)
    return oracle.harvey_forward(a, q, psi, 1)


def _inv_ref(A, q, idx=None):
    """Canonical inverse transform (inputs below 2q), as _fwd_ref."""
    psi = oracle.min_root(A.size, q)
    if A.size <= 1024:
        return oracle.ntt_inverse(A, q, psi)
    return oracle.harvey_inverse(A, q, psi, 1)


def _prod_ref(a, b, q):
    """Canonical negacyclic product: schoolbook up to N = 1024, above that through the
    oracle's transforms (pinned to the schoolbook product on the CPU)."""
    if a.size <= 1024:
        return oracle.negacyclic_mul(a, b, q)
    return oracle.product_batch(a, b, a.size, q)


def _at(x, idx):
    return x if idx is None else x[idx]


def _run(nt, wide, fn):
    nt.set_wide_range(wide)
    try:
        return fn()
    finally:
        nt.set_wide_range(True)


LOGNS = [1, 2, 3, 4, 5, 8, 10, 12, 13, 14]


@pytest.mark.parametrize("logN", LOGNS)
def test_wide_forward_against_exact_and_definition(nt, logN):
    N = 1 << logN
    moduli = _moduli(logN)
    B = 2
    idx = _idx(N, 300 + logN)
    for in_f in (1, 2, 4):
        a = _rns(301 + in_f, N, moduli, B, in_f)
        da = to_dev(a)

        def fwd(out_f):
            d = empty_dev(a.size)
            nt.ntt_forward_rns(d, da, N, moduli, B, in_f, out_f)
            return from_dev(d)
        lazy_w, canon_w = _run(nt, True, lambda: fwd(4)), _run(nt, True, lambda: fwd(1))
        lazy_x, canon_x = _run(nt, False, lambda: fwd(4)), _run(nt, False, lambda: fwd(1))
        assert np.array_equal(canon_w, canon_x), in_f
        for s, q in _segs(N, moduli, B):
            ref = _fwd_ref(a[s], q, idx)
            assert np.array_equal(_at(canon_w[s], idx), ref), (in_f, q)
            assert np.all(lazy_w[s] < np.uint64(4 * q)), (in_f, q)
            assert np.array_equal(lazy_w[s] % np.uint64(q), canon_w[s]), (in_f, q)
            assert np.array_equal(lazy_x[s], oracle.harvey_forward(a[s], q, oracle.min_root(N, q), 4)), (in_f, q)


@pytest.mark.parametrize("logN", LOGNS)
def test_wide_inverse_against_exact_and_definition(nt, logN):
    N = 1 << logN
    moduli = _moduli(logN)
    B = 2
    idx = _idx(N, 310 + logN)
    for in_f in (1, 2):
        A = _rns(311 + in_f, N, moduli, B, in_f)
        dA = to_dev(A)

        def inv(out_f):
            d = empty_dev(A.size)
            nt.ntt_inverse_rns(d, dA, N, moduli, B, in_f, out_f)
            return from_dev(d)
        lazy_w, canon_w = _run(nt, True, lambda: inv(2)), _run(nt, True, lambda: inv(1))
        canon_x = _run(nt, False, lambda: inv(1))
        assert np.array_equal(canon_w, canon_x), in_f
        for s, q in _segs(N, moduli, B):
            assert np.array_equal(_at(canon_w[s], idx), _inv_ref(A[s], q, idx)), (in_f, q)
            assert np.all(lazy_w[s] < np.uint64(2 * q)), (in_f, q)
            assert np.array_equal(lazy_w[s] % np.uint64(q), canon_w[s]), (in_f, q)


@pytest.mark.parametrize("logN", [1, 3, 5, 10, 13, 14])
def test_wide_fused_modes(nt, logN):
    """Forward fused with the multiply, inverse fused with the accumulate, and the three
    product calls: wide and paper paths give the same words, equal to the oracle's
    element-wise product / sum of its transforms."""
    N = 1 << logN
    moduli = _moduli(logN)
    L, B = len(moduli), 2
    idx = _idx(N, 320 + logN, 12)
    a = _rns(321, N, moduli, B, 4)
    m = _rns(322, N, moduli, B, 4)
    acc0 = _rns(323, N, moduli, B, 1)
    A = _rns(324, N, moduli, B, 2)
    b = _rns(325, N, moduli, B, 1)
    a1 = _rns(326, N, moduli, B, 1)
    ws = empty_dev(2 * a.size)

    def all_calls():
        r = {}
        d = empty_dev(a.size)
        nt.ntt_forward_mul_rns(d, to_dev(a), to_dev(m), N, moduli, B, 4, ws)
        r["fwd_mul"] = from_dev(d)
        d = to_dev(acc0)
        nt.ntt_inverse_acc_rns(d, to_dev(A), N, moduli, B, 2, ws)
        r["inv_acc"] = from_dev(d)
        d = empty_dev(a.size)
        nt.poly_mul_rns(d, to_dev(a1), to_dev(b), N, moduli, B, ws)
        r["mul"] = from_dev(d)
        d = to_dev(acc0)
        nt.poly_mul_acc_rns(d, to_dev(a1), to_dev(b), N, moduli, B, ws)
        r["mul_acc"] = from_dev(d)
        d = to_dev(acc0)
        nt.poly_mul_acc_ntt_rns(d, to_dev(m), to_dev(b), N, moduli, B, ws)
        r["mul_acc_ntt"] = from_dev(d)
        return r
    w = _run(nt, True, all_calls)
    x = _run(nt, False, all_calls)
    for k in w:
        assert np.array_equal(w[k], x[k]), k
    for s, q in _segs(N, moduli, B):
        qq = np.uint64(q)
        assert np.array_equal(_at(w["fwd_mul"][s], idx),
                              oracle.eltwise_mult(_fwd_ref(a[s], q, idx), _at(m[s], idx) % qq, q)), q
        assert np.array_equal(_at(w["inv_acc"][s], idx),
                              oracle.eltwise_add(_at(acc0[s], idx), _inv_ref(A[s], q, idx), q)), q
        prod = _prod_ref(a1[s], b[s], q)
        assert np.array_equal(_at(w["mul"][s], idx), prod), q
        assert np.array_equal(_at(w["mul_acc"][s], idx), oracle.eltwise_add(_at(acc0[s], idx), prod, q)), q
        pm = oracle.eltwise_mult(_fwd_ref(b[s], q), m[s] % qq, q)
        assert np.array_equal(_at(w["mul_acc_ntt"][s], idx),
                              oracle.eltwise_add(_at(acc0[s], idx), _inv_ref(pm, q, idx), q)), q


@pytest.mark.parametrize("logN", [12, 13, 14])
def test_wide_growth_bound_worst_case(nt, logN):
    """The largest prime below 2^58 that is 1 mod 2N, every input at the top of its range
    (4q - 1 for the forward, 2q - 1 for the inverse, q - 1 for the products, 4q - 1 for
    the transformed multiplier): the largest values the wide forward can reach.  Canonical
    results equal the paper path's and the definitions; lazy results stay in range."""
    N = 1 << logN
    q = oracle.find_primes(58, 2 << logN, 1)[0]
    idx = _idx(N, 330 + logN, 12)
    top4 = np.full(N, 4 * q - 1, dtype=np.uint64)
    alt4 = np.where(np.arange(N) % 2 == 0, np.uint64(4 * q - 1), np.uint64(0)).astype(np.uint64)
    for a in (top4, alt4):
        def fwd(out_f):
            d = empty_dev(N)
            nt.ntt_forward(d, to_dev(a), N, q, 4, out_f)
            return from_dev(d)
        lazy_w, canon_w = _run(nt, True, lambda: fwd(4)), _run(nt, True, lambda: fwd(1))
        assert np.array_equal(canon_w, _run(nt, False, lambda: fwd(1)))
        assert np.array_equal(_at(canon_w, idx), _fwd_ref(a, q, idx))
        assert np.all(lazy_w < np.uint64(4 * q))
        assert np.array_equal(lazy_w % np.uint64(q), canon_w)
    A = np.full(N, 2 * q - 1, dtype=np.uint64)

    def inv():
        d = empty_dev(N)
        nt.ntt_inverse(d, to_dev(A), N, q, 2, 1)
        return from_dev(d)
    got = _run(nt, True, inv)
    assert np.array_equal(got, _run(nt, False, inv))
    assert np.array_equal(_at(got, idx), _inv_ref(A, q, idx))
    b = np.full(N, q - 1, dtype=np.uint64)
    m = np.full(N, 4 * q - 1, dtype=np.uint64)
    acc0 = np.full(N, q - 1, dtype=np.uint64)

    def prods():
        d1 = empty_dev(N)
        nt.poly_mul_rns(d1, to_dev(b), to_dev(b), N, [q], 1)
        d2 = to_dev(acc0)
        nt.poly_mul_acc_ntt_rns(d2, to_dev(m), to_dev(b), N, [q], 1)
        return from_dev(d1), from_dev(d2)
    (p_w, acc_w), (p_x, acc_x) = _run(nt, True, prods), _run(nt, False, prods)
    assert np.array_equal(p_w, p_x) and np.array_equal(acc_w, acc_x)
    assert np.array_equal(p_w, _prod_ref(b, b, q))
    assert np.array_equal(acc_w, oracle.eltwise_add(acc0, _inv_ref(oracle.eltwise_mult(_fwd_ref(b, q), m % np.uint64(q), q), q), q))


def test_wide_selection_per_launch(nt):
    """A launch takes the wide butterflies only when every modulus is below 2^58: with a
    60-bit limb in the launch, all limbs' lazy words equal the Harvey model; with only
    small moduli they are other representatives (checked on these seeded inputs); with the
    switch off, the model's words again."""
    logN = 12
    N = 1 << logN
    small = _moduli(logN)[-2:]
    big = oracle.find_primes(60, 2 << logN, 1)
    a_mixed = _rns(340, N, small + big, 1, 1)
    d = empty_dev(a_mixed.size)
    nt.ntt_forward_rns(d, to_dev(a_mixed), N, small + big, 1, 1, 4)
    got = from_dev(d)
    for s, q in _segs(N, small + big, 1):
        assert np.array_equal(got[s], oracle.harvey_forward(a_mixed[s], q, oracle.min_root(N, q), 4)), q
    a = _rns(341, N, small, 1, 1)

    def fwd():
        d = empty_dev(a.size)
        nt.ntt_forward_rns(d, to_dev(a), N, small, 1, 1, 4)
        return from_dev(d)
    w, x = _run(nt, True, fwd), _run(nt, False, fwd)
    for s, q in _segs(N, small, 1):
        model = oracle.harvey_forward(a[s], q, oracle.min_root(N, q), 4)
        assert np.array_equal(x[s], model), q
        assert not np.array_equal(w[s], model), q
        assert np.array_equal(w[s] % np.uint64(q), model % np.uint64(q)), q
    assert nt.get_wide_range()
