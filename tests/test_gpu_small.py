"""GPU parity of the word-size-2^32 path (moduli below 2^30, N <= 2^17; two passes at 2^16
and 2^17) through the C ABI.

Forward lazy outputs must be the exact words of Algorithms 2 + 4 at beta = 2^32
(the oracle's word-size model, itself pinned to the direct definition);
canonical outputs must equal the direct definitions of Section 2.2; the inverse
(N^{-1} fused into its last stage) must give the definition mod q within
[0, 2q); products must equal the schoolbook negacyclic product of Section 2.
"""
import json
import os

import numpy as np
import pytest

import oracle
from synthetic import lazy_mod, uniform_mod, unit_seed
from gpu_util import have_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRIMES = json.load(open(os.path.join(ROOT, "tests", "golden", "primes.json")))
EDGE30 = PRIMES["edge"]["by_bits"]["30"]          # smallest 30-bit primes = 1 mod 2^18
SMALL = PRIMES["small_16384"]["moduli"]           # largest primes < 2^30 = 1 mod 2^15


@pytest.fixture(scope="module")
def nt():
    import paper_2103_16400_amd as nt
    return nt


def dev32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to("cuda:0")


def host32(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32).astype(np.uint64)


def empty32(n):
    import torch
    return torch.empty(n, dtype=torch.int32, device="cuda:0")


def _moduli(N, L):
    """L moduli below 2^30 valid for N: the 30-bit edge primes and the small set, then
    12289 and 17 where N allows them."""
    pool = list(EDGE30) + list(SMALL)
    pool = [q for q in pool if (q - 1) % (2 * N) == 0]
    if (12289 - 1) % (2 * N) == 0:
        pool = [12289] + pool
    if (17 - 1) % (2 * N) == 0:
        pool = [17] + pool
    return pool[:L]


def _inputs(tag, N, moduli, B, f):
    L = len(moduli)
    out = np.empty(B * L * N, dtype=np.uint64)
    for p in range(B):
        for l, q in enumerate(moduli):
            x = lazy_mod(unit_seed(tag, p, l, q, f), N, q, f)
            x[-1] = np.uint64(f * q - 1)
            out[(p * L + l) * N:(p * L + l + 1) * N] = x
    return out


def _idx(N, seed, k=24):
    r = uniform_mod(unit_seed(seed, N), k, N).astype(np.uint64)
    return np.unique(np.concatenate([r, np.array([0, 1, N // 2, N - 1], dtype=np.uint64)]))


LOGNS = [1, 2, 3, 4, 5, 8, 10, 11, 12, 13, 14, 15, 16, 17]


def _ws(N, size):
    """The products' workspace: needed from N = 2^16 (two passes)."""
    return empty32(size) if N > (1 << 15) else None


@pytest.mark.parametrize("logN", LOGNS)
def test_forward32_words_and_definition(nt, logN):
    N = 1 << logN
    moduli = _moduli(N, 3)
    B = 2
    for in_f in (1, 2, 4):
        a = _inputs(200 + in_f, N, moduli, B, in_f)
        lazy, canon = empty32(a.size), empty32(a.size)
        da = dev32(a)
        nt.ntt_forward_rns32(lazy, da, N, moduli, B, in_f, 4)
        nt.ntt_forward_rns32(canon, da, N, moduli, B, in_f, 1)
        gl, gc = host32(lazy), host32(canon)
        for p in range(B):
            for l, q in enumerate(moduli):
                s = slice((p * len(moduli) + l) * N, (p * len(moduli) + l + 1) * N)
                psi = oracle.min_root(N, q)
                model = oracle.harvey_forward_w(a[s], q, psi, out_f=4, bits=32)
                assert np.array_equal(gl[s], model), (in_f, p, l, q)
                assert np.array_equal(gc[s], oracle.harvey_forward_w(a[s], q, psi, out_f=1, bits=32))
                if N <= 1024:
                    assert np.array_equal(gc[s], oracle.ntt_forward(a[s], q, psi))
                else:
                    idx = _idx(N, 201)
                    assert np.array_equal(gc[s][idx], oracle.ntt_forward_at(a[s], idx, q, psi))


@pytest.mark.parametrize("logN", LOGNS)
def test_inverse32_definition_and_ranges(nt, logN):
    N = 1 << logN
    moduli = _moduli(N, 3)
    B = 2
    for in_f in (1, 2):
        A = _inputs(210 + in_f, N, moduli, B, in_f)
        lazy, canon = empty32(A.size), empty32(A.size)
        dA = dev32(A)
        nt.ntt_inverse_rns32(lazy, dA, N, moduli, B, in_f, 2)
        nt.ntt_inverse_rns32(canon, dA, N, moduli, B, in_f, 1)
        gl, gc = host32(lazy), host32(canon)
        for p in range(B):
            for l, q in enumerate(moduli):
                s = slice((p * len(moduli) + l) * N, (p * len(moduli) + l + 1) * N)
                psi = oracle.min_root(N, q)
                assert np.all(gl[s] < np.uint64(2 * q)) and np.all(gc[s] < np.uint64(q))
                assert np.array_equal(gl[s] % np.uint64(q), gc[s])
                assert np.array_equal(gc[s], oracle.harvey_inverse(A[s], q, psi, 1)), (in_f, p, l, q)
                if N <= 1024:
                    assert np.array_equal(gc[s], oracle.ntt_inverse(A[s], q, psi)), (in_f, p, l, q)
                else:
                    idx = _idx(N, 211)
                    assert np.array_equal(gc[s][idx], oracle.ntt_inverse_at(A[s], idx, q, psi))


def test_round_trip32_in_place(nt):
    """The canonical forward in place, then the canonical inverse in place, gives the
    input back (three polynomials of eight limbs at N = 2^14)."""
    N = 1 << 14
    moduli = SMALL
    B = 3
    a = _inputs(220, N, moduli, B, 1)
    d = dev32(a)
    nt.ntt_forward_rns32(d, d, N, moduli, B, 1, 1)
    nt.ntt_inverse_rns32(d, d, N, moduli, B, 1, 1)
    assert np.array_equal(host32(d), a)


@pytest.mark.parametrize("logN", [1, 3, 6, 10, 12, 13, 14, 15, 16, 17])
def test_product32_against_schoolbook(nt, logN):
    N = 1 << logN
    moduli = _moduli(N, 3)
    B = 2
    a = _inputs(230, N, moduli, B, 1)
    b = _inputs(231, N, moduli, B, 1)
    out = empty32(a.size)
    nt.poly_mul_rns32(out, dev32(a), dev32(b), N, moduli, B, _ws(N, a.size))
    got = host32(out)
    # in place on a
    da = dev32(a)
    nt.poly_mul_rns32(da, da, dev32(b), N, moduli, B, _ws(N, a.size))
    assert np.array_equal(host32(da), got)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * len(moduli) + l) * N, (p * len(moduli) + l + 1) * N)
            if N <= 1024:
                assert np.array_equal(got[s], oracle.negacyclic_mul(a[s], b[s], q)), (p, l, q)
            else:
                # every output: the oracle's product through its transforms (pinned to the schoolbook
                # product on the CPU), and sampled outputs of the schoolbook definition itself
                assert np.array_equal(got[s], oracle.product_batch(a[s], b[s], N, q)), (p, l, q)
                idx = _idx(N, 232, 12)
                assert np.array_equal(got[s][idx], oracle.negacyclic_mul_at(a[s], b[s], idx, q)), (p, l, q)


@pytest.mark.parametrize("logN", [2, 10, 14, 15, 16, 17])
def test_product32_acc_with_lazy_multipliers(nt, logN):
    """acc += InvNTT(NTT(b) (.) m) with m crafted in [0, 4q) up to 4q - 1 (the input
    factor 4 of the multiply), against the oracle's transforms and element-wise product."""
    N = 1 << logN
    moduli = _moduli(N, 4)
    m = _inputs(240, N, moduli, 1, 4)
    for l, q in enumerate(moduli):
        ext = np.array([0, q - 1, q, 2 * q, 3 * q + 1, 4 * q - 1], dtype=np.uint64)
        m[l * N:l * N + min(N, ext.size)] = ext[:N]
    b = _inputs(241, N, moduli, 1, 1)
    acc0 = _inputs(242, N, moduli, 1, 1)
    dacc = dev32(acc0)
    nt.poly_mul_acc_ntt_rns32(dacc, dev32(m), dev32(b), N, moduli, 1, _ws(N, m.size))
    got = host32(dacc)
    for l, q in enumerate(moduli):
        s = slice(l * N, (l + 1) * N)
        psi = oracle.min_root(N, q)
        if N <= 1024:
            pm = oracle.eltwise_mult(oracle.ntt_forward(b[s], q, psi), m[s] % np.uint64(q), q)
            assert np.array_equal(got[s], oracle.eltwise_add(acc0[s], oracle.ntt_inverse(pm, q, psi), q)), (l, q)
        else:
            pm = oracle.eltwise_mult(oracle.harvey_forward(b[s], q, psi, 1), m[s] % np.uint64(q), q)
            want = oracle.eltwise_add(acc0[s], oracle.harvey_inverse(pm, q, psi, 1), q)
            assert np.array_equal(got[s], want), (l, q)


def test_product32_pipeline_matches_64bit_path(nt):
    """The same small-modulus product through the 32-bit calls and the 64-bit calls:
    canonical results are equal word for word."""
    from gpu_util import empty_dev, from_dev, to_dev
    N = 1 << 12
    moduli = SMALL[:4]
    B = 2
    a = _inputs(250, N, moduli, B, 1)
    b = _inputs(251, N, moduli, B, 1)
    r32 = empty32(a.size)
    nt.poly_mul_rns32(r32, dev32(a), dev32(b), N, moduli, B)
    r64 = empty_dev(a.size)
    nt.poly_mul_rns(r64, to_dev(a), to_dev(b), N, moduli, B, None)
    assert np.array_equal(host32(r32), from_dev(r64))


@pytest.mark.parametrize("key,B", [("small_16384", 512), ("small_65536", 128)])
def test_small_prime_step_full_size(nt, key, B):
    """The benchmark's word-size-2^32 steps at their full size: B polynomials x 8 limbs of the
    largest primes below 2^30 that suit N (N = 2^14 on chip, N = 2^16 in two passes), forward(a)
    1 -> 4 then the fused product into acc, twice (so acc accumulates).  The canonical
    accumulator equals the 64-bit path's on the same moduli word for word over the whole array,
    and whole limbs equal the oracle's product (Section 2), with sampled outputs of the
    schoolbook definition."""
    import torch
    from gpu_util import empty_dev, from_dev, to_dev
    N = PRIMES[key]["N"]
    moduli = PRIMES[key]["moduli"]
    L = len(moduli)
    a = _inputs(260, N, moduli, B, 1)
    b = _inputs(261, N, moduli, B, 1)
    da32, db32 = dev32(a), dev32(b)
    c32, acc32 = empty32(a.size), torch.zeros(a.size, dtype=torch.int32, device="cuda:0")
    da64, db64 = to_dev(a), to_dev(b)
    c64, acc64 = empty_dev(a.size), torch.zeros(a.size, dtype=torch.int64, device="cuda:0")
    ws32 = _ws(N, a.size)
    ws64 = empty_dev(2 * a.size) if N > (1 << 14) else None
    for _ in range(2):
        nt.ntt_forward_rns32(c32, da32, N, moduli, B, 1, 4)
        nt.poly_mul_acc_ntt_rns32(acc32, c32, db32, N, moduli, B, ws32)
        nt.ntt_forward_rns(c64, da64, N, moduli, B, 1, 4)
        nt.poly_mul_acc_ntt_rns(acc64, c64, db64, N, moduli, B, ws64)
    got = host32(acc32)
    assert np.array_equal(got, from_dev(acc64))
    idx = _idx(N, 262, 6)
    for p, l in [(0, 0), (B // 2, 3), (B - 1, 7)]:
        q = moduli[l]
        s = slice((p * L + l) * N, (p * L + l + 1) * N)
        whole = oracle.product_batch(a[s], b[s], N, q)
        assert np.array_equal(got[s], oracle.eltwise_add(whole, whole, q)), (p, l)
        prod = oracle.negacyclic_mul_at(a[s], b[s], idx, q)
        assert np.array_equal(got[s][idx], oracle.eltwise_add(prod, prod, q)), (p, l)
