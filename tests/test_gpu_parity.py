"""GPU parity: every HIP result is compared with the CPU oracle on the same
seeded inputs.  Integer work, so the bar is bit-exact: canonical outputs equal
the oracle; lazy outputs (output_mod_factor 4 forward, 2 inverse) lie in
[0, f q) and reduce to the oracle's value mod q; where the kernels run the
paper's butterflies, forward lazy outputs also equal the Harvey model bit for
bit (the wide-range butterflies give other representatives; test_gpu_wide.py)."""
import json
import os

import numpy as np
import pytest

import oracle
from synthetic import lazy_mod, uniform_mod, unit_seed
from gpu_util import empty_dev, from_dev, have_gpu, lazy_words_exact, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRIMES = json.load(open(os.path.join(ROOT, "tests", "golden", "primes.json")))


@pytest.fixture(scope="module")
def nt():
    import paper_2103_16400_amd as nt
    return nt


def _prime(logN, which=0, bits=50):
    return oracle.find_primes(bits, 2 << logN, which + 1)[which]


def _edge(Q, k=0):
    return PRIMES["edge"]["by_bits"][str(Q)][k]


def _fwd_check(out, a, q, psi, out_f, full=True, idx=None):
    import paper_2103_16400_amd as nt
    assert np.all(out < np.uint64(out_f * q)), "output outside [0, out_f q)"
    if full:
        ref = oracle.ntt_forward(a, q, psi)
        assert np.array_equal(out % np.uint64(q), ref)
        if out_f == 4 and lazy_words_exact(nt, a.size, [q]):
            assert np.array_equal(out, oracle.harvey_forward(a, q, psi, 4))
    else:
        ref = oracle.ntt_forward_at(a, idx, q, psi)
        assert np.array_equal(out[idx] % np.uint64(q), ref)
        assert np.array_equal(out % np.uint64(q), oracle.harvey_forward(a, q, psi, 1))


def _sample_idx(N, seed, k=48):
    r = uniform_mod(unit_seed(seed, N), k, N).astype(np.uint64)
    return np.unique(np.concatenate([r, np.array([0, 1, N // 2, N - 1], dtype=np.uint64)]))


def _prod_ref(a, b, q):
    """Canonical negacyclic product of one limb: the schoolbook definition (Section 2) up to
    N = 1024, above that the oracle's O(N log N) pipeline through its transforms (the product
    listing of Section 4), which CPU tests pin to the schoolbook product."""
    if a.size <= 1024:
        return oracle.negacyclic_mul(a, b, q)
    return oracle.product_batch(a, b, a.size, q)


def _fwd_canon(a, q):
    """Canonical forward transform of one limb (inputs below 4q): direct sums up to N = 1024,
    above that the Harvey model with a final correction (pinned to the direct sums)."""
    psi = oracle.min_root(a.size, q)
    return oracle.ntt_forward(a, q, psi) if a.size <= 1024 else oracle.harvey_forward(a, q, psi, 1)


def _inv_canon(A, q):
    """Canonical inverse transform of one limb (inputs below 2q), as _fwd_canon."""
    psi = oracle.min_root(A.size, q)
    return oracle.ntt_inverse(A, q, psi) if A.size <= 1024 else oracle.harvey_inverse(A, q, psi, 1)


# ---------------------------------------------------------------- element-wise

@pytest.mark.parametrize("n", [1, 2, 3, 17, 1024, 4097, (1 << 20) + 3])
def test_eltwise_add_and_mult(nt, n):
    for q in [2, 3, 12289, _edge(50), _edge(62, 1), (1 << 62) - 57]:
        a = uniform_mod(unit_seed(1, n, q), n, q)
        b = uniform_mod(unit_seed(2, n, q), n, q)
        da, db, dc = to_dev(a), to_dev(b), empty_dev(n)
        nt.eltwise_add_mod(dc, da, db, n, q)
        assert np.array_equal(from_dev(dc), oracle.eltwise_add(a, b, q))
        nt.eltwise_mult_mod(dc, da, db, n, q, 1)
        assert np.array_equal(from_dev(dc), oracle.eltwise_mult(a, b, q))
    q = (1 << 63) - 25
    a = uniform_mod(unit_seed(3, n), n, q)
    b = uniform_mod(unit_seed(4, n), n, q)
    dc = empty_dev(n)
    nt.eltwise_add_mod(dc, to_dev(a), to_dev(b), n, q)
    assert np.array_equal(from_dev(dc), oracle.eltwise_add(a, b, q))


@pytest.mark.parametrize("n", [1, 3, 1024, 4097, (1 << 18) + 5])
def test_eltwise_fma_sub_negate(nt, n):
    """Algorithm 10 (vector-scalar multiply-add) for every input factor, with and
    without the addend, in place; subtraction and negation (zero residues too)."""
    for q in [2, 3, 12289, _edge(50), _edge(61), (1 << 61) - 1]:
        for f in (1, 2, 4, 8):
            if f * q >= (1 << 64):
                continue
            a = lazy_mod(unit_seed(20, n, q, f), n, q, f)
            z = lazy_mod(unit_seed(21, n, q, f), n, q, f)
            top = np.uint64(f * q - 1)
            a[: max(1, n // 8)] = top
            for y in (0, 1, q - 1, int(uniform_mod(unit_seed(22, q, f), 1, q)[0]), q + 5):
                da, dz, dc = to_dev(a), to_dev(z), empty_dev(n)
                nt.eltwise_fma_mod(dc, da, y, dz, n, q, f)
                assert np.array_equal(from_dev(dc), oracle.eltwise_fma(a, y, z, q)), (q, f, y)
                nt.eltwise_fma_mod(da, da, y, None, n, q, f)                  # in place, no addend
                assert np.array_equal(from_dev(da), oracle.eltwise_fma(a, y, None, q)), (q, f, y)
        a = uniform_mod(unit_seed(23, n, q), n, q)
        b = uniform_mod(unit_seed(24, n, q), n, q)
        a[0] = 0
        b[-1] = a[-1]
        da, db, dc = to_dev(a), to_dev(b), empty_dev(n)
        nt.eltwise_sub_mod(dc, da, db, n, q)
        assert np.array_equal(from_dev(dc), oracle.eltwise_sub(a, b, q))
        nt.eltwise_negate_mod(da, da, n, q)
        assert np.array_equal(from_dev(da), oracle.eltwise_negate(a, q))


def test_eltwise_fma_rns(nt):
    N, B = 4096 + 2, 3
    moduli = PRIMES["serving"]["moduli"][:5]
    moduli = [q for q in moduli if q < (1 << 61)][:3]
    L = len(moduli)
    scalars = [int(uniform_mod(unit_seed(25, l), 1, q)[0]) for l, q in enumerate(moduli)]
    a = np.concatenate([lazy_mod(unit_seed(26, p, l), N, q, 4) for p in range(B) for l, q in enumerate(moduli)])
    z = np.concatenate([lazy_mod(unit_seed(27, p, l), N, q, 4) for p in range(B) for l, q in enumerate(moduli)])
    dc = empty_dev(a.size)
    nt.eltwise_fma_mod_rns(dc, to_dev(a), scalars, to_dev(z), N, moduli, B, 4)
    got = from_dev(dc)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            assert np.array_equal(got[s], oracle.eltwise_fma(a[s], scalars[l], z[s], q)), (p, l)


@pytest.mark.parametrize("Q", list(range(30, 63)))
def test_eltwise_mult_barrett_edges(nt, Q):
    """Smallest Q-bit primes (Barrett's quotient estimate is weakest just above
    2^(Q-1)), all input factors, uniform operands and operands near f q - 1."""
    n = 1 << 14
    for q in PRIMES["edge"]["by_bits"][str(Q)]:
        for f in (1, 2, 4):
            if f * q >= (1 << 63):
                continue
            a = lazy_mod(unit_seed(5, Q, q, f), n, q, f)
            b = lazy_mod(unit_seed(6, Q, q, f), n, q, f)
            top = np.uint64(f * q - 1)
            a[: n // 8] = top - (a[: n // 8] % np.uint64(1024))
            b[: n // 16] = top
            dc = empty_dev(n)
            nt.eltwise_mult_mod(dc, to_dev(a), to_dev(b), n, q, f)
            assert np.array_equal(from_dev(dc), oracle.eltwise_mult(a, b, q)), (q, f)


def test_eltwise_in_place_and_unaligned(nt):
    q = _edge(55)
    n = 1001
    a = uniform_mod(unit_seed(7), n + 1, q)
    b = uniform_mod(unit_seed(8), n + 1, q)
    da, db = to_dev(a), to_dev(b)
    # unaligned views (offset by one word) take the scalar path
    dc = empty_dev(n + 1)
    nt.eltwise_mult_mod(dc[1:], da[1:], db[1:], n, q, 1)
    assert np.array_equal(from_dev(dc)[1:], oracle.eltwise_mult(a[1:], b[1:], q))
    nt.eltwise_add_mod(da, da, db, n + 1, q)          # in place
    assert np.array_equal(from_dev(da), oracle.eltwise_add(a, b, q))


# ---------------------------------------------------------------- single-limb NTT

@pytest.mark.parametrize("logN", list(range(1, 14)))
def test_forward_inverse_small(nt, logN):
    N = 1 << logN
    for q in [_prime(logN, 0, 50), _prime(logN, 0, 62), _prime(logN, 1, 40)]:
        psi = oracle.min_root(N, q)
        for in_f in (1, 2, 4):
            a = lazy_mod(unit_seed(10, logN, q, in_f), N, q, in_f)
            da = to_dev(a)
            for out_f in (1, 4):
                dout = empty_dev(N)
                nt.ntt_forward(dout, da, N, q, in_f, out_f)
                _fwd_check(from_dev(dout), a, q, psi, out_f)
        A = oracle.ntt_forward(uniform_mod(unit_seed(11, logN, q), N, q), q, psi)
        for in_f in (1, 2):
            Ain = lazy_mod(unit_seed(12, logN, q, in_f), N, q, in_f)
            ref = oracle.ntt_inverse(Ain, q, psi)
            dA = to_dev(Ain)
            for out_f in (1, 2):
                dout = empty_dev(N)
                nt.ntt_inverse(dout, dA, N, q, in_f, out_f)
                out = from_dev(dout)
                assert np.all(out < np.uint64(out_f * q))
                assert np.array_equal(out % np.uint64(q), ref)
        # round trip in place
        a = uniform_mod(unit_seed(13, logN, q), N, q)
        d = to_dev(a)
        nt.ntt_forward(d, d, N, q, 1, 4)
        d2 = to_dev(from_dev(d) % np.uint64(q))
        nt.ntt_inverse(d2, d2, N, q, 1, 1)
        assert np.array_equal(from_dev(d2), a)


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("logN", [10, 14, 16])
def test_transform_words_across_modulus_sizes(nt, logN, wide):
    """Every modulus size Q = 30..62 (the smallest Q-bit prime = 1 mod 2^18), through the
    on-chip (2^10), split-exchange on-chip (2^14) and two-pass (2^16) kernels: the forward's
    lazy words equal the Harvey model in full where the paper's butterflies run (always with
    the wide range off; with it on, the lazy words are checked by range and residue), and the
    inverse's canonical output equals the model's (itself pinned to the definition)."""
    N = 1 << logN
    nt.set_wide_range(wide)
    try:
        for Q in range(30, 63):
            _words_one_size(nt, N, logN, Q)
    finally:
        nt.set_wide_range(True)


def _words_one_size(nt, N, logN, Q):
    q = _edge(Q)
    psi = oracle.min_root(N, q)
    a = lazy_mod(unit_seed(24, logN, Q), N, q, 4)
    a[-1] = np.uint64(4 * q - 1)
    dout = empty_dev(N)
    nt.ntt_forward(dout, to_dev(a), N, q, 4, 4)
    model = oracle.harvey_forward(a, q, psi, 4)
    got = from_dev(dout)
    if lazy_words_exact(nt, N, [q]):
        assert np.array_equal(got, model), Q
    else:
        assert np.all(got < np.uint64(4 * q)), Q
        assert np.array_equal(got % np.uint64(q), model % np.uint64(q)), Q
    A = lazy_mod(unit_seed(25, logN, Q), N, q, 2)
    A[0] = np.uint64(2 * q - 1)
    nt.ntt_inverse(dout, to_dev(A), N, q, 2, 1)
    assert np.array_equal(from_dev(dout), oracle.harvey_inverse(A, q, psi, 1)), Q


@pytest.mark.parametrize("logN", [14, 15, 16, 17])
def test_forward_inverse_multipass(nt, logN):
    N = 1 << logN
    for q in [_prime(logN, 0, 50), _prime(logN, 0, 61)]:
        psi = oracle.min_root(N, q)
        idx = _sample_idx(N, logN)
        for in_f, out_f in [(1, 1), (4, 4), (2, 4)]:
            a = lazy_mod(unit_seed(20, logN, q, in_f), N, q, in_f)
            dout = empty_dev(N)
            nt.ntt_forward(dout, to_dev(a), N, q, in_f, out_f)
            out = from_dev(dout)
            _fwd_check(out, a, q, psi, out_f, full=False, idx=idx)
            if out_f == 4:   # the whole lazy output equals the Harvey model (O(N log N) on the CPU)
                model = oracle.harvey_forward(a, q, psi, 4)
                if lazy_words_exact(nt, N, [q]):
                    assert np.array_equal(out, model)
                else:
                    assert np.array_equal(out % np.uint64(q), model % np.uint64(q))
        for in_f, out_f in [(1, 1), (2, 2)]:
            A = lazy_mod(unit_seed(21, logN, q, in_f), N, q, in_f)
            dout = empty_dev(N)
            nt.ntt_inverse(dout, to_dev(A), N, q, in_f, out_f)
            out = from_dev(dout)
            assert np.all(out < np.uint64(out_f * q))
            assert np.array_equal(out[idx] % np.uint64(q), oracle.ntt_inverse_at(A, idx, q, psi))
            assert np.array_equal(out % np.uint64(q), oracle.harvey_inverse(A, q, psi, 1))
        # round trip
        a = uniform_mod(unit_seed(22, logN, q), N, q)
        d = to_dev(a)
        nt.ntt_forward(d, d, N, q, 1, 1)
        nt.ntt_inverse(d, d, N, q, 1, 1)
        assert np.array_equal(from_dev(d), a)


def test_explicit_root_plans(nt):
    for logN in [3, 10, 14]:
        N = 1 << logN
        q = _prime(logN, 2, 58)
        psi_min = oracle.min_root(N, q)
        psi = pow(psi_min, 2 * 5 + 1, q)       # another primitive 2N-th root
        plan = nt.Plan(N, q, psi)
        assert plan.root == psi
        assert nt.Plan(N, q).root == psi_min
        a = uniform_mod(unit_seed(30, logN), N, q)
        d, o = to_dev(a), empty_dev(N)
        plan.forward(o, d, 1, 1)
        out = from_dev(o)
        if N <= 4096:
            assert np.array_equal(out, oracle.ntt_forward(a, q, psi))
        else:
            idx = _sample_idx(N, 31)
            assert np.array_equal(out[idx], oracle.ntt_forward_at(a, idx, q, psi))
            assert np.array_equal(out, oracle.harvey_forward(a, q, psi, 1))
        plan.inverse(o, o, 1, 1)
        assert np.array_equal(from_dev(o), a)
        plan.close()
    with pytest.raises(nt.NttError) as e:
        nt.Plan(8, 17, 2)          # 2^8 = 1 mod 17, not -1: not a primitive 16th root
    assert e.value.status == nt.NTT_EINVAL_ROOT
    with pytest.raises(nt.NttError) as e:
        nt.Plan(8, 17 * 97 + 0, 0)
    assert e.value.status == nt.NTT_EINVAL_MODULUS


def test_composite_modulus_rejected(nt):
    N = 1024
    q = 2049 * 2048 + 1           # = 1 mod 2048
    while oracle.is_prime(q):
        q += 2048
    d = empty_dev(N)
    with pytest.raises(nt.NttError) as e:
        nt.ntt_forward(d, d, N, q)
    assert e.value.status == nt.NTT_EINVAL_MODULUS


# ---------------------------------------------------------------- RNS batches

def _rns_inputs(tag, N, moduli, B, f=1):
    L = len(moduli)
    out = np.empty(B * L * N, dtype=np.uint64)
    for p in range(B):
        for l, q in enumerate(moduli):
            out[(p * L + l) * N:(p * L + l + 1) * N] = lazy_mod(unit_seed(tag, p, l, q), N, q, f)
    return out


def _variant_count(nt, N):
    v = 0
    while True:
        try:
            nt.set_variant(N, 2, True, v)
        except nt.NttError:
            return v
        v += 1


@pytest.mark.parametrize("logN", [15, 16, 17])
def test_two_pass_schedule_variants(nt, logN):
    """Every schedule variant of the two-pass kernels (threads per tile of each
    pass) gives the oracle's words: forward lazy (equal to the Harvey model),
    canonical and fused multiply; inverse canonical and fused accumulate."""
    N = 1 << logN
    moduli = PRIMES["serving"]["moduli"][7:9]
    L = len(moduli)
    psis = [oracle.min_root(N, q) for q in moduli]
    a = _rns_inputs(80, N, moduli, 1, 4)
    m = _rns_inputs(81, N, moduli, 1, 4)
    acc0 = _rns_inputs(82, N, moduli, 1, 1)
    A = _rns_inputs(83, N, moduli, 1, 2)
    idx = _sample_idx(N, 84, 10)
    ref_fwd = [oracle.ntt_forward_at(a[l * N:(l + 1) * N], idx, q, psis[l]) for l, q in enumerate(moduli)]
    harvey0 = oracle.harvey_forward(a[:N], moduli[0], psis[0], 4)
    ref_inv = [oracle.ntt_inverse_at(A[l * N:(l + 1) * N], idx, q, psis[l]) for l, q in enumerate(moduli)]
    full_fwd = [oracle.harvey_forward(a[l * N:(l + 1) * N], q, psis[l], 1) for l, q in enumerate(moduli)]
    full_inv = [oracle.harvey_inverse(A[l * N:(l + 1) * N], q, psis[l], 1) for l, q in enumerate(moduli)]
    nv = _variant_count(nt, N)
    assert nv >= 11                     # thread shapes, half-size tiles, two other splits, three passes
    ws = empty_dev(L * N)
    try:
        for v in range(nv):
            nt.set_variant(N, L, True, v)
            nt.set_variant(N, L, False, v)
            da, dout = to_dev(a), empty_dev(L * N)
            nt.ntt_forward_rns(dout, da, N, moduli, 1, 4, 4)
            lazy = from_dev(dout)
            assert np.array_equal(lazy[:N], harvey0), v
            nt.ntt_forward_rns(dout, da, N, moduli, 1, 4, 1)
            canon = from_dev(dout)
            for l, q in enumerate(moduli):
                s = slice(l * N, (l + 1) * N)
                assert np.array_equal(canon[s][idx], ref_fwd[l]), (v, l)
                assert np.array_equal(canon[s], full_fwd[l]), (v, l)
                assert np.array_equal(canon[s], lazy[s] % np.uint64(q)), (v, l)
            dm = to_dev(m)
            nt.ntt_forward_mul_rns(dm, da, dm, N, moduli, 1, 4, ws)
            prod = from_dev(dm)
            for l, q in enumerate(moduli):
                s = slice(l * N, (l + 1) * N)
                assert np.array_equal(prod[s], oracle.eltwise_mult(canon[s], m[s], q)), (v, l)
            dA = to_dev(A)
            nt.ntt_inverse_rns(dout, dA, N, moduli, 1, 2, 1)
            inv = from_dev(dout)
            for l, q in enumerate(moduli):
                assert np.array_equal(inv[l * N:(l + 1) * N][idx], ref_inv[l]), (v, l)
                assert np.array_equal(inv[l * N:(l + 1) * N], full_inv[l]), (v, l)
            dacc = to_dev(acc0)
            nt.ntt_inverse_acc_rns(dacc, dA, N, moduli, 1, 2, ws)
            assert np.array_equal(from_dev(dacc), np.concatenate(
                [oracle.eltwise_add(acc0[l * N:(l + 1) * N], inv[l * N:(l + 1) * N], q) for l, q in enumerate(moduli)])), v
    finally:
        nt.set_variant(N, L, True, 0)
        nt.set_variant(N, L, False, 0)


@pytest.mark.parametrize("logN", [10, 11, 12, 13, 14])
def test_single_pass_variants(nt, logN):
    """Both thread shapes of the single-pass kernel (variant 1: half the coefficients per thread)
    give the oracle's words in every output mode, with the paper's butterflies (a modulus of 60
    bits in the launch) and with the wide-range ones (every modulus below 2^58)."""
    N = 1 << logN
    serving = PRIMES["serving"]["moduli"]
    assert _variant_count(nt, N) == 2
    B = 3
    for moduli in ([serving[2], serving[10]], [serving[0], serving[7]]):
        L = len(moduli)
        items = B * L
        psis = [oracle.min_root(N, q) for q in moduli]
        a = _rns_inputs(86, N, moduli, B, 4)
        A = _rns_inputs(87, N, moduli, B, 2)
        m = _rns_inputs(88, N, moduli, B, 4)
        acc0 = _rns_inputs(89, N, moduli, B, 1)
        lim = [(p * L + l, moduli[l], psis[l]) for p in range(B) for l in range(L)]
        sl = lambda i: slice(i * N, (i + 1) * N)
        harvey = [oracle.harvey_forward(a[sl(i)], q, psi, 4) for i, q, psi in lim]
        fwd_c = [oracle.harvey_forward(a[sl(i)], q, psi, 1) for i, q, psi in lim]
        inv_c = [oracle.harvey_inverse(A[sl(i)], q, psi, 1) for i, q, psi in lim]
        exact = lazy_words_exact(nt, N, moduli)
        ws = empty_dev(items * N)
        try:
            for v in (0, 1):
                nt.set_variant(N, items, True, v)
                nt.set_variant(N, items, False, v)
                da, dout = to_dev(a), empty_dev(items * N)
                nt.ntt_forward_rns(dout, da, N, moduli, B, 4, 4)
                lazy = from_dev(dout)
                nt.ntt_forward_rns(dout, da, N, moduli, B, 4, 1)
                canon = from_dev(dout)
                dm = to_dev(m)
                nt.ntt_forward_mul_rns(dm, da, dm, N, moduli, B, 4, ws)
                prod = from_dev(dm)
                dA = to_dev(A)
                nt.ntt_inverse_rns(dout, dA, N, moduli, B, 2, 1)
                inv = from_dev(dout)
                nt.ntt_inverse_rns(dout, dA, N, moduli, B, 2, 2)
                inv_lazy = from_dev(dout)
                dacc = to_dev(acc0)
                nt.ntt_inverse_acc_rns(dacc, dA, N, moduli, B, 2, ws)
                acc = from_dev(dacc)
                for k, (i, q, psi) in enumerate(lim):
                    s, qq = sl(i), np.uint64(q)
                    assert np.all(lazy[s] < 4 * qq) and np.array_equal(lazy[s] % qq, fwd_c[k]), (v, i)
                    if exact:
                        assert np.array_equal(lazy[s], harvey[k]), (v, i)
                    assert np.array_equal(canon[s], fwd_c[k]), (v, i)
                    assert np.array_equal(prod[s], oracle.eltwise_mult(fwd_c[k], m[s], q)), (v, i)
                    assert np.array_equal(inv[s], inv_c[k]), (v, i)
                    assert np.all(inv_lazy[s] < 2 * qq) and np.array_equal(inv_lazy[s] % qq, inv_c[k]), (v, i)
                    assert np.array_equal(acc[s], oracle.eltwise_add(acc0[s], inv_c[k], q)), (v, i)
        finally:
            nt.set_variant(N, items, True, 0)
            nt.set_variant(N, items, False, 0)


@pytest.mark.parametrize("key,B", [("rns_16384", 2), ("large_65536", 1)])
def test_rns_forward_inverse(nt, key, B):
    N = PRIMES[key]["N"]
    moduli = PRIMES[key]["moduli"]
    L = len(moduli)
    a = _rns_inputs(40, N, moduli, B)
    d = to_dev(a)
    o = empty_dev(a.size)
    nt.ntt_forward_rns(o, d, N, moduli, B, 1, 4)
    out = from_dev(o)
    idx = _sample_idx(N, 41, 16)
    exact = lazy_words_exact(nt, N, moduli)
    for p in range(B):
        for l, q in enumerate(moduli):
            seg = out[(p * L + l) * N:(p * L + l + 1) * N]
            src = a[(p * L + l) * N:(p * L + l + 1) * N]
            assert np.all(seg < np.uint64(4 * q))
            psi = PRIMES[key]["psi"][l]
            if l in (0, L - 1):
                assert np.array_equal(seg[idx] % np.uint64(q), oracle.ntt_forward_at(src, idx, q, psi))
            model = oracle.harvey_forward(src, q, psi, 4)
            if exact:
                assert np.array_equal(seg, model), (p, l)
            else:
                assert np.array_equal(seg % np.uint64(q), model % np.uint64(q)), (p, l)
    # lazy [0, 4q) is not a legal inverse input: reduce on the host first
    canon = to_dev(np.concatenate([
        out[(p * L + l) * N:(p * L + l + 1) * N] % np.uint64(q)
        for p in range(B) for l, q in enumerate(moduli)]))
    nt.ntt_inverse_rns(canon, canon, N, moduli, B, 1, 1)
    assert np.array_equal(from_dev(canon), a)


def test_rns_eltwise(nt):
    N = 4096
    moduli = PRIMES["serving"]["moduli"][:12]
    B = 3
    a = _rns_inputs(50, N, moduli, B, 4)
    b = _rns_inputs(51, N, moduli, B, 4)
    c = empty_dev(a.size)
    nt.eltwise_mult_mod_rns(c, to_dev(a), to_dev(b), N, moduli, B, 4)
    out = from_dev(c)
    L = len(moduli)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            assert np.array_equal(out[s], oracle.eltwise_mult(a[s], b[s], q))
    a1 = _rns_inputs(52, N, moduli, B, 1)
    b1 = _rns_inputs(53, N, moduli, B, 1)
    nt.eltwise_add_mod_rns(c, to_dev(a1), to_dev(b1), N, moduli, B)
    out = from_dev(c)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            assert np.array_equal(out[s], oracle.eltwise_add(a1[s], b1[s], q))


@pytest.mark.parametrize("logN,L,B", [(1, 1, 3), (4, 2, 2), (10, 3, 2), (12, 40, 1), (13, 2, 1), (14, 8, 2),
                                      (16, 2, 1), (17, 1, 1)])
def test_poly_mul_rns(nt, logN, L, B):
    N = 1 << logN
    moduli = PRIMES["serving"]["moduli"][:L]
    a = _rns_inputs(60, N, moduli, B)
    b = _rns_inputs(61, N, moduli, B)
    c = empty_dev(a.size)
    ws = empty_dev(a.size)
    nt.poly_mul_rns(c, to_dev(a), to_dev(b), N, moduli, B, ws)
    out = from_dev(c)
    idx = _sample_idx(N, 62, 12)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            assert np.array_equal(out[s], _prod_ref(a[s], b[s], q)), (p, l)
            if N > 1024:
                assert np.array_equal(out[s][idx], oracle.negacyclic_mul_at(a[s], b[s], idx, q))
    # in place: result == a
    da = to_dev(a)
    nt.poly_mul_rns(da, da, to_dev(b), N, moduli, B, ws)
    assert np.array_equal(from_dev(da), out)


def _lazy_multiplier(tag, N, moduli):
    """Multipliers in [0, 4q) per limb: lazy residues plus the extremes 0, q - 1, q, 2q, 4q - 1."""
    out = _rns_inputs(tag, N, moduli, 1, 4)
    for l, q in enumerate(moduli):
        ext = np.array([0, q - 1, q, 2 * q, 3 * q + 1, 4 * q - 1, 4 * q - 2], dtype=np.uint64)
        out[l * N:l * N + min(N, ext.size)] = ext[:N]
        out[(l + 1) * N - 1] = np.uint64(4 * q - 1)
    return out


# Moduli from 30 to 62 bits, alone and mixed in one launch: the smallest Q-bit
# primes, where Algorithm 8's Barrett quotient estimate is weakest, with
# multipliers crafted up to 4q - 1 (the input factor 4 of the product step).
MUL_EDGE_GROUPS = [[33], [58], [33, 34, 50, 57, 58], [30, 31, 32], [59], [62], [32, 33, 58, 59]]


@pytest.mark.parametrize("logN", [10, 14])
@pytest.mark.parametrize("bits", MUL_EDGE_GROUPS, ids=lambda b: "q" + "_".join(map(str, b)))
def test_product_multiply_edges(nt, logN, bits):
    """acc += InvNTT(NTT(b) (.) m) with m in [0, 4q) crafted up to 4q - 1, through the fused
    on-chip product, against the oracle's transforms and element-wise product; and the
    forward fused with the multiply against NTT(b) (.) (m mod q)."""
    N = 1 << logN
    moduli = [_edge(bt) for bt in bits]
    L = len(moduli)
    b = _rns_inputs(95, N, moduli, 1)
    m = _lazy_multiplier(96, N, moduli)
    acc0 = _rns_inputs(97, N, moduli, 1)
    dacc = to_dev(acc0)
    nt.poly_mul_acc_ntt_rns(dacc, to_dev(m), to_dev(b), N, moduli, 1)
    got = from_dev(dacc)
    dprod = empty_dev(N * L)
    nt.ntt_forward_mul_rns(dprod, to_dev(b), to_dev(m), N, moduli, 1)
    prod = from_dev(dprod)
    for l, q in enumerate(moduli):
        s = slice(l * N, (l + 1) * N)
        fb = _fwd_canon(b[s], q)
        pm = oracle.eltwise_mult(fb, m[s] % np.uint64(q), q)
        assert np.array_equal(prod[s], pm), ("fwd_mul", bits, l)
        want = oracle.eltwise_add(acc0[s], _inv_canon(pm, q), q)
        assert np.array_equal(got[s], want), ("product", bits, l)


@pytest.mark.parametrize("logN,L,B", [(1, 1, 2), (6, 2, 2), (10, 3, 2), (12, 4, 1), (13, 2, 2), (14, 8, 2),
                                      (15, 2, 1), (17, 1, 1)])
def test_poly_mul_acc_ntt(nt, logN, L, B):
    """acc += a * b with a in NTT form: the on-chip fused product (N <= 2^14) and
    the two-launch form above agree with the schoolbook product plus acc."""
    N = 1 << logN
    moduli = PRIMES["serving"]["moduli"][3:3 + L]
    a = _rns_inputs(90, N, moduli, B)
    b = _rns_inputs(91, N, moduli, B)
    acc0 = _rns_inputs(92, N, moduli, B)
    a_ntt = empty_dev(a.size)
    nt.ntt_forward_rns(a_ntt, to_dev(a), N, moduli, B, 1, 4)
    dacc = to_dev(acc0)
    ws = empty_dev(2 * a.size) if N > (1 << 14) else None
    nt.poly_mul_acc_ntt_rns(dacc, a_ntt, to_dev(b), N, moduli, B, ws)
    got = from_dev(dacc)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            ref = oracle.eltwise_add(acc0[s], _prod_ref(a[s], b[s], q), q)
            assert np.array_equal(got[s], ref), (p, l)
    # and the same words as the three-step form through the public entry points
    dacc2 = to_dev(acc0)
    ws2 = empty_dev(2 * a.size)
    nt.poly_mul_acc_rns(dacc2, to_dev(a), to_dev(b), N, moduli, B, ws2)
    assert np.array_equal(from_dev(dacc2), got)


@pytest.mark.parametrize("logN,L,B", [(3, 2, 2), (11, 3, 2), (14, 8, 1), (15, 2, 1), (17, 1, 1)])
def test_fused_forward_mul_and_inverse_acc(nt, logN, L, B):
    N = 1 << logN
    moduli = PRIMES["serving"]["moduli"][5:5 + L]
    a = _rns_inputs(70, N, moduli, B, 4)               # operand with input factor 4
    m = _rns_inputs(71, N, moduli, B, 4)               # lazy multiplier in [0, 4q)
    acc0 = _rns_inputs(72, N, moduli, B, 1)
    A2 = _rns_inputs(73, N, moduli, B, 2)              # inverse operand with input factor 2
    ws = empty_dev(a.size)
    dm = to_dev(m)
    r = empty_dev(a.size)
    nt.ntt_forward_mul_rns(r, to_dev(a), dm, N, moduli, B, 4, ws)
    out = from_dev(r)
    dacc = to_dev(acc0)
    nt.ntt_inverse_acc_rns(dacc, to_dev(A2), N, moduli, B, 2, ws)
    acc = from_dev(dacc)
    idx = _sample_idx(N, 74, 12)
    psis = {q: oracle.min_root(N, q) for q in moduli}
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            fa = _fwd_canon(a[s], q)
            assert np.array_equal(out[s], oracle.eltwise_mult(fa, m[s], q)), (p, l)
            ia = _inv_canon(A2[s], q)
            assert np.array_equal(acc[s], oracle.eltwise_add(acc0[s], ia, q)), (p, l)
            if N > 4096:
                fa = oracle.ntt_forward_at(a[s], idx, q, psis[q])
                assert np.array_equal(out[s][idx], oracle.eltwise_mult(fa, m[s][idx], q))
    # in place: result == multiplier
    nt.ntt_forward_mul_rns(dm, to_dev(a), dm, N, moduli, B, 4, ws)
    assert np.array_equal(from_dev(dm), out)


@pytest.mark.parametrize("logN,L,B", [(5, 3, 2), (12, 4, 2), (14, 8, 2), (16, 2, 1)])
def test_poly_mul_acc_rns(nt, logN, L, B):
    N = 1 << logN
    moduli = PRIMES["serving"]["moduli"][10:10 + L]
    a = _rns_inputs(80, N, moduli, B)
    b = _rns_inputs(81, N, moduli, B)
    acc0 = _rns_inputs(82, N, moduli, B)
    dacc = to_dev(acc0)
    ws = empty_dev(2 * a.size)
    nt.poly_mul_acc_rns(dacc, to_dev(a), to_dev(b), N, moduli, B, ws)
    nt.poly_mul_acc_rns(dacc, to_dev(a), to_dev(b), N, moduli, B, ws)     # twice: acc + 2ab
    acc = from_dev(dacc)
    idx = _sample_idx(N, 83, 10)
    for p in range(B):
        for l, q in enumerate(moduli):
            s = slice((p * L + l) * N, (p * L + l + 1) * N)
            ab = _prod_ref(a[s], b[s], q)
            assert np.array_equal(acc[s], oracle.eltwise_add(oracle.eltwise_add(acc0[s], ab, q), ab, q)), (p, l)
            if N > 1024:
                ab = oracle.negacyclic_mul_at(a[s], b[s], idx, q)
                ref = oracle.eltwise_add(oracle.eltwise_add(acc0[s][idx], ab, q), ab, q)
                assert np.array_equal(acc[s][idx], ref)


# ---------------------------------------------------------------- uneven batches (persistent launch)

def _batch_case(nt, seed, specs):
    """specs: list of (op, logN, q).  Returns (items, host inputs, device tensors)."""
    tasks, host = [], []
    for k, (op, logN, q) in enumerate(specs):
        N = 1 << logN
        a = uniform_mod(unit_seed(seed, k, 1), N, q)
        b = uniform_mod(unit_seed(seed, k, 2), N, q) if op == nt.BATCH_PRODUCT else None
        da = to_dev(a)
        db = to_dev(b) if b is not None else None
        out = empty_dev(N)
        tmp = empty_dev(N) if (op == nt.BATCH_PRODUCT and logN > 14) else None
        tasks.append((op, out, da, db, tmp, N, q))
        host.append((op, logN, q, a, b))
    return tasks, host


def _check_batch_outputs(nt, tasks, host):
    for (op, out, _, _, _, N, q), (_, logN, _, a, b) in zip(tasks, host):
        got = from_dev(out)
        psi = oracle.min_root(N, q)
        full = N <= 2048
        idx = None if full else _sample_idx(N, 90 + logN, 12)
        if op == nt.BATCH_PRODUCT:
            assert np.array_equal(got, _prod_ref(a, b, q)), ("product", logN)
            if not full:
                assert np.array_equal(got[idx], oracle.negacyclic_mul_at(a, b, idx, q)), ("product", logN)
            continue
        fwd = op in (nt.BATCH_FWD, nt.BATCH_FWD_LAZY)
        bound = {nt.BATCH_FWD: 1, nt.BATCH_FWD_LAZY: 4, nt.BATCH_INV: 1, nt.BATCH_INV_LAZY: 2}[op]
        assert np.all(got < np.uint64(bound * q))
        if fwd:
            ref = oracle.ntt_forward(a, q, psi) if full else oracle.ntt_forward_at(a, idx, q, psi)
        else:
            ref = oracle.ntt_inverse(a, q, psi) if full else oracle.ntt_inverse_at(a, idx, q, psi)
        assert np.array_equal((got if full else got[idx]) % np.uint64(q), ref), (op, logN)
        whole = _fwd_canon(a, q) if fwd else _inv_canon(a, q)
        assert np.array_equal(got % np.uint64(q), whole), (op, logN)
        if fwd and bound == 4 and lazy_words_exact(nt, N, [q]):   # the paper's butterflies' lazy words
            assert np.array_equal(got, oracle.harvey_forward(a, q, psi, 4)), logN


def test_batch_uneven_mixed_ops(nt):
    serving = PRIMES["serving"]["moduli"]
    specs = []
    ops = [nt.BATCH_FWD_LAZY, nt.BATCH_FWD, nt.BATCH_INV_LAZY, nt.BATCH_INV, nt.BATCH_PRODUCT]
    k = 0
    for logN in range(10, 18):
        for op in ops:
            specs.append((op, logN, serving[k % len(serving)]))
            k += 1
    tasks, host = _batch_case(nt, 100, specs)
    batch = nt.Batch(64)
    # with the wide-range butterflies (on-chip tasks whose modulus is below 2^58) and with the
    # paper's everywhere: the oracle's results, and the per-call path's words under the same switch
    try:
        for wide in (True, False):
            nt.set_wide_range(wide)
            for t in tasks:
                t[1].zero_()
            batch.run(tasks)
            _check_batch_outputs(nt, tasks, host)
            for (op, out, da, db, tmp, N, q) in tasks:
                ref = empty_dev(N)
                if op == nt.BATCH_FWD_LAZY:
                    nt.ntt_forward(ref, da, N, q, 1, 4)
                elif op == nt.BATCH_FWD:
                    nt.ntt_forward(ref, da, N, q, 1, 1)
                elif op == nt.BATCH_INV:
                    nt.ntt_inverse(ref, da, N, q, 1, 1)
                elif op == nt.BATCH_PRODUCT:
                    nt.poly_mul_rns(ref, da, db, N, [q], 1, empty_dev(N))
                else:
                    continue                 # lazy inverse representatives may differ between schedules
                assert np.array_equal(from_dev(ref), from_dev(out)), (wide, op, N)
    finally:
        nt.set_wide_range(True)
    batch.close()


def test_batch_partial_units_in_place(nt):
    """Blocks whose last unit is partial (N <= 2^14 runs 8, 4, 2, 2, 1 limbs per workgroup; the
    spare sub-groups repeat the unit's first limb and store nothing), half of the transforms in
    place (out = in, which the spare sub-groups read while the first limb is written), and tile
    pairs of the two-pass sizes with an odd number of limbs: every output against the oracle."""
    serving = PRIMES["serving"]["moduli"]
    per_unit = {10: 8, 11: 4, 12: 2, 13: 2, 14: 1}
    specs = []
    for logN, g in per_unit.items():
        for op in (nt.BATCH_FWD_LAZY, nt.BATCH_INV, nt.BATCH_PRODUCT):
            specs += [(op, logN, serving[(logN + j) % len(serving)]) for j in range(2 * g + max(1, g - 1))]
    for logN in (15, 16):
        specs += [(nt.BATCH_FWD, logN, serving[j % len(serving)]) for j in range(3)]
        specs += [(nt.BATCH_INV_LAZY, logN, serving[(j + 5) % len(serving)]) for j in range(3)]
    tasks, host = _batch_case(nt, 140, specs)
    # every other transform in place
    for k, t in enumerate(tasks):
        if t[0] != nt.BATCH_PRODUCT and k % 2 == 0:
            tasks[k] = (t[0], t[2], t[2], t[3], t[4], t[5], t[6])
    batch = nt.Batch(len(tasks))
    batch.run(tasks)
    _check_batch_outputs(nt, tasks, host)
    batch.close()


@pytest.mark.parametrize("shape", [1, 2])
def test_batch_shape_one(nt, shape):
    """Unit shape 1 (twice the threads per limb for N <= 2^13 and per tile of the two-pass sizes;
    2^14 transforms and products keep shape 0) and shape 2 (twice the threads per tile only) give
    the oracle's results for every op and size, with partial units and transforms in place, plain
    and graph-replayed."""
    serving = PRIMES["serving"]["moduli"]
    specs = []
    for logN in range(10, 18):
        for j, op in enumerate((nt.BATCH_FWD_LAZY, nt.BATCH_FWD, nt.BATCH_INV_LAZY, nt.BATCH_INV,
                                nt.BATCH_PRODUCT)):
            specs += [(op, logN, serving[(logN + j + r) % len(serving)]) for r in range(3 if logN <= 13 else 1)]
    tasks, host = _batch_case(nt, 160, specs)
    for k, t in enumerate(tasks):
        if t[0] != nt.BATCH_PRODUCT and k % 3 == 1:
            tasks[k] = (t[0], t[2], t[2], t[3], t[4], t[5], t[6])
    batch = nt.Batch(len(tasks))
    assert batch.config() == (0, 0)
    batch.set_shape(shape)
    for bad in (-1, 3):
        with pytest.raises(nt.NttError):
            batch.set_shape(bad)
    assert batch.config() == (0, shape)
    batch.run(tasks)
    _check_batch_outputs(nt, tasks, host)
    # graph replay on fresh inputs (the in-place tasks consumed theirs)
    tasks, host = _batch_case(nt, 161, specs)
    batch.run(tasks, graph=True)
    _check_batch_outputs(nt, tasks, host)
    batch.close()


def test_batch_item_factors(nt):
    """Per-item input and output factors (the NTT class's input_mod_factor and
    output_mod_factor, Section 4): a batched forward of lazy inputs in [0, 4q) with crafted
    extremes, to lazy and canonical outputs; an inverse of inputs in [0, 2q); a product of
    inputs in [0, 4q); each against the oracle on whole arrays.  Factors outside the
    allowed sets are refused."""
    serving = PRIMES["serving"]["moduli"]
    specs = []
    for k, logN in enumerate([10, 12, 14, 15, 16]):
        q = serving[(5 * k) % len(serving)]
        specs += [(nt.BATCH_FWD_LAZY, logN, q, 4, 4), (nt.BATCH_FWD_LAZY, logN, q, 4, 1),
                  (nt.BATCH_FWD, logN, q, 2, 4), (nt.BATCH_INV, logN, q, 2, 2), (nt.BATCH_INV_LAZY, logN, q, 2, 1),
                  (nt.BATCH_PRODUCT, logN, q, 4, 1)]
    tasks, hosts = [], []
    for k, (op, logN, q, fi, fo) in enumerate(specs):
        N = 1 << logN
        a = lazy_mod(unit_seed(130, k, 1), N, q, fi)
        a[:4] = np.array([fi * q - 1, 0, q - 1, q], dtype=np.uint64)
        b = lazy_mod(unit_seed(130, k, 2), N, q, fi) if op == nt.BATCH_PRODUCT else None
        out = empty_dev(N)
        tmp = empty_dev(N) if (op == nt.BATCH_PRODUCT and logN > 14) else None
        tasks.append((op, out, to_dev(a), to_dev(b) if b is not None else None, tmp, N, q, fi, fo))
        hosts.append((op, N, q, a, b, fo))
    batch = nt.Batch(len(tasks))
    batch.run(tasks)
    for (op, out, *_), (_, N, q, a, b, fo) in zip(tasks, hosts):
        got = from_dev(out)
        qq = np.uint64(q)
        if op == nt.BATCH_PRODUCT:
            assert np.array_equal(got, _prod_ref(a % qq, b % qq, q)), (op, N)
            continue
        fwd = op in (nt.BATCH_FWD, nt.BATCH_FWD_LAZY)
        assert np.all(got < np.uint64(fo * q)), (op, N, fo)
        want = _fwd_canon(a, q) if fwd else _inv_canon(a, q)
        assert np.array_equal(got % qq, want), (op, N, fo)
    d = empty_dev(1024)
    q = PRIMES["single_1024"]["moduli"][0]
    for op, fi, fo in [(nt.BATCH_FWD, 3, 0), (nt.BATCH_FWD, 1, 2), (nt.BATCH_INV, 4, 0), (nt.BATCH_INV, 1, 4),
                       (nt.BATCH_PRODUCT, 1, 4), (nt.BATCH_PRODUCT, 8, 0)]:
        with pytest.raises(nt.NttError) as e:
            batch.run([(op, d, d, d, None, 1024, q, fi, fo)])
        assert e.value.status == nt.NTT_EINVAL_FACTOR, (op, fi, fo)
    batch.close()


def test_batch_graph_replays(nt):
    moduli = PRIMES["uneven"]["moduli"]
    specs1 = [(nt.BATCH_FWD_LAZY, 12 + (k % 4), moduli[k % 16]) for k in range(40)]
    specs2 = [(nt.BATCH_INV, 12 + ((k + 1) % 4), moduli[(3 * k) % 16]) for k in range(23)]
    t1, h1 = _batch_case(nt, 110, specs1)
    t2, h2 = _batch_case(nt, 111, specs2)
    batch = nt.Batch(64)
    batch.run(t1, graph=True)
    _check_batch_outputs(nt, t1, h1)
    first = [from_dev(t[1]).copy() for t in t1]
    import torch
    for rep in range(3):
        for t in t1:
            t[1].zero_()
        torch.cuda.synchronize()
        batch.run(t1, graph=True)                 # replay: same graph, same descriptors
        torch.cuda.synchronize()
        for t, f in zip(t1, first):
            assert np.array_equal(from_dev(t[1]), f), rep
        batch.run(t2, graph=True)                 # replay with a different, smaller batch
        torch.cuda.synchronize()
        _check_batch_outputs(nt, t2, h2)
    batch.close()


def test_batch_counters_across_grids_and_modes(nt):
    """Each phase's claim counter is cleared by the workgroup that draws the phase's last claim
    (units + grid - 1), so it must hold whatever the grid and however plain and graph-replayed
    runs alternate: a grid smaller than the units, one larger than them, a change of grid between
    runs, a change of unit shape (other block layouts on the same counters), batches with and
    without a second phase, all against the oracle."""
    moduli = PRIMES["uneven"]["moduli"]
    with_split = [(nt.BATCH_FWD_LAZY, 12 + (k % 4), moduli[k % 16]) for k in range(9)]   # 2^15 limbs too
    no_split = [(nt.BATCH_INV, 10 + (k % 3), moduli[(5 * k) % 16]) for k in range(7)]
    cases = [_batch_case(nt, 150, with_split), _batch_case(nt, 151, no_split)]
    batch = nt.Batch(16)
    import torch
    for rnd, (grid, graph, shape) in enumerate([(0, False, 0), (3, False, 1), (3, True, 2), (1000, False, 2),
                                                (1000, True, 0), (0, True, 1), (5, False, 0)]):
        batch.set_grid(grid)
        batch.set_shape(shape)
        for tasks, host in cases:
            for t in tasks:
                t[1].zero_()
            torch.cuda.synchronize()
            batch.run(tasks, graph=graph)
            torch.cuda.synchronize()
            _check_batch_outputs(nt, tasks, host)
    batch.close()


def test_batch_one_shot_calls(nt):
    """ntt_batch_forward / _inverse / _product: uneven task lists of one kind through the
    library-owned per-thread context (grown past its first size), against the oracle;
    a task of another kind is refused."""
    serving = PRIMES["serving"]["moduli"]
    for rnd, count in enumerate([30, 3000]):               # the second list outgrows the first context (1024)
        base = [(10 + (k % 8), serving[(k * 7) % len(serving)]) for k in range(count)]
        small = [(lg, q) for lg, q in base if lg <= 12] if count > 100 else base
        for kind, ops, fn in [("fwd", [nt.BATCH_FWD_LAZY, nt.BATCH_FWD], nt.batch_forward),
                              ("inv", [nt.BATCH_INV_LAZY, nt.BATCH_INV], nt.batch_inverse),
                              ("prod", [nt.BATCH_PRODUCT], nt.batch_product)]:
            specs = [(ops[k % len(ops)], lg, q) for k, (lg, q) in enumerate(small)]
            tasks, host = _batch_case(nt, 120 + rnd, specs)
            fn(tasks)
            idx = list(range(0, len(tasks), max(1, len(tasks) // 24)))
            _check_batch_outputs(nt, [tasks[i] for i in idx], [host[i] for i in idx])
    d = empty_dev(1024)
    q = PRIMES["single_1024"]["moduli"][0]
    with pytest.raises(nt.NttError) as e:
        nt.batch_forward([(nt.BATCH_INV, d, d, None, None, 1024, q)])
    assert e.value.status == nt.NTT_EINVAL_FACTOR


def test_batch_rejects_bad_items(nt):
    batch = nt.Batch(4)
    d = empty_dev(1024)
    q = PRIMES["single_1024"]["moduli"][0]
    with pytest.raises(nt.NttError) as e:
        batch.run([(nt.BATCH_PRODUCT, d, d, None, None, 1024, q)])
    assert e.value.status == nt.NTT_EINVAL_POINTER
    with pytest.raises(nt.NttError) as e:
        batch.run([(nt.BATCH_FWD, d, d, None, None, 512, q)])
    assert e.value.status == nt.NTT_EINVAL_DEGREE
    with pytest.raises(nt.NttError) as e:
        batch.run([(nt.BATCH_FWD, d, d, None, None, 1024, q)] * 5)
    assert e.value.status == nt.NTT_EINVAL_COUNT
    batch.close()


def test_bench_step_full_size(nt):
    """The benchmark's step at its full size and launch configuration: 512 polynomials x 8
    limbs of the 50-bit primes at N = 2^14, forward(a) 1 -> 4 in one launch, then the fused
    on-chip product accumulating into acc in one launch.  Checked four ways: every output of
    every limb against the oracle (its product through the transforms, pinned on the CPU to
    the schoolbook product), sampled outputs against the schoolbook definition of Section 2,
    the whole arrays against the same step run with the paper's butterflies
    (ntt_set_wide_range(0)), and every forward output inside [0, 4q)."""
    import torch
    N = PRIMES["rns_16384"]["N"]
    moduli = PRIMES["rns_16384"]["moduli"]
    L, B = len(moduli), 512
    a = _rns_inputs(950, N, moduli, B, 1)
    b = _rns_inputs(951, N, moduli, B, 1)
    acc0 = _rns_inputs(952, N, moduli, B, 1)
    da, db = to_dev(a), to_dev(b)
    results = {}
    try:
        for wide in (True, False):
            nt.set_wide_range(wide)
            a_ntt = empty_dev(a.size)
            nt.ntt_forward_rns(a_ntt, da, N, moduli, B, 1, 4)
            acc = to_dev(acc0)
            nt.poly_mul_acc_ntt_rns(acc, a_ntt, db, N, moduli, B)
            torch.cuda.synchronize()
            qs = torch.tensor([4 * q for q in moduli], dtype=torch.int64, device="cuda:0").repeat(B)
            assert bool((a_ntt.view(B * L, N) < qs[:, None]).all()), wide
            results[wide] = acc
            del a_ntt
    finally:
        nt.set_wide_range(True)
    assert torch.equal(results[True], results[False])
    got = from_dev(results[True])
    # every output of every limb: the oracle's product through its transforms, plus acc
    want = oracle.add_rns(acc0, oracle.product_rns(a, b, N, moduli), N, moduli)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, ("limbs differing from the oracle", np.unique(bad // N)[:16])
    idx = _sample_idx(N, 953, 6)
    for p, l in [(0, 0), (1, 7), (255, 3), (511, 5), (511, 7)]:
        q = moduli[l]
        s = slice((p * L + l) * N, (p * L + l + 1) * N)
        want = oracle.eltwise_add(acc0[s][idx], oracle.negacyclic_mul_at(a[s], b[s], idx, q), q)
        assert np.array_equal(got[s][idx], want), (p, l)


def test_batch_full_size_uneven(nt):
    """The benchmark's uneven batch at its full size and launch configuration: 256
    polynomials, N uniform in {2^12..2^15}, 2..16 limbs of the 50-bit pool (2371 limb
    transforms), the grid autotuned, run as one persistent launch and from a captured
    graph.  Every limb's forward (1 -> 4) and inverse (1 -> 1) equals the per-call path's
    words and the oracle's (Harvey model for the lazy forward, canonical inverse) on the
    whole array, and sampled limbs equal the direct definition at sampled indices."""
    import torch
    from synthetic import uniform_int
    pool = PRIMES["uneven"]["moduli"]
    P = 256
    logNs = uniform_int(unit_seed(4, 0), P, 12, 15)
    Ls = uniform_int(unit_seed(4, 1), P, 2, 16)
    limbs = [(int(logNs[p]), pool[l]) for p in range(P) for l in range(int(Ls[p]))]
    total = sum(1 << n for n, _ in limbs)
    host = np.empty(total, dtype=np.uint64)
    offs, off = [], 0
    for k, (n, q) in enumerate(limbs):
        N = 1 << n
        host[off:off + N] = uniform_mod(unit_seed(5, k, q), N, q)
        offs.append(off)
        off += N
    src = to_dev(host)
    dst, ref = empty_dev(total), empty_dev(total)
    batch = nt.Batch(len(limbs))
    samples = [0, 1, len(limbs) // 2, len(limbs) - 1]
    try:
        for wide in (False, True):
            nt.set_wide_range(wide)       # the batch kernel and the per-call reference take the same butterflies
            for op, fwd in ((nt.BATCH_FWD_LAZY, True), (nt.BATCH_INV, False)):
                items, cnt = nt.Batch.make_items([(op, dst[o:o + (1 << n)], src[o:o + (1 << n)], None, None, 1 << n, q)
                                                  for o, (n, q) in zip(offs, limbs)])
                batch.autotune(items, cnt)
                for graph in (False, True):
                    dst.zero_()
                    batch.run(items, cnt, graph=graph)
                    for o, (n, q) in zip(offs, limbs):
                        N = 1 << n
                        if fwd:
                            nt.ntt_forward(ref[o:o + N], src[o:o + N], N, q, 1, 4)
                        else:
                            nt.ntt_inverse(ref[o:o + N], src[o:o + N], N, q, 1, 1)
                    torch.cuda.synchronize()
                    assert torch.equal(dst, ref), (wide, op, graph)
                got = from_dev(dst)
                # every limb against the oracle: limbs grouped by (N, q), the forward's lazy words equal
                # the Harvey model's (paper butterflies), the inverse's canonical values the definition's
                groups = {}
                for k, (n, q) in enumerate(limbs):
                    groups.setdefault((n, q), []).append(k)
                for (n, q), ks in groups.items():
                    N = 1 << n
                    psi = oracle.min_root(N, q)
                    src_g = np.concatenate([host[offs[k]:offs[k] + N] for k in ks])
                    got_g = np.concatenate([got[offs[k]:offs[k] + N] for k in ks])
                    if fwd and lazy_words_exact(nt, N, [q]):
                        assert np.array_equal(got_g, oracle.harvey_forward_batch(src_g, N, q, psi, 4)), (op, n, q)
                    elif fwd:
                        assert np.all(got_g < np.uint64(4 * q)), (op, n, q)
                        assert np.array_equal(got_g % np.uint64(q), oracle.harvey_forward_batch(src_g, N, q, psi, 1)), (op, n, q)
                    else:
                        assert np.array_equal(got_g, oracle.harvey_inverse_batch(src_g, N, q, psi, 1)), (op, n, q)
                for k in samples:
                    n, q = limbs[k]
                    N, o = 1 << n, offs[k]
                    a = host[o:o + N]
                    idx = _sample_idx(N, 960 + k, 8)
                    psi = oracle.min_root(N, q)
                    want = oracle.ntt_forward_at(a, idx, q, psi) if fwd else oracle.ntt_inverse_at(a, idx, q, psi)
                    assert np.array_equal(got[o:o + N][idx] % np.uint64(q), want), (op, k)
                    if fwd:
                        assert np.all(got[o:o + N] < np.uint64(4 * q))
                    else:
                        assert np.all(got[o:o + N] < np.uint64(q))
    finally:
        nt.set_wide_range(True)
        batch.close()
