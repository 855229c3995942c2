"""GPU tests of the validation mode (ntt_set_validate): with it on, calls whose operand
values leave the stated range [0, f q) return NTT_ERANGE and launch nothing; calls with
values inside the range (up to f q - 1) run and give the same words as with it off."""
import json
import os

import numpy as np
import pytest

from synthetic import lazy_mod, unit_seed
from gpu_util import empty_dev, from_dev, have_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRIMES = json.load(open(os.path.join(ROOT, "tests", "golden", "primes.json")))
MODS = PRIMES["rns_16384"]["moduli"][:3]
SMALL = PRIMES["small_16384"]["moduli"][:2]


@pytest.fixture()
def nt():
    import paper_2103_16400_amd as nt
    nt.set_validate(True)
    try:
        yield nt
    finally:
        nt.set_validate(False)


def _lazy(tag, N, moduli, f, B=1):
    out = np.concatenate([lazy_mod(unit_seed(tag, p, l, q), N, q, f) for p in range(B) for l, q in enumerate(moduli)])
    for p in range(B):
        for l, q in enumerate(moduli):
            out[(p * len(moduli) + l + 1) * N - 1] = np.uint64(f * q - 1)     # the top of the range
    return out.astype(np.uint64)


def _erange(nt, fn):
    with pytest.raises(nt.NttError) as e:
        fn()
    assert e.value.status == nt.NTT_ERANGE


def test_in_range_runs_and_matches_unvalidated(nt):
    N = 1 << 12
    a = _lazy(1, N, MODS, 4, 2)
    out_v = empty_dev(a.size)
    nt.ntt_forward_rns(out_v, to_dev(a), N, MODS, 2, 4, 4)
    nt.set_validate(False)
    out = empty_dev(a.size)
    nt.ntt_forward_rns(out, to_dev(a), N, MODS, 2, 4, 4)
    nt.set_validate(True)
    assert np.array_equal(from_dev(out_v), from_dev(out))


def test_out_of_range_rejected_before_launch(nt):
    N = 1 << 12
    L = len(MODS)
    sentinel = np.full(N * L, 7, dtype=np.uint64)
    for f, fwd in [(1, True), (2, True), (4, True), (1, False), (2, False)]:
        a = _lazy(2, N, MODS, f)
        a[L * N // 2] = np.uint64(f * MODS[1])                 # limb 1 gets the value f q
        out = to_dev(sentinel)
        call = nt.ntt_forward_rns if fwd else nt.ntt_inverse_rns
        _erange(nt, lambda: call(out, to_dev(a), N, MODS, 1, f, 1))
        assert np.array_equal(from_dev(out), sentinel), (f, fwd)
        a[L * N // 2] = np.uint64(f * MODS[1] - 1)
        call(out, to_dev(a), N, MODS, 1, f, 1)                 # the top of the range is accepted
    # single-modulus calls and a plan
    q = MODS[0]
    x = _lazy(3, N, [q], 1)
    x[5] = np.uint64(q)
    o = empty_dev(N)
    _erange(nt, lambda: nt.ntt_forward(o, to_dev(x), N, q, 1, 1))
    plan = nt.Plan(N, q)
    _erange(nt, lambda: plan.forward(o, to_dev(x), 1, 1))


def test_element_wise_and_products(nt):
    N = 1 << 10
    L = len(MODS)
    ok = _lazy(4, N, MODS, 1)
    bad = ok.copy()
    bad[N + 3] = np.uint64(MODS[1])
    d_ok, d_bad, o = to_dev(ok), to_dev(bad), empty_dev(ok.size)
    _erange(nt, lambda: nt.eltwise_mult_mod_rns(o, d_ok, d_bad, N, MODS, 1, 1))
    _erange(nt, lambda: nt.eltwise_add_mod_rns(o, d_bad, d_ok, N, MODS, 1))
    nt.eltwise_mult_mod_rns(o, d_ok, d_ok, N, MODS, 1, 1)
    two = _lazy(5, N, MODS, 2)
    nt.eltwise_mult_mod_rns(o, to_dev(two), d_ok, N, MODS, 1, 2)
    two[0] = np.uint64(2 * MODS[0])
    _erange(nt, lambda: nt.eltwise_mult_mod_rns(o, to_dev(two), d_ok, N, MODS, 1, 2))
    q = MODS[0]
    s_ok, s_bad = to_dev(ok[:N]), to_dev(np.full(N, q, dtype=np.uint64))
    o1 = empty_dev(N)
    _erange(nt, lambda: nt.eltwise_sub_mod(o1, s_ok, s_bad, N, q))
    _erange(nt, lambda: nt.eltwise_negate_mod(o1, s_bad, N, q))
    _erange(nt, lambda: nt.eltwise_fma_mod(o1, s_bad, 5, None, N, q, 1))
    nt.eltwise_fma_mod(o1, s_bad, 5, None, N, q, 2)            # q < 2q: in range for factor 2
    # products: b and acc below q, the transformed operand below 4q
    m = _lazy(6, N, MODS, 4)
    acc = to_dev(ok)
    nt.poly_mul_acc_ntt_rns(acc, to_dev(m), d_ok, N, MODS, 1)
    m[7] = np.uint64(4 * MODS[0])
    _erange(nt, lambda: nt.poly_mul_acc_ntt_rns(acc, to_dev(m), d_ok, N, MODS, 1))
    _erange(nt, lambda: nt.poly_mul_rns(o, d_ok, d_bad, N, MODS, 1, None))


def test_small_word_batch_and_server(nt):
    import torch
    N = 1 << 12
    x = _lazy(7, N, SMALL, 1)
    d = torch.from_numpy(x.astype(np.uint32).view(np.int32)).cuda()
    o = torch.empty_like(d)
    nt.ntt_forward_rns32(o, d, N, SMALL, 1, 1, 4)
    x[N + 1] = np.uint64(SMALL[1])
    d = torch.from_numpy(x.astype(np.uint32).view(np.int32)).cuda()
    _erange(nt, lambda: nt.ntt_forward_rns32(o, d, N, SMALL, 1, 1, 4))
    # batch: a forward task whose input holds q
    q = MODS[0]
    good = to_dev(_lazy(8, N, [q], 1))
    badv = _lazy(8, N, [q], 1)
    badv[0] = np.uint64(q)
    bad_d = to_dev(badv)
    out1, out2 = empty_dev(N), empty_dev(N)
    b = nt.Batch(4)
    b.run([(nt.BATCH_FWD, out1, good, None, None, N, q)])
    with pytest.raises(nt.NttError) as e:
        b.run([(nt.BATCH_FWD, out1, good, None, None, N, q), (nt.BATCH_FWD, out2, bad_d, None, None, N, q)])
    assert e.value.status == nt.NTT_ERANGE
    b.close()
    # server: a request whose operand holds q is rejected at submission
    srv = nt.Server(hbm_budget=1 << 24)
    st, t = srv.submit_status(bad_d, good, N, [q])
    assert st == nt.NTT_ERANGE and t == 0
    t = srv.submit(good, good, N, [q])
    srv.wait(t, timeout_s=30)
    srv.release(t)
    srv.close()
