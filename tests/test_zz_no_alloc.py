"""GPU test of poly_mul_rns_noalloc, the entry point that allocates nothing: called through
the C ABI, its results must equal poly_mul_rns's (given a caller workspace) word for word,
on two calls in a row, the second with a smaller input, and at the on-chip size; sizes
beyond its static workspace and uncached plans are refused before any launch."""
import ctypes
import json
import os

import numpy as np
import pytest

from synthetic import uniform_mod, unit_seed
from gpu_util import empty_dev, from_dev, have_gpu, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a ROCm GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POOL = json.load(open(os.path.join(ROOT, "tests", "golden", "primes.json")))["serving"]["moduli"]


def _inputs(tag, N, moduli, B):
    L = len(moduli)
    out = np.empty(B * L * N, dtype=np.uint64)
    for p in range(B):
        for l, q in enumerate(moduli):
            out[(p * L + l) * N:(p * L + l + 1) * N] = uniform_mod(unit_seed(tag, p, l, q), N, q)
    return out


def _addr(t):
    return t if isinstance(t, int) else t.data_ptr()


def _call_noalloc(nt, res, a, b, N, moduli, B):
    """Straight through the C ABI (ctypes), no binding helpers in between."""
    import torch
    mods = (ctypes.c_uint64 * len(moduli))(*moduli)
    return nt._lib.poly_mul_rns_noalloc(ctypes.c_void_p(_addr(res)), ctypes.c_void_p(_addr(a)),
                                        ctypes.c_void_p(_addr(b)), ctypes.c_uint64(N), mods,
                                        ctypes.c_uint64(len(moduli)), ctypes.c_uint64(B),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("cases", [[(16, 4, 2), (15, 2, 1)], [(17, 3, 1), (14, 5, 2)]],
                         ids=["2^16x4x2_then_2^15x2x1", "2^17x3x1_then_2^14x5x2"])
def test_noalloc_matches_poly_mul_rns(cases):
    import paper_2103_16400_amd as nt
    for k, (logN, L, B) in enumerate(cases):
        N = 1 << logN
        moduli = POOL[k:k + L]
        a = _inputs(700 + k, N, moduli, B)
        b = _inputs(710 + k, N, moduli, B)
        da, db = to_dev(a), to_dev(b)
        ref = empty_dev(a.size)
        nt.poly_mul_rns(ref, da, db, N, moduli, B, empty_dev(a.size))    # also creates the plans
        got = empty_dev(a.size)
        got.fill_(-1)
        assert _call_noalloc(nt, got, da, db, N, moduli, B) == 0
        assert np.array_equal(from_dev(got), from_dev(ref)), (logN, L, B)
        # in place (result == a), as poly_mul_rns allows
        assert _call_noalloc(nt, da, da, db, N, moduli, B) == 0
        assert np.array_equal(from_dev(da), from_dev(ref)), (logN, L, B, "in place")


def test_noalloc_refusals():
    """Both refusals happen on the host before any launch: the pointers are distinct
    addresses that are never dereferenced."""
    import oracle
    import paper_2103_16400_amd as nt
    far = [(k + 1) << 44 for k in range(3)]
    moduli = POOL[:33]                                   # 33 limbs x 2^17 words > the 32 MiB workspace
    assert _call_noalloc(nt, far[0], far[1], far[2], 1 << 17, moduli, 1) == nt.NTT_EINVAL_COUNT
    q_new = oracle.find_primes(45, 2 << 15, 40)[37]      # a modulus no other test plans
    assert _call_noalloc(nt, far[0], far[1], far[2], 1 << 15, [q_new], 1) == nt.NTT_ENOTFOUND
