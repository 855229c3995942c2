"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntt_hip.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def nt():
    import paper_2103_16400_amd as nt
    return nt


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["ntt_forward", "ntt_inverse", "eltwise_mult_mod", "eltwise_add_mod", "ntt_plan_create",
                     "ntt_forward_rns", "poly_mul_rns", "ntt_batch_run", "ntt_server_create", "ntt_server_submit",
                     "ntt_server_poll", "ntt_server_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol(nt):
    lib = ctypes.CDLL(nt.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(nt):
    for code in range(0, -13, -1):
        s = nt.status_string(code)
        assert s and s != "unknown status"
    assert nt.status_string(-999) == "unknown status"


def _raw(nt):
    return nt.lib()


def test_argument_validation_without_device(nt):
    L = _raw(nt)
    q = 1125899906826241          # 1 mod 2048, prime
    fake = ctypes.c_void_p(0x1000000)
    other = ctypes.c_void_p(0x40000000)
    # null pointers
    assert L.ntt_forward(None, fake, 1024, q, 1, 1, None) == nt.NTT_EINVAL_POINTER
    assert L.eltwise_add_mod(fake, None, fake, 4, 17, None) == nt.NTT_EINVAL_POINTER
    # bad factors (checked before anything else)
    assert L.ntt_forward(fake, other, 1024, q, 3, 1, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_forward(fake, other, 1024, q, 1, 2, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_inverse(fake, other, 1024, q, 4, 1, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_inverse(fake, other, 1024, q, 1, 4, None) == nt.NTT_EINVAL_FACTOR
    assert L.eltwise_mult_mod(fake, other, other, 4, 17, 3, None) == nt.NTT_EINVAL_FACTOR
    # bad degrees
    for N in [0, 1, 3, 1000, 1 << 18]:
        assert L.ntt_forward(fake, other, N, q, 1, 1, None) == nt.NTT_EINVAL_DEGREE
    # bad moduli: not 1 mod 2N, too large, even
    assert L.ntt_forward(fake, other, 1 << 14, q, 1, 1, None) == nt.NTT_EINVAL_MODULUS   # q != 1 mod 2^15
    assert L.ntt_forward(fake, other, 1024, (1 << 62) + 2049, 1, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_mult_mod(fake, other, other, 4, 1 << 62, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_mult_mod(fake, other, other, 4, (1 << 61) + 1, 4, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_add_mod(fake, other, other, 4, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_add_mod(fake, other, other, 4, 1 << 63, None) == nt.NTT_EINVAL_MODULUS
    # fused multiply-add, subtraction, negation
    assert L.eltwise_fma_mod(fake, None, 3, None, 4, 17, 1, None) == nt.NTT_EINVAL_POINTER
    assert L.eltwise_fma_mod(fake, other, 3, None, 4, 17, 3, None) == nt.NTT_EINVAL_FACTOR
    assert L.eltwise_fma_mod(fake, other, 3, None, 4, 1 << 61, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_fma_mod(fake, other, 3, None, 4, 1, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_fma_mod(fake, other, 3, None, 0, 17, 1, None) == nt.NTT_EINVAL_COUNT
    assert L.eltwise_fma_mod(ctypes.c_void_p(0x1000000 + 8), fake, 3, None, 1024, 17, 1, None) == nt.NTT_EALIAS
    assert L.eltwise_fma_mod(ctypes.c_void_p(0x1000000 + 8), other, 3, fake, 1024, 17, 1, None) == nt.NTT_EALIAS
    assert L.eltwise_sub_mod(fake, other, None, 4, 17, None) == nt.NTT_EINVAL_POINTER
    assert L.eltwise_sub_mod(fake, other, other, 4, 1 << 63, None) == nt.NTT_EINVAL_MODULUS
    assert L.eltwise_negate_mod(None, other, 4, 17, None) == nt.NTT_EINVAL_POINTER
    assert L.eltwise_negate_mod(ctypes.c_void_p(0x1000000 + 8), fake, 1024, 17, None) == nt.NTT_EALIAS
    # partial overlap of output and input
    shifted = ctypes.c_void_p(0x1000000 + 8)
    assert L.ntt_forward(shifted, fake, 1024, q, 1, 1, None) == nt.NTT_EALIAS
    assert L.eltwise_add_mod(shifted, fake, other, 1024, 17, None) == nt.NTT_EALIAS
    # counts
    assert L.eltwise_add_mod(fake, other, other, 0, 17, None) == nt.NTT_EINVAL_COUNT
    mod = (ctypes.c_uint64 * 1)(q)
    assert L.ntt_forward_rns(fake, other, 1024, mod, 0, 1, 1, 1, None) == nt.NTT_EINVAL_COUNT
    assert L.ntt_forward_rns(fake, other, 1024, mod, 65, 1, 1, 1, None) == nt.NTT_EINVAL_COUNT
    assert L.poly_mul_rns(fake, other, fake, 1024, mod, 1, 1, None, None) == nt.NTT_EALIAS
    assert L.ntt_plan_destroy(None) == nt.NTT_EINVAL_POINTER
    assert L.ntt_plan_root(None) == 0


def test_server_config_validation_without_device(nt):
    """Invalid server configurations are refused before any device call."""
    lib = _raw(nt)
    h = ctypes.c_void_p()
    assert lib.ntt_server_create(None, None) == -5
    for kw in ({"mode": 3}, {"streams": 5}, {"max_batch_tasks": 10}, {"max_batch_tasks": (1 << 20) + 1},
               {"wide_min_log_degree": 9}, {"wide_min_log_degree": 19}):
        cfg = nt.ServerConfig(**kw)
        assert lib.ntt_server_create(ctypes.byref(h), ctypes.byref(cfg)) == -7, kw
        assert not h.value
    assert lib.ntt_server_submit(None, None, None) == -5
    assert lib.ntt_server_poll(None, 1, None) == -5
    assert lib.ntt_server_drain(None, 0) == -5
    assert lib.ntt_server_release(None, 1) == -5
    assert lib.ntt_server_destroy(None) == -5
    assert lib.ntt_server_now_ns() > 0


def test_small_modulus_validation_without_device(nt):
    """The word-size-2^32 calls reject moduli of 2^30 or more, N above 2^17, bad
    factors, null pointers, empty batches, partial overlaps and a missing product
    workspace at N >= 2^16 before any device work."""
    L = _raw(nt)
    fake = ctypes.c_void_p(0x1000000)
    other = ctypes.c_void_p(0x40000000)
    shifted = ctypes.c_void_p(0x1000000 + 4)
    small = (ctypes.c_uint64 * 1)(1073643521)      # < 2^30, 1 mod 2^15
    big = (ctypes.c_uint64 * 1)(1 << 30)
    q31 = (ctypes.c_uint64 * 1)(1074266113)        # 31-bit NTT prime: 4q does not fit 32 bits
    assert L.ntt_forward_rns32(fake, other, 1024, big, 1, 1, 1, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.ntt_forward_rns32(fake, other, 1024, q31, 1, 1, 1, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.ntt_inverse_rns32(fake, other, 1024, q31, 1, 1, 1, 1, None) == nt.NTT_EINVAL_MODULUS
    assert L.ntt_forward_rns32(fake, other, 1 << 18, small, 1, 1, 1, 1, None) == nt.NTT_EINVAL_DEGREE
    assert L.ntt_forward_rns32(fake, other, 1000, small, 1, 1, 1, 1, None) == nt.NTT_EINVAL_DEGREE
    assert L.ntt_forward_rns32(fake, other, 1024, small, 1, 1, 3, 1, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_forward_rns32(fake, other, 1024, small, 1, 1, 1, 2, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_inverse_rns32(fake, other, 1024, small, 1, 1, 4, 1, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_inverse_rns32(fake, other, 1024, small, 1, 1, 1, 4, None) == nt.NTT_EINVAL_FACTOR
    assert L.ntt_forward_rns32(None, other, 1024, small, 1, 1, 1, 1, None) == nt.NTT_EINVAL_POINTER
    assert L.ntt_forward_rns32(fake, other, 1024, None, 1, 1, 1, 1, None) == nt.NTT_EINVAL_POINTER
    assert L.ntt_forward_rns32(fake, other, 1024, small, 0, 1, 1, 1, None) == nt.NTT_EINVAL_COUNT
    assert L.ntt_forward_rns32(fake, other, 1024, small, 1, 0, 1, 1, None) == nt.NTT_EINVAL_COUNT
    assert L.ntt_forward_rns32(shifted, fake, 1024, small, 1, 1, 1, 1, None) == nt.NTT_EALIAS
    assert L.poly_mul_rns32(fake, other, fake, 1024, small, 1, 1, None, None) == nt.NTT_EALIAS
    assert L.poly_mul_rns32(fake, None, other, 1024, small, 1, 1, None, None) == nt.NTT_EINVAL_POINTER
    assert L.poly_mul_acc_ntt_rns32(fake, fake, other, 1024, small, 1, 1, None, None) == nt.NTT_EALIAS
    assert L.poly_mul_acc_ntt_rns32(fake, other, shifted, 1024, small, 1, 1, None, None) == nt.NTT_EALIAS
    assert L.poly_mul_acc_ntt_rns32(fake, other, other, 1 << 18, small, 1, 1, None, None) == nt.NTT_EINVAL_DEGREE
    assert L.poly_mul_acc_ntt_rns32(fake, other, other, 1024, big, 1, 1, None, None) == nt.NTT_EINVAL_MODULUS
    third = ctypes.c_void_p(0x80000000)
    assert L.poly_mul_rns32(fake, other, third, 1 << 16, small, 1, 1, None, None) == nt.NTT_EINVAL_POINTER
    assert L.poly_mul_acc_ntt_rns32(fake, other, third, 1 << 17, small, 1, 1, None, None) == nt.NTT_EINVAL_POINTER
    assert L.poly_mul_rns32(fake, other, third, 1 << 16, small, 1, 1, ctypes.c_void_p(0x1000000 + 8), None) == nt.NTT_EALIAS


def test_validation_toggle_without_device(nt):
    """Validation mode is off by default, switches on and off, and has its own status."""
    L = _raw(nt)
    was = L.ntt_get_validate()
    try:
        assert L.ntt_set_validate(1) == nt.NTT_OK and L.ntt_get_validate() == 1
        assert L.ntt_set_validate(0) == nt.NTT_OK and L.ntt_get_validate() == 0
    finally:
        L.ntt_set_validate(was)
    assert nt.NTT_ERANGE == -13 and "outside" in nt.status_string(nt.NTT_ERANGE)


def test_wide_range_switch_without_device(nt):
    """The wide-range butterflies are on by default and switch off and on again."""
    L = _raw(nt)
    assert L.ntt_get_wide_range() == 1 and nt.get_wide_range()
    try:
        assert L.ntt_set_wide_range(0) == nt.NTT_OK and L.ntt_get_wide_range() == 0
        assert not nt.get_wide_range()
        nt.set_wide_range(True)
        assert L.ntt_get_wide_range() == 1
    finally:
        L.ntt_set_wide_range(1)
