"""Python access to the CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The library path never imports it.

All array arguments are numpy uint64 arrays; results are new numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None
_U64P = ctypes.POINTER(ctypes.c_uint64)
_U64 = ctypes.c_uint64


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.OUT
        if not os.path.exists(path):
            build_oracle.build()
        L = ctypes.CDLL(path)
        for name, res, args in [
            ("or_mulmod", _U64, [_U64, _U64, _U64]),
            ("or_addmod", _U64, [_U64, _U64, _U64]),
            ("or_powmod", _U64, [_U64, _U64, _U64]),
            ("or_invmod", _U64, [_U64, _U64]),
            ("or_is_prime", ctypes.c_int, [_U64]),
            ("or_brv", _U64, [_U64, ctypes.c_int]),
            ("or_min_root", _U64, [_U64, _U64]),
            ("or_find_primes", _U64, [ctypes.c_int, _U64, _U64, _U64P]),
            ("or_find_primes_up", _U64, [ctypes.c_int, _U64, _U64, _U64P]),
            ("or_eltwise_add", None, [_U64P, _U64P, _U64P, _U64, _U64]),
            ("or_eltwise_mult", None, [_U64P, _U64P, _U64P, _U64, _U64]),
            ("or_eltwise_fma", None, [_U64P, _U64P, _U64, ctypes.c_void_p, _U64, _U64]),
            ("or_eltwise_sub", None, [_U64P, _U64P, _U64P, _U64, _U64]),
            ("or_eltwise_negate", None, [_U64P, _U64P, _U64, _U64]),
            ("or_ntt_forward", None, [_U64P, _U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_ntt_inverse", None, [_U64P, _U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_ntt_forward_at", None, [_U64P, _U64P, _U64P, _U64, _U64, _U64, _U64, ctypes.c_int]),
            ("or_ntt_inverse_at", None, [_U64P, _U64P, _U64P, _U64, _U64, _U64, _U64, ctypes.c_int]),
            ("or_negacyclic_mul", None, [_U64P, _U64P, _U64P, _U64, _U64, ctypes.c_int]),
            ("or_negacyclic_mul_at", None, [_U64P, _U64P, _U64P, _U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_harvey_forward", None, [_U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_harvey_inverse", None, [_U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_harvey_forward_w", None, [_U64P, _U64, _U64, _U64, ctypes.c_int, ctypes.c_int]),
            ("or_harvey_inverse_w", None, [_U64P, _U64, _U64, _U64, ctypes.c_int, ctypes.c_int]),
            ("or_harvey_fwd_bfly_w", None, [_U64P, _U64P, _U64, _U64, _U64, ctypes.c_int]),
            ("or_harvey_forward_batch", None, [_U64P, _U64, _U64, _U64, _U64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int]),
            ("or_harvey_inverse_batch", None, [_U64P, _U64, _U64, _U64, _U64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int]),
            ("or_product_batch", None, [_U64P, _U64P, _U64P, _U64, _U64, _U64, _U64, ctypes.c_int]),
        ]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _threads(n):
    return int(n) if n else max(1, min(16, os.cpu_count() or 1))


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_U64P)


def mulmod(a, b, q): return int(lib().or_mulmod(a, b, q))
def addmod(a, b, q): return int(lib().or_addmod(a, b, q))
def powmod(a, e, q): return int(lib().or_powmod(a, e, q))
def invmod(a, q): return int(lib().or_invmod(a, q))
def is_prime(n): return bool(lib().or_is_prime(n))
def brv(i, logn): return int(lib().or_brv(i, logn))
def min_root(N, q): return int(lib().or_min_root(N, q))


def find_primes(bits: int, m: int, count: int) -> list:
    """The `count` largest primes below 2^bits that are 1 mod m, descending."""
    out = np.zeros(count, dtype=np.uint64)
    k = lib().or_find_primes(bits, m, count, _p(out))
    return [int(x) for x in out[:k]]


def find_primes_up(bits: int, m: int, count: int) -> list:
    """The `count` smallest primes of exactly `bits` bits that are 1 mod m, ascending."""
    out = np.zeros(count, dtype=np.uint64)
    k = lib().or_find_primes_up(bits, m, count, _p(out))
    return [int(x) for x in out[:k]]


def eltwise_add(a, b, q):
    a, b = _arr(a), _arr(b)
    c = np.empty_like(a)
    lib().or_eltwise_add(_p(c), _p(a), _p(b), a.size, q)
    return c


def eltwise_mult(a, b, q):
    a, b = _arr(a), _arr(b)
    c = np.empty_like(a)
    lib().or_eltwise_mult(_p(c), _p(a), _p(b), a.size, q)
    return c


def eltwise_fma(a, y, z, q):
    """(a_i * y + z_i) mod q; z may be None (no addition)."""
    a = _arr(a)
    c = np.empty_like(a)
    zp = None
    if z is not None:
        z = _arr(z)
        zp = z.ctypes.data
    lib().or_eltwise_fma(_p(c), _p(a), y, zp, a.size, q)
    return c


def eltwise_sub(a, b, q):
    a, b = _arr(a), _arr(b)
    c = np.empty_like(a)
    lib().or_eltwise_sub(_p(c), _p(a), _p(b), a.size, q)
    return c


def eltwise_negate(a, q):
    a = _arr(a)
    c = np.empty_like(a)
    lib().or_eltwise_negate(_p(c), _p(a), a.size, q)
    return c


def ntt_forward(a, q, psi, threads=None):
    a = _arr(a)
    out = np.empty_like(a)
    lib().or_ntt_forward(_p(out), _p(a), a.size, q, psi, _threads(threads))
    return out


def ntt_inverse(a, q, psi, threads=None):
    a = _arr(a)
    out = np.empty_like(a)
    lib().or_ntt_inverse(_p(out), _p(a), a.size, q, psi, _threads(threads))
    return out


def ntt_forward_at(a, idx, q, psi, threads=None):
    a, idx = _arr(a), _arr(idx)
    out = np.empty(idx.size, dtype=np.uint64)
    lib().or_ntt_forward_at(_p(out), _p(a), _p(idx), idx.size, a.size, q, psi, _threads(threads))
    return out


def ntt_inverse_at(a, idx, q, psi, threads=None):
    a, idx = _arr(a), _arr(idx)
    out = np.empty(idx.size, dtype=np.uint64)
    lib().or_ntt_inverse_at(_p(out), _p(a), _p(idx), idx.size, a.size, q, psi, _threads(threads))
    return out


def negacyclic_mul(a, b, q, threads=None):
    a, b = _arr(a), _arr(b)
    c = np.empty_like(a)
    lib().or_negacyclic_mul(_p(c), _p(a), _p(b), a.size, q, _threads(threads))
    return c


def negacyclic_mul_at(a, b, idx, q, threads=None):
    a, b, idx = _arr(a), _arr(b), _arr(idx)
    c = np.empty(idx.size, dtype=np.uint64)
    lib().or_negacyclic_mul_at(_p(c), _p(a), _p(b), _p(idx), idx.size, a.size, q, _threads(threads))
    return c


def harvey_forward(a, q, psi, out_f=4):
    a = _arr(a).copy()
    lib().or_harvey_forward(_p(a), a.size, q, psi, out_f)
    return a


def harvey_inverse(a, q, psi, out_f=2):
    a = _arr(a).copy()
    lib().or_harvey_inverse(_p(a), a.size, q, psi, out_f)
    return a


def _check_word(q, bits):
    if bits not in (32, 64) or (bits == 32 and 4 * q >= (1 << 32)):
        raise ValueError("word size 2^32 needs 4q < 2^32; bits must be 32 or 64")


def harvey_forward_w(a, q, psi, out_f=4, bits=64):
    """Algorithm 2 with Algorithm 4 butterflies at word size 2^bits (64, or 32 for q < 2^30)."""
    _check_word(q, bits)
    a = _arr(a).copy()
    lib().or_harvey_forward_w(_p(a), a.size, q, psi, out_f, bits)
    return a


def harvey_inverse_w(a, q, psi, out_f=2, bits=64):
    """Algorithm 3 with Algorithm 5 butterflies at word size 2^bits, then N^{-1}."""
    _check_word(q, bits)
    a = _arr(a).copy()
    lib().or_harvey_inverse_w(_p(a), a.size, q, psi, out_f, bits)
    return a


def harvey_fwd_bfly_w(x0, x1, w, q, bits=64):
    """One Algorithm 4 butterfly per element pair at word size 2^bits; returns (X0', X1')."""
    _check_word(q, bits)
    x0, x1 = _arr(x0).copy(), _arr(x1).copy()
    lib().or_harvey_fwd_bfly_w(_p(x0), _p(x1), x0.size, w, q, bits)
    return x0, x1


def harvey_forward_batch(a, N, q, psi, out_f=4, bits=64, threads=None):
    """Forward Harvey model of every length-N limb of `a` (all of modulus q), in a new array."""
    _check_word(q, bits)
    a = _arr(a).copy()
    assert a.size % N == 0
    lib().or_harvey_forward_batch(_p(a), a.size // N, N, q, psi, out_f, bits, _threads(threads))
    return a


def harvey_inverse_batch(a, N, q, psi, out_f=2, bits=64, threads=None):
    """Inverse Harvey model (then N^{-1}) of every length-N limb of `a` (all of modulus q)."""
    _check_word(q, bits)
    a = _arr(a).copy()
    assert a.size % N == 0
    lib().or_harvey_inverse_batch(_p(a), a.size // N, N, q, psi, out_f, bits, _threads(threads))
    return a


def product_batch(a, b, N, q, psi=None, threads=None):
    """Negacyclic product of every length-N limb pair of a and b (all of modulus q), canonical,
    through the transforms (O(N log N) per limb); the result does not depend on psi."""
    a, b = _arr(a), _arr(b)
    assert a.size == b.size and a.size % N == 0
    if psi is None:
        psi = min_root(N, q)
    c = np.empty_like(a)
    lib().or_product_batch(_p(c), _p(a), _p(b), a.size // N, N, q, psi, _threads(threads))
    return c


def _limb_rows(x, N, L):
    """View of a [B][L][N] array as (B, L, N)."""
    return _arr(x).reshape(-1, L, N)


def product_rns(a, b, N, moduli, threads=None):
    """c = a * b per RNS limb for [B][L][N] operands (limb l of every polynomial mod moduli[l])."""
    L = len(moduli)
    A, Bv = _limb_rows(a, N, L), _limb_rows(b, N, L)
    C = np.empty_like(A)
    for l, q in enumerate(moduli):
        C[:, l, :] = product_batch(np.ascontiguousarray(A[:, l, :]), np.ascontiguousarray(Bv[:, l, :]), N, int(q),
                                   threads=threads).reshape(-1, N)
    return C.reshape(-1)


def forward_rns(a, N, moduli, out_f=1, threads=None):
    """Forward transform (Harvey model, smallest root) of every limb of a [B][L][N] array; with
    out_f = 1 the canonical values, which equal the direct definition."""
    L = len(moduli)
    A = _limb_rows(a, N, L)
    C = np.empty_like(A)
    for l, q in enumerate(moduli):
        C[:, l, :] = harvey_forward_batch(np.ascontiguousarray(A[:, l, :]), N, int(q), min_root(N, int(q)), out_f,
                                          threads=threads).reshape(-1, N)
    return C.reshape(-1)


def inverse_rns(a, N, moduli, out_f=1, threads=None):
    """Inverse transform (Harvey model, smallest root) of every limb of a [B][L][N] array (inputs
    below 2q); with out_f = 1 the canonical values, which equal the direct definition."""
    L = len(moduli)
    A = _limb_rows(a, N, L)
    C = np.empty_like(A)
    for l, q in enumerate(moduli):
        C[:, l, :] = harvey_inverse_batch(np.ascontiguousarray(A[:, l, :]), N, int(q), min_root(N, int(q)), out_f,
                                          threads=threads).reshape(-1, N)
    return C.reshape(-1)


def add_rns(a, b, N, moduli):
    """(a + b) mod q_l per limb of [B][L][N] arrays (inputs interpreted mod q_l)."""
    L = len(moduli)
    A, Bv = _limb_rows(a, N, L), _limb_rows(b, N, L)
    C = np.empty_like(A)
    for l, q in enumerate(moduli):
        C[:, l, :] = eltwise_add(np.ascontiguousarray(A[:, l, :]).reshape(-1), np.ascontiguousarray(Bv[:, l, :]).reshape(-1),
                                 int(q)).reshape(-1, N)
    return C.reshape(-1)
