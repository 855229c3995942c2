"""Python binding of the MI355X negacyclic NTT library (C ABI in include/ntt_hip.h).

Argument marshalling only: every operation runs in the HIP kernels of
libntt_hip.so.  Tensors must be contiguous torch tensors of dtype uint64 (or
int64 holding the same bits) on a ROCm device; they provide device memory, and
torch's current stream (or an explicit one) orders the work.  There is no CPU
fallback: if the library is not built, importing this package raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libntt_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libntt_hip.so is not built (expected at %s); run `python paper_2103_16400_amd/build.py` "
        "or __graft_entry__.build()" % LIB_PATH)

# torch ships its own HIP runtime (same soname as ROCm's); loading it first makes
# this library bind to that one runtime instead of bringing in a second copy.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_U64 = ctypes.c_uint64
_P = ctypes.c_void_p
_ST = ctypes.c_int

_SIGS = {
    "ntt_status_string": (ctypes.c_char_p, [_ST]),
    "ntt_shutdown": (_ST, []),
    "ntt_plan_create": (_ST, [ctypes.POINTER(_P), _U64, _U64, _U64]),
    "ntt_plan_destroy": (_ST, [_P]),
    "ntt_plan_root": (_U64, [_P]),
    "ntt_forward": (_ST, [_P, _P, _U64, _U64, _U64, _U64, _P]),
    "ntt_inverse": (_ST, [_P, _P, _U64, _U64, _U64, _U64, _P]),
    "ntt_forward_plan": (_ST, [_P, _P, _P, _U64, _U64, _P]),
    "ntt_inverse_plan": (_ST, [_P, _P, _P, _U64, _U64, _P]),
    "eltwise_mult_mod": (_ST, [_P, _P, _P, _U64, _U64, _U64, _P]),
    "eltwise_add_mod": (_ST, [_P, _P, _P, _U64, _U64, _P]),
    "ntt_forward_rns": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _U64, _P]),
    "ntt_inverse_rns": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _U64, _P]),
    "eltwise_mult_mod_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _U64, _P]),
    "eltwise_add_mod_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P]),
    "poly_mul_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P, _P]),
    "poly_mul_rns_noalloc": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P]),
    "ntt_forward_mul_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _U64, _P, _P]),
    "ntt_inverse_acc_rns": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _P, _P]),
    "poly_mul_acc_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P, _P]),
    "ntt_batch_create": (_ST, [ctypes.POINTER(_P), ctypes.c_size_t]),
    "ntt_batch_destroy": (_ST, [_P]),
    "ntt_batch_set_grid": (_ST, [_P, ctypes.c_int]),
    "ntt_batch_set_shape": (_ST, [_P, ctypes.c_int]),
    "ntt_batch_get_config": (_ST, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ntt_batch_run": (_ST, [_P, _P, ctypes.c_size_t, _P]),
    "ntt_batch_run_graph": (_ST, [_P, _P, ctypes.c_size_t, _P]),
    "ntt_batch_autotune": (_ST, [_P, _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_int)]),
    "eltwise_fma_mod": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _P]),
    "poly_mul_acc_ntt_rns": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P, _P]),
    "ntt_batch_forward": (_ST, [_P, ctypes.c_size_t, _P]),
    "ntt_batch_inverse": (_ST, [_P, ctypes.c_size_t, _P]),
    "ntt_batch_product": (_ST, [_P, ctypes.c_size_t, _P]),
    "ntt_set_validate": (_ST, [ctypes.c_int]),
    "ntt_get_validate": (ctypes.c_int, []),
    "ntt_set_wide_range": (_ST, [ctypes.c_int]),
    "ntt_get_wide_range": (ctypes.c_int, []),
    "ntt_forward_rns32": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _U64, _P]),
    "ntt_inverse_rns32": (_ST, [_P, _P, _U64, _P, _U64, _U64, _U64, _U64, _P]),
    "poly_mul_rns32": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P, _P]),
    "poly_mul_acc_ntt_rns32": (_ST, [_P, _P, _P, _U64, _P, _U64, _U64, _P, _P]),
    "eltwise_fma_mod_rns": (_ST, [_P, _P, _P, _P, _U64, _P, _U64, _U64, _U64, _P]),
    "eltwise_sub_mod": (_ST, [_P, _P, _P, _U64, _U64, _P]),
    "eltwise_negate_mod": (_ST, [_P, _P, _U64, _U64, _P]),
    "ntt_server_create": (_ST, [ctypes.POINTER(_P), _P]),
    "ntt_server_submit": (_ST, [_P, _P, ctypes.POINTER(_U64)]),
    "ntt_server_poll": (_ST, [_P, _U64, _P]),
    "ntt_server_query": (_ST, [_P, _P, ctypes.c_size_t, _P]),
    "ntt_server_wait": (_ST, [_P, _U64, ctypes.c_int64, _P]),
    "ntt_server_drain": (_ST, [_P, ctypes.c_int64]),
    "ntt_server_read": (_ST, [_P, _U64, _P, _P]),
    "ntt_server_release": (_ST, [_P, _U64]),
    "ntt_server_stats_get": (_ST, [_P, _P]),
    "ntt_server_now_ns": (ctypes.c_int64, []),
    "ntt_server_destroy": (_ST, [_P]),
    "ntt_autotune": (_ST, [_U64, _P, _U64, _U64, _P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "ntt_set_variant": (_ST, [_U64, _U64, ctypes.c_int, ctypes.c_int]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

# status codes (include/ntt_hip.h)
NTT_OK = 0
NTT_EINVAL_DEGREE = -1
NTT_EINVAL_MODULUS = -2
NTT_EINVAL_ROOT = -3
NTT_EINVAL_FACTOR = -4
NTT_EINVAL_POINTER = -5
NTT_EALIAS = -6
NTT_EINVAL_COUNT = -7
NTT_EDEVICE = -8
NTT_ENOMEM = -9
NTT_ENOTFOUND = -10
NTT_EBUSY = -11
NTT_ETIMEDOUT = -12
NTT_ERANGE = -13


class NttError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (what, status_string(status), status))


def set_validate(on: bool):
    """Validation mode: calls check operand ranges on the device and raise NttError
    (status NTT_ERANGE) for out-of-range values.  A debugging aid: it synchronises."""
    _check(_lib.ntt_set_validate(1 if on else 0), "ntt_set_validate")


def get_validate() -> bool:
    return bool(_lib.ntt_get_validate())


def set_wide_range(on: bool):
    """Wide-range butterflies for N <= 2^14 and moduli below 2^58 (on by default);
    off: every kernel produces the lazy words of Algorithms 4 and 5."""
    _check(_lib.ntt_set_wide_range(1 if on else 0), "ntt_set_wide_range")


def get_wide_range() -> bool:
    return bool(_lib.ntt_get_wide_range())


def status_string(status: int) -> str:
    return _lib.ntt_status_string(status).decode()


def lib():
    """The loaded ctypes library (for callers that pass raw pointers)."""
    return _lib


def _check(status: int, what: str):
    if status != NTT_OK:
        raise NttError(status, what)


def _ptr(t, bits=64):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    ok = (torch.uint64, torch.int64) if bits == 64 else (torch.uint32, torch.int32)
    if t.dtype not in ok:
        raise TypeError("expected a uint%d (or int%d) tensor, got %s" % (bits, bits, t.dtype))
    if not t.is_cuda:
        raise ValueError("tensor must be on a ROCm device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _ptr32(t):
    return _ptr(t, 32)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _moduli(moduli):
    arr = (_U64 * len(moduli))(*[int(q) for q in moduli])
    return arr, len(moduli)


class Plan:
    """Device-resident tables for one (N, q, psi) (the paper's NTT object)."""

    def __init__(self, N: int, q: int, root_of_unity: int = 0):
        h = _P()
        _check(_lib.ntt_plan_create(ctypes.byref(h), N, q, root_of_unity), "ntt_plan_create")
        self._h = h
        self.N, self.q = N, q
        self.root = int(_lib.ntt_plan_root(h))

    def close(self):
        if self._h:
            _lib.ntt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, result, operand, input_mod_factor=1, output_mod_factor=1, stream=None):
        _check(_lib.ntt_forward_plan(self._h, _ptr(result), _ptr(operand), input_mod_factor,
                                     output_mod_factor, _stream(stream)), "ntt_forward_plan")

    def inverse(self, result, operand, input_mod_factor=1, output_mod_factor=1, stream=None):
        _check(_lib.ntt_inverse_plan(self._h, _ptr(result), _ptr(operand), input_mod_factor,
                                     output_mod_factor, _stream(stream)), "ntt_inverse_plan")


def ntt_forward(result, operand, N, q, input_mod_factor=1, output_mod_factor=1, stream=None):
    _check(_lib.ntt_forward(_ptr(result), _ptr(operand), N, q, input_mod_factor, output_mod_factor,
                            _stream(stream)), "ntt_forward")


def ntt_inverse(result, operand, N, q, input_mod_factor=1, output_mod_factor=1, stream=None):
    _check(_lib.ntt_inverse(_ptr(result), _ptr(operand), N, q, input_mod_factor, output_mod_factor,
                            _stream(stream)), "ntt_inverse")


def eltwise_mult_mod(result, operand1, operand2, n, modulus, input_mod_factor=1, stream=None):
    _check(_lib.eltwise_mult_mod(_ptr(result), _ptr(operand1), _ptr(operand2), n, modulus, input_mod_factor,
                                 _stream(stream)), "eltwise_mult_mod")


def eltwise_add_mod(result, operand1, operand2, n, modulus, stream=None):
    _check(_lib.eltwise_add_mod(_ptr(result), _ptr(operand1), _ptr(operand2), n, modulus, _stream(stream)),
           "eltwise_add_mod")


def ntt_forward_rns(result, operand, N, moduli, num_polys, input_mod_factor=1, output_mod_factor=1, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.ntt_forward_rns(_ptr(result), _ptr(operand), N, m, L, num_polys, input_mod_factor,
                                output_mod_factor, _stream(stream)), "ntt_forward_rns")


def ntt_inverse_rns(result, operand, N, moduli, num_polys, input_mod_factor=1, output_mod_factor=1, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.ntt_inverse_rns(_ptr(result), _ptr(operand), N, m, L, num_polys, input_mod_factor,
                                output_mod_factor, _stream(stream)), "ntt_inverse_rns")


def eltwise_mult_mod_rns(result, operand1, operand2, N, moduli, num_polys, input_mod_factor=1, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.eltwise_mult_mod_rns(_ptr(result), _ptr(operand1), _ptr(operand2), N, m, L, num_polys,
                                     input_mod_factor, _stream(stream)), "eltwise_mult_mod_rns")


def eltwise_add_mod_rns(result, operand1, operand2, N, moduli, num_polys, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.eltwise_add_mod_rns(_ptr(result), _ptr(operand1), _ptr(operand2), N, m, L, num_polys,
                                    _stream(stream)), "eltwise_add_mod_rns")


def poly_mul_rns(result, a, b, N, moduli, num_polys, workspace=None, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_rns(_ptr(result), _ptr(a), _ptr(b), N, m, L, num_polys, _ptr(workspace),
                             _stream(stream)), "poly_mul_rns")


def poly_mul_rns_noalloc(result, a, b, N, moduli, num_polys, stream=None):
    """poly_mul_rns with the library's static workspace and cached plans only (allocates nothing)."""
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_rns_noalloc(_ptr(result), _ptr(a), _ptr(b), N, m, L, num_polys, _stream(stream)),
           "poly_mul_rns_noalloc")


def ntt_forward_mul_rns(result, operand, multiplier, N, moduli, num_polys, input_mod_factor=1, workspace=None,
                        stream=None):
    m, L = _moduli(moduli)
    _check(_lib.ntt_forward_mul_rns(_ptr(result), _ptr(operand), _ptr(multiplier), N, m, L, num_polys,
                                    input_mod_factor, _ptr(workspace), _stream(stream)), "ntt_forward_mul_rns")


def ntt_inverse_acc_rns(acc, operand, N, moduli, num_polys, input_mod_factor=1, workspace=None, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.ntt_inverse_acc_rns(_ptr(acc), _ptr(operand), N, m, L, num_polys, input_mod_factor,
                                    _ptr(workspace), _stream(stream)), "ntt_inverse_acc_rns")


def poly_mul_acc_rns(acc, a, b, N, moduli, num_polys, workspace, stream=None):
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_acc_rns(_ptr(acc), _ptr(a), _ptr(b), N, m, L, num_polys, _ptr(workspace),
                                 _stream(stream)), "poly_mul_acc_rns")


def autotune(N, moduli, num_polys, stream=None):
    """Times the kernel variants for this shape and keeps the fastest; returns (fwd, inv) choices."""
    m, L = _moduli(moduli)
    f, i = ctypes.c_int(0), ctypes.c_int(0)
    _check(_lib.ntt_autotune(N, m, L, num_polys, _stream(stream), ctypes.byref(f), ctypes.byref(i)), "ntt_autotune")
    return f.value, i.value


def set_variant(N, num_items, forward, variant):
    _check(_lib.ntt_set_variant(N, num_items, 1 if forward else 0, variant), "ntt_set_variant")


class BatchItem(ctypes.Structure):
    """ntt_batch_item of include/ntt_hip.h."""
    _fields_ = [("out", _P), ("in_", _P), ("in2", _P), ("tmp", _P), ("N", _U64), ("q", _U64),
                ("op", ctypes.c_uint32), ("input_mod_factor", ctypes.c_uint16),
                ("output_mod_factor", ctypes.c_uint16)]


BATCH_FWD_LAZY, BATCH_FWD, BATCH_INV_LAZY, BATCH_INV, BATCH_PRODUCT = 0, 1, 2, 3, 4


class Batch:
    """A reusable batch context: runs lists of limb tasks of mixed N in one persistent launch."""

    def __init__(self, capacity: int):
        h = _P()
        _check(_lib.ntt_batch_create(ctypes.byref(h), capacity), "ntt_batch_create")
        self._h = h
        self.capacity = capacity

    def close(self):
        if self._h:
            _lib.ntt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_grid(self, workgroups: int):
        _check(_lib.ntt_batch_set_grid(self._h, workgroups), "ntt_batch_set_grid")

    def set_shape(self, shape: int):
        """0: the per-call kernels' shapes; 1: twice the threads per limb or tile; 2: per tile only."""
        _check(_lib.ntt_batch_set_shape(self._h, shape), "ntt_batch_set_shape")

    def config(self):
        """(workgroups, shape) of the context (workgroups 0 = automatic)."""
        g, sh = ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib.ntt_batch_get_config(self._h, ctypes.byref(g), ctypes.byref(sh)), "ntt_batch_get_config")
        return g.value, sh.value

    @staticmethod
    def make_items(tasks):
        """tasks: iterable of (op, out, in, in2, tmp, N, q[, input_mod_factor, output_mod_factor]) with
        torch tensors (or None); the factors default to 0 (the op's own)."""
        tasks = list(tasks)
        arr = (BatchItem * max(1, len(tasks)))()
        for k, task in enumerate(tasks):
            op, out, inp, in2, tmp, N, q = task[:7]
            if len(task) > 7:
                arr[k].input_mod_factor = task[7]
                arr[k].output_mod_factor = task[8] if len(task) > 8 else 0
            arr[k].out = _ptr(out)
            arr[k].in_ = _ptr(inp)
            arr[k].in2 = _ptr(in2)
            arr[k].tmp = _ptr(tmp)
            arr[k].N = N
            arr[k].q = q
            arr[k].op = op
        return arr, len(tasks)

    def autotune(self, items, count=None, stream=None):
        if not isinstance(items, ctypes.Array):
            items, count = self.make_items(items)
        g = ctypes.c_int(0)
        _check(_lib.ntt_batch_autotune(self._h, items, count, _stream(stream), ctypes.byref(g)), "ntt_batch_autotune")
        return g.value

    def run(self, items, count=None, stream=None, graph=False):
        if not isinstance(items, ctypes.Array):
            items, count = self.make_items(items)
        fn = _lib.ntt_batch_run_graph if graph else _lib.ntt_batch_run
        _check(fn(self._h, items, count, _stream(stream)), "ntt_batch_run_graph" if graph else "ntt_batch_run")


def _oneshot(name, tasks, stream):
    items, count = Batch.make_items(tasks)
    _check(getattr(_lib, name)(ctypes.cast(items, _P), count, _stream(stream)), name)


def batch_forward(tasks, stream=None):
    """One-shot batch of forward tasks (op, out, in, in2, tmp, N, q), op BATCH_FWD_LAZY or BATCH_FWD."""
    _oneshot("ntt_batch_forward", tasks, stream)


def batch_inverse(tasks, stream=None):
    """One-shot batch of inverse tasks, op BATCH_INV_LAZY or BATCH_INV."""
    _oneshot("ntt_batch_inverse", tasks, stream)


def batch_product(tasks, stream=None):
    """One-shot batch of product tasks, op BATCH_PRODUCT."""
    _oneshot("ntt_batch_product", tasks, stream)


def poly_mul_acc_ntt_rns(acc, a_ntt, b, N, moduli, num_polys, workspace=None, stream=None):
    """acc += a * b with a given as its forward NTT (lazy outputs allowed)."""
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_acc_ntt_rns(_ptr(acc), _ptr(a_ntt), _ptr(b), N, m, L, num_polys, _ptr(workspace),
                                     _stream(stream)), "poly_mul_acc_ntt_rns")


def ntt_forward_rns32(result, operand, N, moduli, num_polys, input_mod_factor=1, output_mod_factor=1, stream=None):
    """Forward NTT at word size 2^32 (moduli below 2^30, N <= 2^15); uint32 coefficients."""
    m, L = _moduli(moduli)
    _check(_lib.ntt_forward_rns32(_ptr32(result), _ptr32(operand), N, m, L, num_polys, input_mod_factor,
                                  output_mod_factor, _stream(stream)), "ntt_forward_rns32")


def ntt_inverse_rns32(result, operand, N, moduli, num_polys, input_mod_factor=1, output_mod_factor=1, stream=None):
    """Inverse NTT at word size 2^32 (moduli below 2^30, N <= 2^15); uint32 coefficients."""
    m, L = _moduli(moduli)
    _check(_lib.ntt_inverse_rns32(_ptr32(result), _ptr32(operand), N, m, L, num_polys, input_mod_factor,
                                  output_mod_factor, _stream(stream)), "ntt_inverse_rns32")


def poly_mul_rns32(result, a, b, N, moduli, num_polys, workspace=None, stream=None):
    """result = a * b mod (X^N + 1, q_l) per limb at word size 2^32 (workspace needed at N >= 2^16)."""
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_rns32(_ptr32(result), _ptr32(a), _ptr32(b), N, m, L, num_polys, _ptr32(workspace),
                               _stream(stream)), "poly_mul_rns32")


def poly_mul_acc_ntt_rns32(acc, a_ntt, b, N, moduli, num_polys, workspace=None, stream=None):
    """acc += a * b at word size 2^32, with a given as its forward NTT (lazy outputs allowed)."""
    m, L = _moduli(moduli)
    _check(_lib.poly_mul_acc_ntt_rns32(_ptr32(acc), _ptr32(a_ntt), _ptr32(b), N, m, L, num_polys, _ptr32(workspace),
                                       _stream(stream)), "poly_mul_acc_ntt_rns32")


def eltwise_fma_mod(result, arg1, arg2, arg3, n, modulus, input_mod_factor=1, stream=None):
    """result = (arg1 * arg2 + arg3) mod q (arg3 may be None); Algorithm 10."""
    _check(_lib.eltwise_fma_mod(_ptr(result), _ptr(arg1), int(arg2), _ptr(arg3), n, modulus, input_mod_factor,
                                _stream(stream)), "eltwise_fma_mod")


def eltwise_fma_mod_rns(result, arg1, scalars, arg3, N, moduli, num_polys, input_mod_factor=1, stream=None):
    m, L = _moduli(moduli)
    y, Ly = _moduli(scalars)
    if Ly != L:
        raise ValueError("one scalar per limb expected")
    _check(_lib.eltwise_fma_mod_rns(_ptr(result), _ptr(arg1), y, _ptr(arg3), N, m, L, num_polys, input_mod_factor,
                                    _stream(stream)), "eltwise_fma_mod_rns")


def eltwise_sub_mod(result, operand1, operand2, n, modulus, stream=None):
    _check(_lib.eltwise_sub_mod(_ptr(result), _ptr(operand1), _ptr(operand2), n, modulus, _stream(stream)),
           "eltwise_sub_mod")


def eltwise_negate_mod(result, operand, n, modulus, stream=None):
    _check(_lib.eltwise_negate_mod(_ptr(result), _ptr(operand), n, modulus, _stream(stream)), "eltwise_negate_mod")


class ServerConfig(ctypes.Structure):
    """ntt_server_config of include/ntt_hip.h."""
    _fields_ = [("hbm_budget", _U64), ("mode", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("max_batch_tasks", ctypes.c_uint32), ("max_queue", ctypes.c_uint32),
                ("release_on_completion", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("wide_min_log_degree", ctypes.c_uint32), ("wide_max_inflight", ctypes.c_uint32)]


class Request(ctypes.Structure):
    """ntt_request of include/ntt_hip.h."""
    _fields_ = [("N", _U64), ("num_limbs", _U64), ("moduli", ctypes.POINTER(_U64)), ("a", _P), ("b", _P),
                ("arrival_ns", ctypes.c_int64)]


class RequestInfo(ctypes.Structure):
    """ntt_request_info of include/ntt_hip.h."""
    _fields_ = [("state", ctypes.c_uint32), ("status", ctypes.c_int), ("result", _P), ("arrival_ns", ctypes.c_int64),
                ("admit_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    """ntt_server_stats of include/ntt_hip.h."""
    _fields_ = [(n, _U64) for n in ("submitted", "rejected", "completed", "failed", "launches", "tasks", "waiting",
                                    "in_flight", "arena_bytes", "arena_in_use", "arena_peak", "deferred")]


SERVE_BATCHED, SERVE_FIFO, SERVE_FIFO_PER_LIMB = 0, 1, 2
REQ_WAITING, REQ_ADMITTED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3, 4


def now_ns() -> int:
    """The serving clock (monotonic, nanoseconds)."""
    return _lib.ntt_server_now_ns()


class Server:
    """Continuous-batching server for negacyclic products (ntt_server_* of include/ntt_hip.h)."""

    def __init__(self, hbm_budget=0, mode=SERVE_BATCHED, streams=0, max_batch_tasks=0, max_queue=0,
                 release_on_completion=False, use_graph=False, wide_min_log_degree=0, wide_max_inflight=0):
        cfg = ServerConfig(hbm_budget, mode, streams, max_batch_tasks, max_queue, int(bool(release_on_completion)),
                           int(bool(use_graph)), wide_min_log_degree, wide_max_inflight)
        h = _P()
        _check(_lib.ntt_server_create(ctypes.byref(h), ctypes.byref(cfg)), "ntt_server_create")
        self._h = h

    def close(self):
        if self._h:
            _lib.ntt_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_status(self, a, b, N, moduli, arrival_ns=0):
        """Returns (status, ticket) without raising."""
        mods = (_U64 * max(1, len(moduli)))(*[int(q) for q in moduli])
        req = Request(N, len(moduli), mods, _ptr(a), _ptr(b), arrival_ns)
        t = _U64(0)
        st = _lib.ntt_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        return st, t.value

    def submit(self, a, b, N, moduli, arrival_ns=0) -> int:
        st, t = self.submit_status(a, b, N, moduli, arrival_ns)
        _check(st, "ntt_server_submit")
        return t

    def poll(self, ticket) -> RequestInfo:
        info = RequestInfo()
        _check(_lib.ntt_server_poll(self._h, ticket, ctypes.byref(info)), "ntt_server_poll")
        return info

    def query(self, tickets):
        n = len(tickets)
        arr = (_U64 * max(1, n))(*tickets)
        infos = (RequestInfo * max(1, n))()
        _check(_lib.ntt_server_query(self._h, arr, n, infos), "ntt_server_query")
        return infos[:n]

    def wait(self, ticket, timeout_s=None) -> RequestInfo:
        info = RequestInfo()
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        _check(_lib.ntt_server_wait(self._h, ticket, t, ctypes.byref(info)), "ntt_server_wait")
        return info

    def drain(self, timeout_s=None):
        t = -1 if timeout_s is None else int(timeout_s * 1e9)
        _check(_lib.ntt_server_drain(self._h, t), "ntt_server_drain")

    def read(self, ticket, dst, stream=None):
        _check(_lib.ntt_server_read(self._h, ticket, _ptr(dst), _stream(stream)), "ntt_server_read")

    def release(self, ticket):
        _check(_lib.ntt_server_release(self._h, ticket), "ntt_server_release")

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.ntt_server_stats_get(self._h, ctypes.byref(s)), "ntt_server_stats_get")
        return {n: getattr(s, n) for n, _ in ServerStats._fields_}


def shutdown():
    _check(_lib.ntt_shutdown(), "ntt_shutdown")
