"""Helpers for the GPU parity tests: host numpy uint64 <-> device tensors."""
import numpy as np


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda:0")


def from_dev(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def empty_dev(n: int):
    import torch
    return torch.empty(n, dtype=torch.int64, device="cuda:0")


def have_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


WIDE_BOUND = 1 << 58


def lazy_words_exact(nt, N, moduli) -> bool:
    """True when a single-limb-size transform at degree N over these moduli yields the lazy
    words of Algorithms 4 and 5.  The wide-range butterflies (on unless switched off) run for
    N <= 2^14 when every modulus is below 2^58; their lazy outputs are other representatives."""
    return not (nt.get_wide_range() and N <= (1 << 14) and max(int(q) for q in moduli) < WIDE_BOUND)
