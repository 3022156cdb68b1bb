"""float32 -> bfloat16 rounding written from its definition (test
infrastructure): of the two bfloat16 neighbours of x, a (toward zero) and b
(away from zero), take the one nearer to x, measured exactly in float64; on a
tie take the one whose last stored bit is 0 (round half to even).  Past the
largest finite bfloat16 the neighbour b is infinity, which counts as 2^128
(IEEE overflow: rounding as if the exponent range were unbounded).  An
infinity stays itself; every NaN becomes the quiet NaN 0x7fc0.

Works on CPU or GPU tensors; used to pin torch's conversion (CPU) and the
library's conversion kernel (GPU) over all 2^32 float32 bit patterns.
"""
import torch

_QNAN = 0x7FC0
_INF_BITS = 0x7F80


def bf16_nearest_even(u: torch.Tensor) -> torch.Tensor:
    """u: int32 tensor of float32 bit patterns.  Returns int32 tensor of the
    bfloat16 bit patterns (0..0xffff)."""
    u = u.to(torch.int64) & 0xFFFFFFFF
    sign = u >> 31
    mag = u & 0x7FFFFFFF
    a_bits = mag >> 16
    b_bits = a_bits + 1
    f64 = lambda bits32: bits32.to(torch.int32).view(torch.float32).to(torch.float64)  # noqa: E731
    x = f64(mag)
    a = f64(a_bits << 16)
    b = torch.where(b_bits == _INF_BITS, torch.full_like(x, 2.0 ** 128), f64(b_bits << 16))
    finite = mag < 0x7F800000
    da = torch.where(finite, x - a, torch.zeros_like(x))
    db = torch.where(finite, b - x, torch.ones_like(x))
    tie_pick = torch.where((a_bits & 1) == 0, a_bits, b_bits)
    pick = torch.where(da < db, a_bits, torch.where(db < da, b_bits, tie_pick))
    out = (sign << 15) | pick
    out = torch.where(mag > 0x7F800000, torch.full_like(out, _QNAN), out)
    return out.to(torch.int32)


def bit_patterns(start: int, count: int, device) -> torch.Tensor:
    """int32 tensor holding the float32 bit patterns start .. start+count-1
    (unsigned 32-bit numbers, start + count <= 2^32)."""
    v = torch.arange(start, start + count, dtype=torch.int64, device=device)
    return torch.where(v >= (1 << 31), v - (1 << 32), v).to(torch.int32)
