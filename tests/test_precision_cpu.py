"""Pins of the float32 -> bfloat16 rounding definition used by the precision
checks (CPU): hand-worked IEEE cases, and torch's conversion on every low
half-word under the high half-words where the rule changes (zero and
subnormals, an odd and an even last kept bit, the largest finite values next
to overflow, infinity and NaN, both signs) plus a seeded random sample of all
bit patterns.  torch's vectorized CPU conversion writes 0xffff for every NaN
(its scalar path 0x7fc0), so NaN inputs are compared as NaN outputs; every
other input bit for bit.  The GPU suite sweeps all 2^32 patterns."""
import numpy as np
import torch

from bf16_definition import bf16_nearest_even, bit_patterns


def _u32(vals):
    return torch.tensor([v - (1 << 32) if v >= (1 << 31) else v for v in vals], dtype=torch.int64).to(torch.int32)


def test_hand_worked_cases():
    cases = {
        0x3F800000: 0x3F80,  # 1.0 exact
        0x3F800001: 0x3F80,  # just above 1: down
        0x3F808000: 0x3F80,  # halfway, kept bit even: down
        0x3F818000: 0x3F82,  # halfway, kept bit odd: up
        0x3F808001: 0x3F81,  # above halfway: up
        0xBF808001: 0xBF81,  # same, negative
        0x7F7F7FFF: 0x7F7F,  # largest finite, below halfway to overflow
        0x7F7F8000: 0x7F80,  # halfway to overflow, kept bit odd: infinity
        0x7F7FFFFF: 0x7F80,  # largest float32: infinity
        0x7F800000: 0x7F80,  # +inf
        0xFF800000: 0xFF80,  # -inf
        0x7FC00000: 0x7FC0,  # quiet NaN
        0xFFC00001: 0x7FC0,  # negative NaN with payload
        0x7F800001: 0x7FC0,  # signalling NaN
        0x00000000: 0x0000,
        0x80000000: 0x8000,  # -0
        0x00000001: 0x0000,  # smallest subnormal: down to +0
        0x00008000: 0x0000,  # halfway between 0 and the smallest bf16 subnormal: even (0)
        0x00018000: 0x0002,  # halfway, kept bit odd: up
        0x007FFFFF: 0x0080,  # largest subnormal rounds up to the smallest normal
    }
    got = bf16_nearest_even(_u32(list(cases))).tolist()
    assert [g & 0xFFFF for g in got] == list(cases.values())


def _torch_bf16(u):
    return u.view(torch.float32).to(torch.bfloat16).view(torch.int16).to(torch.int32) & 0xFFFF


def test_definition_equals_torch_on_rule_boundaries_and_sample():
    highs = [0x0000, 0x0001, 0x0002, 0x007F, 0x0080, 0x3F80, 0x3F81, 0x4B7F, 0x7F7E, 0x7F7F, 0x7F80, 0x7F81,
             0x7FC0, 0x7FFF]
    highs += [h | 0x8000 for h in highs]
    parts = [bit_patterns(h << 16, 1 << 16, "cpu") for h in highs]
    rng = np.random.default_rng(20)
    r = rng.integers(0, 1 << 32, size=1 << 22, dtype=np.uint64).astype(np.int64)
    parts.append(torch.from_numpy(np.where(r >= (1 << 31), r - (1 << 32), r)).to(torch.int32))
    u = torch.cat(parts)
    ref = bf16_nearest_even(u) & 0xFFFF
    tb = _torch_bf16(u)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    assert int(nan.sum()) > 5 * (1 << 16)
    assert torch.equal(ref[~nan], tb[~nan])
    assert bool(((tb[nan] & 0x7FFF) > 0x7F80).all()) and bool((ref[nan] == 0x7FC0).all())
