"""The library's float32 -> bfloat16 conversion (the storage rounding of the
bf16 transfer operators of the FP32 cycle) on every one of the 2^32 float32
bit patterns, against the rounding written from its definition (nearest,
ties to even, NaN -> 0x7fc0) and against torch's conversion (NaN inputs
compared as NaN outputs: torch does not fix a single NaN pattern)."""
import pytest
import torch

from bf16_definition import bf16_nearest_even, bit_patterns
from paper_2606_09001_amd import _lib


@pytest.mark.gpu
def test_bf16_conversion_exhaustive():
    L = _lib.load()
    chunk = 1 << 28
    out = torch.empty(chunk, dtype=torch.int16, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    nan_total = 0
    for c in range((1 << 32) // chunk):
        print(f"[bf16] chunk {c}", flush=True)
        u = bit_patterns(c * chunk, chunk, "cuda")
        x = u.view(torch.float32)
        _lib.check(L.amg_convert_bf16(x.data_ptr(), out.data_ptr(), chunk, stream), "amg_convert_bf16")
        got = out.to(torch.int32) & 0xFFFF
        ref = bf16_nearest_even(u) & 0xFFFF
        assert torch.equal(got, ref), c
        del ref
        tb = x.to(torch.bfloat16).view(torch.int16).to(torch.int32) & 0xFFFF
        nan = (u & 0x7FFFFFFF) > 0x7F800000
        nan_total += int(nan.sum())
        assert torch.equal(got[~nan], tb[~nan]), c
        assert bool(((tb[nan] & 0x7FFF) > 0x7F80).all()), c
    assert nan_total == 2 * ((1 << 23) - 1)
