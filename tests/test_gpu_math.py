"""The shading's short square-root and reciprocal sequences are correctly
rounded: for every float of their ranges (about two billion operands each)
they give the same bits as the compiler's correctly rounded sqrtf and
1.0f / y, so the renders keep the operation sequence the oracle evaluates
with IEEE arithmetic.  Run through dr_probe_math."""
import ctypes as C

import pytest
import torch

from paper_2404_09758_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

SQRT_RANGE = (0x0F800000, 0x7E800000)          # [2^-96, 2^126]
RCP_RANGE = (0x01000000, 0x7E000000)           # magnitudes in [2^-125, 2^125]


def mismatches(op, lo, hi):
    lib = L.load()
    bad = torch.zeros(1, dtype=torch.int64, device=DEV)
    first = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    st = lib.dr_probe_math(op, lo, hi, C.c_void_p(bad.data_ptr()), C.c_void_p(first.data_ptr()),
                           C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    return int(bad.item()), int(first.item()) & 0xFFFFFFFF


def test_fast_sqrt_is_correctly_rounded_over_its_range():
    n, first = mismatches(L.PROBE_SQRT, *SQRT_RANGE)
    assert n == 0, f"{n} operands differ, the least {first:#010x}"


@pytest.mark.parametrize("sign", [0, 0x80000000])
def test_fast_reciprocal_is_correctly_rounded_over_its_range(sign):
    lo, hi = RCP_RANGE
    n, first = mismatches(L.PROBE_RCP, lo | sign, hi | sign)
    assert n == 0, f"{n} operands differ, the least {first:#010x}"
