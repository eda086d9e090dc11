"""The library's bandwidth probe (vlbm_copy_probe), the reference copy that
bench.py reports beside the roofline fractions: it must copy exactly, and
reject what it cannot copy without touching the device."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2609_10639_amd import _native

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 20) + 16 * 37, 512 * 16384 * 16 + 16 * 5])
def test_copy_probe_copies_exactly(nbytes):
    g = torch.Generator(device="cpu").manual_seed(nbytes % 1000)
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")   # guard bytes past the end
    stream = torch.cuda.current_stream().cuda_stream
    _native.copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].sum()) == 0


def test_copy_probe_rejects_bad_arguments():
    L = _native.lib()
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.vlbm_copy_probe(p, p, 17, None) == _native.EINVAL
    assert L.vlbm_copy_probe(None, p, 16, None) == _native.EINVAL
    assert L.vlbm_copy_probe(p, None, 16, None) == _native.EINVAL
    assert L.vlbm_copy_probe(p, p, 0, None) == _native.OK   # nothing to copy
    torch.cuda.synchronize()
