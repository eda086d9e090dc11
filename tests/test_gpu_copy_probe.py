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


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, 1 << 26])
def test_read_probe_reads_every_word(nbytes):
    """Read-only mode: the XOR of the per-workgroup words equals the XOR of
    every 16-byte word of the source."""
    g = torch.Generator(device="cpu").manual_seed(nbytes % 997)
    host = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, generator=g)
    src = host.cuda()
    out_bytes = _native.lib().vlbm_copy_probe_read_bytes(nbytes)
    assert 16 <= out_bytes <= 128 * 1024
    dst = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    _native.copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream, 1)
    torch.cuda.synchronize()
    words = host.numpy().view(np.uint64).reshape(-1, 2)
    expect = np.bitwise_xor.reduce(words, axis=0)
    got = np.bitwise_xor.reduce(dst.cpu().numpy().view(np.uint64).reshape(-1, 2), axis=0)
    assert np.array_equal(got, expect)


def test_copy_probe_rejects_bad_arguments():
    L = _native.lib()
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.vlbm_copy_probe(p, p, 17, None, 0) == _native.EINVAL
    assert L.vlbm_copy_probe(None, p, 16, None, 0) == _native.EINVAL
    assert L.vlbm_copy_probe(p, None, 16, None, 0) == _native.EINVAL
    assert L.vlbm_copy_probe(p, p, 16, None, 2) == _native.EINVAL
    assert L.vlbm_copy_probe(p, p, 0, None, 0) == _native.OK   # nothing to copy
    assert L.vlbm_copy_probe(p, p, 0, None, 1) == _native.OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_march_probe_leaves_the_state(precision):
    """The march probe reads the current populations and writes only the spare
    buffer: the state, and the steps that follow, are those of a run without it."""
    from helpers import riemann_case
    from paper_2609_10639_amd import Solver
    W0, cfg, _ = riemann_case(128, 3)
    s = Solver(precision=precision, **cfg)
    s.init(W0)
    s.step(5)
    f0, clock0 = s.f(), s.clock()
    s.probe_march(3)
    torch.cuda.synchronize()
    assert np.array_equal(s.f(), f0) and s.clock() == clock0
    s.step(2)
    ref = Solver(precision=precision, **cfg)
    ref.init(W0)
    ref.step(7)
    assert np.array_equal(s.f(), ref.f())
    d1 = Solver(precision=precision, **dict(cfg, dim=1, ny=1, bc=(1, 1, 1, 1), sensor=1))
    with pytest.raises(_native.VlbmError):
        d1.probe_march(1)
