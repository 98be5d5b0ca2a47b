"""The device-peak microbenchmarks (include/sal_peak.h) do the work they are timed for: every
compute kind leaves its closed-form checksum in every thread, the read kernel sums exactly what
it was given (a grid that does not divide the buffer included), and the copy is exact."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# per-thread checksum per iteration: 4 chains x 4 accumulators x K = 4; 4 chains x 16 x K = 16; 8 chains of +1
PER_ITER = {0: 64, 1: 1024, 2: 1024, 3: 8}


@pytest.fixture(scope="module")
def torch_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06174_amd import _lib
    return torch, _lib


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("iters,blocks", [(1, 1), (37, 5), (16384, 3)])
def test_compute_checksums(torch_lib, kind, iters, blocks):
    torch, _lib = torch_lib
    lib = _lib.load()
    out = torch.full((blocks * 256,), -1.0, dtype=torch.float32, device="cuda")
    _lib.check(lib.sal_peak_compute(kind, iters, blocks, ctypes.c_void_p(out.data_ptr()), _stream(torch)))
    torch.cuda.synchronize()
    assert bool((out == float(PER_ITER[kind] * iters)).all())


@pytest.mark.parametrize("words,blocks", [(1, 1), (1000, 3), (1 << 20, 7)])
def test_stream_read_and_copy(torch_lib, words, blocks):
    torch, _lib = torch_lib
    lib = _lib.load()
    rng = np.random.default_rng(words + blocks)
    # small integers: every partial sum is exact in fp32
    host = rng.integers(-8, 9, size=4 * words).astype(np.float32)
    src = torch.from_numpy(host).cuda()
    out = torch.full((blocks * 256,), np.nan, dtype=torch.float32, device="cuda")
    _lib.check(lib.sal_peak_stream(0, ctypes.c_void_p(src.data_ptr()), None, 16 * words,
                                   ctypes.c_void_p(out.data_ptr()), blocks, _stream(torch)))
    dst = torch.full_like(src, np.nan)
    _lib.check(lib.sal_peak_stream(1, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), 16 * words,
                                   None, blocks, _stream(torch)))
    torch.cuda.synchronize()
    # thread i of the grid read the 16-byte words i, i + G, i + 2G, ... (G threads)
    g = blocks * 256
    per_word = host.reshape(words, 4).astype(np.float64).sum(axis=1)
    expect = np.zeros(g)
    np.add.at(expect, np.arange(words) % g, per_word)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), expect)
    assert torch.equal(dst, src)
