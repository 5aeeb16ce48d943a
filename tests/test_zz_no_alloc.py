"""The allocation-free FFT stages (deblur_debug_fft_noalloc) against the
allocating entry point (deblur_debug_fft): the same stages must give the same
results, also when a call follows one with a larger frame and batch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _input(n, batch, which, seed):
    rng = np.random.default_rng(seed)
    if which == 0:
        return rng.standard_normal((batch, n, n)).astype(np.float32)
    return rng.standard_normal((batch, n // 2, n, 2)).astype(np.float32)


def _compare(torch, n, batch, which, seed):
    from paper_1705_06603_amd._lib import debug_fft
    data = torch.tensor(_input(n, batch, which, seed), device="cuda")
    ref = debug_fft(n, which, data)
    shape = (batch, n, n) if which == 3 else (batch, n // 2, n, 2)
    out = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
    got = debug_fft(n, which, data, out=out, noalloc=True)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, ref), (n, batch, which, float((got - ref).abs().max()))


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_noalloc_fft_equals_the_allocating_stage_on_two_calls(torch, which):
    print(f"noalloc FFT stage {which}: 640 x 6 frames, then 160 x 2", flush=True)
    _compare(torch, 640, 6, which, seed=10 + which)
    _compare(torch, 160, 2, which, seed=20 + which)


def test_noalloc_fft_third_call_mid_size(torch):
    print("noalloc FFT: 320 x 3 frames after the smaller call", flush=True)
    for which in range(4):
        _compare(torch, 320, 3, which, seed=30 + which)


def test_noalloc_fft_rejects_a_batch_beyond_its_scratch(torch):
    from paper_1705_06603_amd import _lib as dl
    L = dl.lib()
    buf = torch.zeros(16, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    rc = L.deblur_debug_fft_noalloc(160, 4097, 0, p, p, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1                                     # DEBLUR_E_ARG
    assert "allocation-free limit of 4096" in L.deblur_last_error(None).decode()
