"""FFT core of the HIP library against numpy's FFT (fp64), stage by stage."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("n", [160, 320, 640])
def test_row_r2c(torch, n):
    from paper_1705_06603_amd._lib import debug_fft
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n, n)).astype(np.float32)
    out = debug_fft(n, 0, torch.tensor(x, device="cuda")).cpu().numpy()
    got = out[..., 0] + 1j * out[..., 1]                     # [b][f][i]
    ref = np.fft.rfft(x.astype(np.float64), axis=2)          # [b][i][f]
    exp = np.transpose(ref[:, :, : n // 2], (0, 2, 1)).copy()
    exp[:, 0, :] = ref[:, :, 0].real + 1j * ref[:, :, n // 2].real
    err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    assert err < 1e-6, err


@pytest.mark.parametrize("n", [160, 320, 640])
@pytest.mark.parametrize("which", [1, 2])
def test_column_fft(torch, n, which):
    from paper_1705_06603_amd._lib import debug_fft
    rng = np.random.default_rng(n + which)
    z = rng.standard_normal((2, n // 2, n)) + 1j * rng.standard_normal((2, n // 2, n))
    inp = np.stack([z.real, z.imag], -1).astype(np.float32)
    out = debug_fft(n, which, torch.tensor(inp, device="cuda")).cpu().numpy()
    got = out[..., 0] + 1j * out[..., 1]
    zz = inp[..., 0].astype(np.float64) + 1j * inp[..., 1]
    exp = np.fft.fft(zz, axis=2) if which == 1 else np.fft.ifft(zz, axis=2) * n
    err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    assert err < 1e-6, err


@pytest.mark.parametrize("n", [160, 320, 640])
def test_row_c2r_inverts_r2c(torch, n):
    from paper_1705_06603_amd._lib import debug_fft
    rng = np.random.default_rng(7 * n)
    x = rng.standard_normal((2, n, n)).astype(np.float32)
    spec = debug_fft(n, 0, torch.tensor(x, device="cuda"))
    back = debug_fft(n, 3, spec).cpu().numpy()
    err = np.linalg.norm(back - x * (n / 2)) / np.linalg.norm(x * (n / 2))
    assert err < 1e-6, err
