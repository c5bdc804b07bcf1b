"""GPU parity of the kernel-level entry points (z-FFT, Hankel-transform GEMM)
against their mathematical definitions computed in FP64 on the CPU."""
import numpy as np
import pytest

from workloads import random_spectral

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_05712_amd import pic
    pic.load()


@pytest.mark.parametrize("nz,rows", [(16, 3), (32, 5), (64, 7), (128, 9), (256, 33), (512, 6), (1024, 4),
                                     (2048, 5), (4096, 3)])
@pytest.mark.parametrize("inverse", [False, True])
def test_fft_z_matches_dft(nz, rows, inverse):
    from paper_1611_05712_amd import pic
    x = random_spectral((rows, nz), seed=nz + rows).astype(np.complex64)
    t = torch.from_numpy(x.copy()).cuda()
    pic.fft_z(t, inverse=inverse)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.complex128)
    xd = x.astype(np.complex128)
    want = np.fft.ifft(xd, axis=-1) if inverse else np.fft.fft(xd, axis=-1)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < 3e-7 * np.log2(nz), rel


def test_fft_z_small_brute_force():
    # O(N^2) DFT of the definition, N = 16
    from paper_1611_05712_amd import pic
    n = 16
    x = random_spectral((2, n), seed=3).astype(np.complex64)
    t = torch.from_numpy(x.copy()).cuda()
    pic.fft_z(t)
    torch.cuda.synchronize()
    j = np.arange(n)
    Wm = np.exp(-2j * np.pi * np.outer(j, j) / n)
    want = x.astype(np.complex128) @ Wm.T
    np.testing.assert_allclose(t.cpu().numpy(), want, rtol=0, atol=5e-6 * np.abs(want).max())


def _gemm_case(n, ncols, batch, prec, seed=0):
    from paper_1611_05712_amd import pic
    rng = np.random.default_rng(seed + n + ncols)
    A = [rng.standard_normal((n, n)) for _ in range(batch)]
    X = [rng.standard_normal((n, ncols)) for _ in range(batch)]
    at = [torch.tensor(a.T.copy(), dtype=torch.float32).cuda() for a in A]
    xs = [torch.tensor(x, dtype=torch.float32).cuda() for x in X]
    ys = [torch.empty((n, ncols), dtype=torch.float32).cuda() for _ in range(batch)]
    pic.dht_gemm(at, xs, ys, prec=prec)
    torch.cuda.synchronize()
    errs = []
    for a, x, y in zip(A, X, ys):
        a32 = a.astype(np.float32).astype(np.float64)
        x32 = x.astype(np.float32).astype(np.float64)
        want = a32 @ x32
        errs.append(np.linalg.norm(y.cpu().numpy() - want) / np.linalg.norm(want))
    return max(errs)


@pytest.mark.parametrize("n,ncols,batch", [(32, 128, 1), (64, 512, 3), (96, 256, 2), (128, 256, 1),
                                           (256, 4096, 2)])
def test_dht_gemm_fp32(n, ncols, batch):
    assert _gemm_case(n, ncols, batch, 0) < 2e-6


@pytest.mark.parametrize("prec,tol", [(1, 3e-5), (2, 3e-6)])
@pytest.mark.parametrize("n,ncols", [(64, 256), (256, 1024)])
def test_dht_gemm_split_precision(prec, tol, n, ncols):
    # hi+lo split keeps ~16 (bf16) / ~22 (fp16) mantissa bits per operand
    assert _gemm_case(n, ncols, 2, prec) < tol
