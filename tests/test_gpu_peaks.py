"""The achievable-peak microbenchmarks: they run, give finite positive rates
below the published peaks' reach, and the copy kernel copies."""
import ctypes

import pytest

from gpu_helpers import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_2002_01184_amd import hmc  # noqa: E402


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_memory_rates_and_copy():
    n = 1 << 24                                    # 64 MiB: halves of 32 MiB for the copy
    buf = torch.arange(n, dtype=torch.float32, device="cuda")
    ptr = ctypes.c_void_p(buf.data_ptr())
    rd = hmc.hmc_peak_memory(ptr, n * 4, 0, 1, 2, _stream())
    rd_cached = hmc.hmc_peak_memory(ptr, n * 4, 0, 4, 2, _stream())
    cp = hmc.hmc_peak_memory(ptr, n * 4, 1, 1, 2, _stream())
    torch.cuda.synchronize()
    for v in (rd, rd_cached, cp):
        assert 10.0 < v < 1e6, v                     # GB/s
    assert torch.equal(buf[n // 2:], torch.arange(n // 2, dtype=torch.float32, device="cuda"))


@pytest.mark.parametrize("kind,peak", [(0, 157.3), (1, 157.3), (2, 2500.0), (3, 157.3), (4, 2500.0)])
@pytest.mark.parametrize("waves", [1, 8])
def test_compute_rates(kind, peak, waves):
    tf, mhz = hmc.hmc_peak_compute(kind, 200, 2, _stream(), with_clock=True, waves_per_simd=waves)
    assert 0.0 < tf < 1.05 * peak, (kind, waves, tf)
    assert 500.0 < mhz < 3500.0, mhz
