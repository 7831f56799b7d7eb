"""The allocation-free weights entry point against the allocating one, through the C ABI:
same kernels, so the weights and the statistics must agree bit for bit. Two calls in a row,
the second with a smaller input (the shared scratch keeps the first call's contents, which
the second must not read), then the size limit."""
import numpy as np
import pytest

from gpu_util import dev, host, note, torch_cuda
from paper_2410_05190_amd import binding

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    ll = rng.normal(-3.0, 2.0, n)
    ll[rng.random(n) < 0.1] = -np.inf  # draws outside the support
    lp = rng.normal(0.0, 0.5, n)
    lq = rng.normal(1.0, 0.5, n)
    return ll, lp, lq


def test_noalloc_weights_equal_the_allocating_call():
    torch = torch_cuda()
    for n, seed in ((3_000_000, 1), (5_000, 2), (1, 3), (0, 4)):
        ll, lp, lq = (dev(x) for x in _inputs(n, seed))
        w_a = torch.full((max(n, 1),), -7.0, dtype=torch.float64, device="cuda")
        w_b = torch.full((max(n, 1),), -7.0, dtype=torch.float64, device="cuda")
        st_a = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
        st_b = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
        binding.pe_weights_ess(ll, lp, lq, n, w_a, st_a)
        binding.pe_weights_ess_noalloc(ll, lp, lq, n, w_b, st_b)
        torch.cuda.synchronize()
        a, b = host(st_a), host(st_b)
        note(f"n={n}: ESS {b[0]:.6g} (allocating call {a[0]:.6g})")
        assert np.array_equal(a, b, equal_nan=True)
        assert np.array_equal(host(w_a)[:n], host(w_b)[:n])
        if n > 0:
            assert b[3] > 0 and abs(host(w_b)[:n].sum() - 1.0) < 1e-12


def test_noalloc_weights_size_limit():
    torch = torch_cuda()
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.PeError):
        binding.pe_weights_ess_noalloc(x, x, x, (1 << 24) + 1, None, torch.zeros(4, dtype=torch.float64,
                                                                                device="cuda"))
