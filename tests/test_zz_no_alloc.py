"""The allocation-free MSE entry point (hfe_nn_mse_noalloc) through the C
ABI against hfe_nn_mse with a caller-provided partial-sum buffer: the same
kernels on the same inputs give the same bits, on two calls in a row, the
second with a smaller input (the library-owned scratch keeps the first
call's rows, which the second must not read)."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_mse_equals_the_workspace_entry_point():
    torch = require_gpu()
    from paper_2207_10657_amd import hfe
    lib = hfe.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(11)
    for n in (3 * 64 ** 3 + 17, 1000):
        announce("no-alloc mse, n =", n)
        pred = torch.tensor(rng.normal(size=n), dtype=torch.float32, device="cuda")
        target = torch.tensor(rng.normal(size=n), dtype=torch.float32, device="cuda")
        g0 = torch.empty(n, dtype=torch.float32, device="cuda")
        g1 = torch.empty(n, dtype=torch.float32, device="cuda")
        loss0 = torch.empty(1, dtype=torch.float64, device="cuda")
        loss1 = torch.empty(1, dtype=torch.float64, device="cuda")
        parts = torch.empty(int(lib.hfe_nn_mse_partials(n)), dtype=torch.float64, device="cuda")
        assert lib.hfe_nn_mse(_ptr(pred), _ptr(target), n, _ptr(g0), _ptr(parts), _ptr(loss0),
                              stream) == 0
        assert lib.hfe_nn_mse_noalloc(_ptr(pred), _ptr(target), n, _ptr(g1), _ptr(loss1),
                                      stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(g0, g1)
        assert loss0.item() == loss1.item()
        # the kernel forms d = pred - target in float32, then sums d*d in float64
        d = (pred.cpu().numpy() - target.cpu().numpy()).astype(np.float64)
        ref = float(np.mean(d * d))
        assert abs(loss1.item() - ref) <= 1e-12 * ref
    # invalid sizes are rejected before any launch
    assert lib.hfe_nn_mse_noalloc(_ptr(pred), _ptr(target), 0, _ptr(g1), _ptr(loss1), stream) == -1
