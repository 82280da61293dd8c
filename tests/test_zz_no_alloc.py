"""lagp_nn_pool_static: the grid-pruned pools built in the library's static
device scratch, for callers that cannot allocate, against lagp_nn_pool_ws
(caller workspace) bit for bit.  Two calls in a row, the second with a smaller
input, so that the second call runs on what the first left in the scratch."""
import ctypes

import numpy as np
import pytest

import workloads
from paper_1310_5182_amd import _lib


def test_static_size_limit_rejected_before_any_launch():
    """A problem whose grid tables exceed the static scratch is refused on the
    host (LAGP_EWORKSPACE), with no device pointer touched."""
    L = _lib.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the call is rejected first
    N, p, M = (1 << 31) - 1, 8, 1000
    need = ctypes.c_size_t(0)
    assert L.lagp_nn_pool_workspace(N, p, M, ctypes.byref(need)) == 0
    assert need.value > (128 << 20)
    rc = L.lagp_nn_pool_static(fake, N, p, fake, M, 100, fake, None)
    assert rc == _lib.LAGP_EWORKSPACE
    assert b"static scratch" in L.lagp_last_error()
    # M = 0 is a no-op, also without a device
    assert L.lagp_nn_pool_static(fake, 1000, p, fake, 0, 100, fake, None) == 0


@pytest.mark.gpu
def test_static_pools_equal_workspace_pools():
    import torch

    import paper_1310_5182_amd as lagp

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    cases = [(2, 60000, 700, 1000), (3, 20000, 300, 400)]  # (config, N, M, N'): the second smaller
    for cfg, N, M, Np in cases:
        W = workloads.make(cfg, N=N, M=M)
        print(f"[no-alloc] config{cfg} N={N} M={M} Np={Np}", flush=True)
        X, XX = dev(W.X), dev(W.XX)
        ref = lagp.nn_pool(X, XX, Np, grid=True)
        out = torch.full((M, Np), -7, dtype=torch.int32, device="cuda")
        got = lagp.nn_pool_static(X, XX, Np, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), (cfg, N, M, Np)
        # and the plain (unpruned) pools: the same again
        assert torch.equal(got, lagp.nn_pool(X, XX, Np))
