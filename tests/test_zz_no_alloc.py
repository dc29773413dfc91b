"""pm_deposit_noalloc (the deposit with library-held scratch, for callers
that cannot allocate) against pm_deposit with a caller workspace, through
the C ABI: bitwise equal grids on two calls in a row, the second smaller,
and sizes beyond the scratch array rejected."""
import ctypes

import numpy as np
import pytest

from workloads import lognormal_particles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    from paper_2604_15434_amd import _lib as L

    return L, L.lib()


def _noalloc(lib, pos, ng, rho):
    dt = 1 if pos.dtype == torch.float64 else 0
    return lib.pm_deposit_noalloc(ctypes.c_void_p(pos.data_ptr()), pos.shape[1], dt, ng,
                                  ctypes.c_void_p(rho.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_deposit_equals_workspace_deposit(dtype):
    import paper_2604_15434_amd as P

    L, lib = _lib()
    assert lib.pm_deposit_noalloc_max_bytes() == 33 << 20
    prev = None
    for ng, npart_side, seed in ((128, 128, 2), (64, 48, 3)):  # the second call smaller
        pos_np, _ = lognormal_particles(ng, 250.0 * ng / 128, seed=seed, n_particles=npart_side**3)
        pos = torch.from_numpy(pos_np).to("cuda", dtype)
        ref = torch.empty((ng, ng, ng), dtype=dtype, device="cuda")
        P.pm_deposit(pos, ng, ref)
        got = torch.full((ng, ng, ng), -1.0, dtype=dtype, device="cuda")
        assert _noalloc(lib, pos, ng, got) == 0
        torch.cuda.synchronize()
        assert torch.equal(got, ref), ng
        if prev is not None:
            assert prev.shape != got.shape
        prev = got
    # beyond the scratch array (16 bytes per cell): rejected, nothing launched
    big = torch.zeros((3, 8), dtype=dtype, device="cuda")
    out = torch.zeros((192, 192, 192), dtype=dtype, device="cuda")
    assert _noalloc(lib, big, 192, out) == L.PM_ENOMEM
    assert float(out.abs().max()) == 0.0
    assert _noalloc(lib, big, 10, out) == L.PM_EINVAL
