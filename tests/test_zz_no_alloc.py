"""The allocation-free residual (sdsl_residual_noalloc) against sdsl_residual
through the C ABI: two calls in a row on one device, the second on a smaller
system, each bitwise equal to the allocating entry point's result (same
kernels, same launch shapes, scratch instead of handle buffers)."""
import numpy as np
import pytest

from ipm_inputs import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2604_23979_amd as sd  # noqa: E402


def _check(system, o, seed):
    sv = sd.from_system(system, o)
    try:
        rng = np.random.default_rng(seed)
        b = torch.as_tensor(system.b, device="cuda:0")
        x = torch.as_tensor(rng.standard_normal(system.n), device="cuda:0")
        r_ref, n_ref = sv.residual(b, x)
        r = torch.full_like(b, float("nan"))
        torch.cuda.synchronize()
        # every device allocation of the library goes through torch's
        # allocator (the handle's hook); the call must add none
        before = torch.cuda.memory_stats()["allocation.all.allocated"]
        nr = sv.residual_noalloc(b, x, r)
        torch.cuda.synchronize()
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
        assert torch.equal(r, r_ref)
        assert nr == n_ref and np.isfinite(nr) and nr > 0
    finally:
        sv.close()


def test_noalloc_residual_matches_residual_twice_second_smaller():
    print("\n[no-alloc residual: C2 x0.02 with its low-rank term, then C1]", flush=True)
    big = gen.c2(0.02)
    _check(big, sd.Options(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM), 3)
    small = gen.c1()
    assert small.n < big.n
    _check(small, sd.Options(), 4)
