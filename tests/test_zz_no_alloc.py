"""The allocation-free energy entry point (pts_energy_device_noalloc)
against pts_energy_device: calls in a row on one fresh context, each
smaller than the one before (1024 partial blocks, then 4, then none),
bitwise equal results, and not one allocation request reaching the
context's allocator."""
import numpy as np
import pytest

from oracle import irls

pytestmark = pytest.mark.gpu


def test_energy_noalloc_matches_energy_device(ptslib):
    import torch

    pts = ptslib
    alloc = pts.TorchAllocator(0)
    ctx = pts.Context(0, allocator=alloc)  # only the allocation-free call runs here
    ref_ctx = pts.Context(0)
    g = torch.Generator().manual_seed(11)
    for n in (400_000, 1_000, 0):
        print(f"case: energy noalloc n={n}", flush=True)
        d = torch.rand(n, generator=g, dtype=torch.float64) * 3.0
        d[: n // 10] *= 1e-3  # some distances below delta (the quadratic branch)
        dist = d.to(torch.float32).cuda()
        out = torch.full((2,), float("nan"), device="cuda")
        ctx.energy_device_noalloc(dist, out)
        ref = ref_ctx.energy_device(dist)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (got, want)
        E, E2 = irls.energy(dist.cpu().numpy().astype(np.float64))
        assert abs(float(got[0]) - E) <= 1e-5 * max(1.0, E), (got[0], E)
        assert abs(float(got[1]) - E2) <= 1e-5 * max(1.0, E2), (got[1], E2)
        assert alloc.calls == 0 and alloc.in_use == 0
    ctx.close()
    ref_ctx.close()
