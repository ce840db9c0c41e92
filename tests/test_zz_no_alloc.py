"""The allocation-free closest-hit entry point (sc_trace_rays_noalloc), for
callers that cannot allocate device memory, against sc_trace_rays: the same
hits bit for bit on two calls in a row (the second smaller, so stale
staging from the first must not leak into it), and sizes beyond the
stated maximum rejected before any work is enqueued."""
import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu


def _rays(rng, n, center, spread):
    O = (center + rng.normal(size=(n, 3)) * spread).astype(np.float32)
    D = rng.normal(size=(n, 3))
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    return torch.from_numpy(O).cuda(), torch.from_numpy(D).cuda()


def test_noalloc_equals_trace_rays():
    import paper_2107_11008_amd as sc
    ctx = sc.Context(0)
    c = sg.config2(tri_scale=0.03, w=64, h=64)
    bvh = ctx.build_bvh(c["scene"])
    rng = np.random.default_rng(5)
    for n in (70001, 1937):
        O, D = _rays(rng, n, np.array([0.0, 0.0, 0.2]), 0.8)
        ref = [x.cpu().numpy() for x in ctx.trace_rays(bvh, O, D)]
        t = torch.full((n,), -1.0, device="cuda")
        prim = torch.full((n,), -2, dtype=torch.int32, device="cuda")
        u = torch.full((n,), -1.0, device="cuda")
        v = torch.full((n,), -1.0, device="cuda")
        ctx.trace_rays_noalloc(bvh, O, D, t, prim, u, v)
        got = [x.cpu().numpy() for x in (t, prim, u, v)]
        for a, b in zip(ref, got):
            assert a.tobytes() == b.tobytes()
        assert (ref[1] != -1).sum() > n // 20
    lib = sc._sc.load()
    big = lib.sc_trace_rays_noalloc_max() + 1
    O = torch.zeros((big, 3), device="cuda")
    D = torch.zeros((big, 3), device="cuda")
    t = torch.empty(big, device="cuda")
    prim = torch.empty(big, dtype=torch.int32, device="cuda")
    with pytest.raises(sc.ScError):
        ctx.trace_rays_noalloc(bvh, O, D, t, prim)
    torch.cuda.synchronize()
    ctx.close()
