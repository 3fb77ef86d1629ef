"""GPU test of numa_hevi_step_mixed_noalloc: the precision-form step with the
library's fixed stage buffers instead of allocated ones.  Three calls in a
row on three contexts, the second grid smaller than the first, the third
over a stratified background, each compared with numa_hevi_step_mixed on the
same input (same kernels and arithmetic, so the results agree bit for bit);
a grid above the fixed size is refused."""
import ctypes as C

import numpy as np
import pytest

from paper_1702_04316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1702_04316_amd import numa
    numa.load()
    return torch, numa


def _grid_state(torch, numa, g, seed, bg=None):
    ctx = numa.Context(g, bg)
    dt = W.dt_for_courant(g, 15.0, "z")
    ctx.factor(dt)
    q0 = torch.from_numpy(W.make_random_state(g, seed)).cuda()
    return ctx, dt, q0


def test_noalloc_matches_allocating_entry_point(env):
    torch, numa = env
    lib = numa.load()
    # first a grid of 96x96x33 = 304,128 nodes (29 MB of the 64 MiB array),
    # then 16x16x17 = 4,352 nodes, then 12x12x25 over a stratified
    # background (whose stage buffers also hold theta' of Q2 and Q3); 100 km
    # elements keep the horizontal Courant number small at vertical Courant
    # number 15
    grids = [(W.Grid(2.4e6, 2.4e6, 8000.0, 24, 24, 8, 4), None),
             (W.Grid(4.0e5, 4.0e5, 4000.0, 4, 4, 4, 4), None),
             (W.Grid(3.0e5, 3.0e5, 8000.0, 3, 3, 6, 4), W.Background(nbv=0.01))]
    for n, (g, bg) in enumerate(grids):
        ctx, dt, q0 = _grid_state(torch, numa, g, seed=30 + n, bg=bg)
        print(f"noalloc case {n}: grid {g.nx}x{g.ny}x{g.nz}, N={g.N}, dt={dt}", flush=True)
        a, b = q0.clone(), q0.clone()
        rc = lib.numa_hevi_step_mixed_noalloc(ctx.ctx, C.c_void_p(b.data_ptr()), dt, 3)
        assert rc == numa.NUMA_OK, numa.last_error(ctx.ctx)
        assert lib.numa_hevi_step_mixed(ctx.ctx, C.c_void_p(a.data_ptr()), dt, 3) == numa.NUMA_OK
        ctx.check()
        x, y = a.cpu().numpy(), b.cpu().numpy()
        diff = np.abs(x - y).max()
        moved = np.abs(x - q0.cpu().numpy()).max()
        print(f"noalloc case {n}: max |noalloc - allocating| = {diff}, max change over the steps = {moved}",
              flush=True)
        assert moved > 0.0
        assert np.array_equal(x, y)
        ctx.close()


def test_noalloc_refuses_grid_above_fixed_size(env):
    torch, numa = env
    lib = numa.load()
    g = W.Grid(3.2e6, 3.2e6, 8000.0, 32, 32, 10, 4)  # 128x128x41 = 671,744 nodes: fits (at most 699,050)
    ctx, dt, q0 = _grid_state(torch, numa, g, seed=40)
    assert lib.numa_hevi_step_mixed_noalloc(ctx.ctx, C.c_void_p(q0.data_ptr()), dt, 1) == numa.NUMA_OK
    ctx.check()
    ctx.close()
    g = W.Grid(3.2e6, 3.2e6, 8000.0, 32, 32, 11, 4)  # 128x128x45 = 737,280 nodes: too large
    ctx, dt, q0 = _grid_state(torch, numa, g, seed=41)
    q1 = q0.clone()
    rc = lib.numa_hevi_step_mixed_noalloc(ctx.ctx, C.c_void_p(q1.data_ptr()), dt, 1)
    assert rc == numa.NUMA_E_UNSUPPORTED
    assert "bytes" in numa.last_error(ctx.ctx)
    ctx.check()
    assert torch.equal(q0, q1)
    assert lib.numa_hevi_step_mixed_noalloc(ctx.ctx, None, dt, 1) == numa.NUMA_E_ARG
    ctx.close()
