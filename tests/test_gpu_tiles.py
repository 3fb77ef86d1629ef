"""GPU tests of the right-hand side's launch configurations: the second tile
shape of every order and the vertical chunks give the same steps as the
default configuration (each node's arithmetic does not depend on the tile or
the chunk, in either form, and the precision form stays within 1e-6 of the
FP64 step), and the autotuner keeps
a configuration that the step then uses.  The default configuration is the
one the oracle parity tests check."""
import numpy as np
import pytest

from paper_1702_04316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def numa_mod():
    from paper_1702_04316_amd import numa
    numa.load()
    return numa


# (N, nex, ney, nez): ragged tile coverage in x and y for both shapes
GRIDS = [(1, 5, 3, 4), (2, 5, 3, 3), (3, 5, 3, 4), (4, 5, 3, 3), (5, 5, 3, 3), (6, 4, 3, 2), (7, 3, 2, 3),
         (8, 2, 2, 2)]


def _steps(torch, numa, g, q0, dt, tile, zchunk, mixed=False, nsteps=2, bg=None):
    ctx = numa.Context(g, bg)
    ctx.factor(dt)
    numa.set_rhs_config(ctx.ctx, tile, zchunk)
    cfg = numa.get_rhs_config(ctx.ctx)
    q = torch.from_numpy(q0.copy()).cuda()
    ctx.step(q, nsteps, mixed=mixed)
    ctx.check()
    out = q.cpu().numpy()
    ctx.close()
    return out, cfg


@pytest.mark.parametrize("N,nex,ney,nez", GRIDS)
def test_tiles_and_chunks_give_the_same_steps(torch_cuda, numa_mod, N, nex, ney, nez):
    g = W.Grid(9000.0 * nex, 7000.0 * ney, 6000.0, nex, ney, nez, N)
    dt = min(W.dt_for_courant(g, 15.0, "z"), W.dt_for_courant(g, 0.4, "x"), W.dt_for_courant(g, 0.4, "y"))
    q0 = W.make_random_state(g, 60 + N, wind=4.0)
    fp64 = None
    for mixed in (False, True):
        ref, cfg0 = _steps(torch_cuda, numa_mod, g, q0, dt, 0, 0, mixed)
        if not mixed:
            fp64 = ref
        assert cfg0["tile"] == 0 and cfg0["TX"] % N == 0 and cfg0["TY"] % N == 0
        for tile, zc in ((0, 1), (1, 0), (1, 1)):
            if tile == 1 and N in (6, 8):
                with pytest.raises(numa_mod.NumaError) as ei:  # one shape at N = 6 and 8
                    _steps(torch_cuda, numa_mod, g, q0, dt, tile, zc, mixed)
                assert ei.value.code == numa_mod.NUMA_E_UNSUPPORTED
                continue
            out, cfg = _steps(torch_cuda, numa_mod, g, q0, dt, tile, zc, mixed)
            assert cfg["tile"] == tile and (zc == 0 or cfg["zchunk"] == zc)
            if tile == 1:
                assert (cfg["TX"], cfg["TY"]) != (cfg0["TX"], cfg0["TY"])
            d = max(np.max(np.abs(out[f] - ref[f])) / np.max(np.abs(ref[f])) for f in range(5))
            print(f"N={N} mixed={mixed} tile {tile} ({cfg['TX']}x{cfg['TY']}) zchunk {cfg['zchunk']}: max rel diff {d}")
            assert d < 1e-14, (tile, zc, d)
            if mixed:  # and the precision form stays within its bar of the FP64 step
                e = max(np.linalg.norm(out[f] - fp64[f]) / np.linalg.norm(fp64[f]) for f in range(5))
                assert e < 1e-6, (tile, zc, e)


def test_autotune_keeps_a_configuration(torch_cuda, numa_mod):
    """The tuner leaves the state unchanged, records a valid configuration,
    and the steps it then runs equal the default configuration's."""
    wl = W.ensemble_small_domains()[2]  # N = 5, 13 vertical elements
    g = wl.grid
    q0 = W.make_initial_state(wl)
    ctx = numa_mod.Context(g, wl.background)
    ctx.factor(wl.dt)
    q = torch_cuda.from_numpy(q0.copy()).cuda()
    cfg = numa_mod.autotune(ctx.ctx, q.data_ptr(), reps=2)
    assert np.array_equal(q.cpu().numpy(), q0)
    assert cfg["tile"] in (0, 1) and 1 <= cfg["zchunk"] <= g.nez
    assert numa_mod.get_rhs_config(ctx.ctx) == cfg
    print(f"autotuned {wl.name}: {cfg}")
    ctx.step(q, 3)
    ctx.check()
    ref, _ = _steps(torch_cuda, numa_mod, g, q0, wl.dt, 0, 0, nsteps=3, bg=wl.background)
    d = max(np.max(np.abs(q.cpu().numpy()[f] - ref[f])) / np.max(np.abs(ref[f])) for f in range(5))
    assert d < 1e-14, d
    ctx.close()


def test_rhs_config_argument_errors(torch_cuda, numa_mod):
    g = W.Grid(30000.0, 20000.0, 8000.0, 3, 2, 4, 4)
    ctx = numa_mod.Context(g)
    for tile, zc in ((2, 0), (-1, 0), (0, 5), (0, -1)):
        with pytest.raises(numa_mod.NumaError) as ei:
            numa_mod.set_rhs_config(ctx.ctx, tile, zc)
        assert ei.value.code == numa_mod.NUMA_E_ARG
    lib = numa_mod.load()
    assert lib.numa_autotune(ctx.ctx, None, 1, None) == numa_mod.NUMA_E_ARG
    ctx.close()
