"""GPU tests of the batched ensemble (numa_ensemble_*): one HIP graph per
step over several domains of different orders and sizes.

The graph launches the same kernels with the same arguments as the eager
step of each context, so every replay must match the eager step bit for
bit.  Replays are interleaved with eager work on the same GPU and each is
checked, in the FP64 form and in the precision form.
"""
import ctypes as C

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


# (N, nex, ney, nez, wind u, v, seed): orders 3..7, ragged tiles, winds, and
# tall columns (N = 5 with 71 levels, N = 7 with 113) whose column solves use
# eight wavefronts and more than 64 KB of LDS per workgroup
DOMAINS = [(3, 6, 5, 4, 12.0, -3.0, 1), (4, 5, 4, 3, 0.0, 0.0, 2), (5, 3, 3, 3, -8.0, 5.0, 3),
           (7, 2, 3, 2, 4.0, 15.0, 4), (4, 9, 2, 5, 20.0, 0.0, 5), (5, 3, 2, 14, 6.0, -6.0, 6),
           (7, 2, 2, 16, -10.0, 2.0, 7)]


def _domain(torch, numa, N, nex, ney, nez, u, v, seed):
    lz = 8000.0
    g = W.Grid(6000.0 * nex, 5000.0 * ney, lz, nex, ney, nez, N)
    dt = min(W.dt_for_courant(g, 15.0, "z"), W.dt_for_courant(g, 0.3, "x"), W.dt_for_courant(g, 0.3, "y"))
    wl = W.Workload(f"d{seed}", g, dt, 5, seed, 2, (0.2, 1.0), (800.0, 1500.0), wind=(u, v))
    ctx = numa.Context(g)
    ctx.factor(dt)
    return ctx, torch.from_numpy(W.make_initial_state(wl)).cuda()


@pytest.mark.parametrize("mixed", [False, True])
def test_ensemble_replays_match_eager_steps(torch_cuda, numa_mod, mixed):
    doms = [_domain(torch_cuda, numa_mod, *d) for d in DOMAINS]
    ctxs = [c for c, _ in doms]
    states = [q for _, q in doms]
    refs = [q.clone() for q in states]
    ens = numa_mod.Ensemble(ctxs, states, mixed=mixed, tune=True)
    z = ens.zchunks()
    assert all(1 <= zc <= c.info()["nz"] for zc, c in zip(z, ctxs)), z
    for replay in range(3):
        ens.step(1)
        ens.sync()
        for c, r in zip(ctxs, refs):  # eager work between replays
            c.step(r, 1, mixed=mixed)
            c.check()
        for i, (q, r) in enumerate(zip(states, refs)):
            assert torch_cuda.equal(q, r), f"domain {i}, replay {replay}"
    # several steps per call
    ens.step(2)
    ens.sync()
    for c, r in zip(ctxs, refs):
        c.step(r, 2, mixed=mixed)
        c.check()
    for q, r in zip(states, refs):
        assert torch_cuda.equal(q, r)
    assert all(float(q.abs().max()) > 0 for q in states)
    ens.close()
    for c in ctxs:
        c.close()


def test_ensemble_argument_errors(torch_cuda, numa_mod):
    g = W.Grid(30000.0, 20000.0, 8000.0, 3, 2, 4, 4)
    a, b = numa_mod.Context(g), numa_mod.Context(g)
    qa = torch_cuda.zeros(a.shape, dtype=torch_cuda.float64, device="cuda")
    qb = torch_cuda.zeros(b.shape, dtype=torch_cuda.float64, device="cuda")
    a.factor(1.0)
    with pytest.raises(numa_mod.NumaError) as ei:  # b not factored
        numa_mod.ensemble_create([a.ctx, b.ctx], [qa.data_ptr(), qb.data_ptr()], [1.0, 1.0])
    assert ei.value.code == numa_mod.NUMA_E_NOT_FACTORED
    b.factor(2.0)
    with pytest.raises(numa_mod.NumaError) as ei:  # dt differs from b's factored dt
        numa_mod.ensemble_create([a.ctx, b.ctx], [qa.data_ptr(), qb.data_ptr()], [1.0, 1.0])
    assert ei.value.code == numa_mod.NUMA_E_DT_MISMATCH
    with pytest.raises(numa_mod.NumaError) as ei:  # one state twice
        numa_mod.ensemble_create([a.ctx, b.ctx], [qa.data_ptr(), qa.data_ptr()], [1.0, 2.0])
    assert ei.value.code == numa_mod.NUMA_E_ARG
    lib = numa_mod.load()
    assert lib.numa_ensemble_destroy(None) == numa_mod.NUMA_OK
    assert lib.numa_ensemble_step(None, 1) == numa_mod.NUMA_E_ARG
    a.close()
    b.close()


def _oracle(O, g, bg):
    return O.Oracle(g.lx, g.ly, g.lz, g.nex, g.ney, g.nez, g.N, theta0=bg.theta0, p00=bg.p00, cp=bg.cp,
                    rgas=bg.rgas, grav=bg.grav, zface=g.zface)


# Relative L2 bars per variable (rho', u, v, w, theta') after up to 50 steps.
ORACLE_BARS = {False: [1e-11] * 5, True: [1e-6] * 5}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mixed", [False, True])
def test_ensemble_matches_oracle(torch_cuda, numa_mod, oracle_mod, mixed):
    """One domain per order (3, 4, 5, 7), 6..16 vertical elements, winds of
    up to 20 m/s, vertical Courant number 15: 50 steps of the captured
    ensemble graph against 50 oracle steps of each domain, compared every 10
    steps (FP64 form to 1e-11; precision form to ORACLE_BARS)."""
    bar = np.array(ORACLE_BARS[mixed])
    doms = W.ensemble_small_domains()
    ctxs, states, orcs, qos = [], [], [], []
    for wl in doms:
        g = wl.grid
        c = numa_mod.Context(g, wl.background)
        c.factor(wl.dt)
        q0 = W.make_initial_state(wl)
        ctxs.append(c)
        states.append(torch_cuda.from_numpy(q0.copy()).cuda())
        o = _oracle(oracle_mod, g, wl.background)
        o.factor_dt(wl.dt)
        orcs.append(o)
        qos.append(q0)
    ens = numa_mod.Ensemble(ctxs, states, mixed=mixed, tune=True)
    worst = np.zeros((len(doms), 5))
    for block in range(5):
        ens.step(10)
        ens.sync()
        for i, wl in enumerate(doms):
            qos[i] = orcs[i].step(qos[i], wl.dt, 10)
            qg = states[i].cpu().numpy()
            e = np.array([np.linalg.norm(qg[f] - qos[i][f]) / np.linalg.norm(qos[i][f]) for f in range(5)])
            print(f"{wl.name} {'mixed' if mixed else 'fp64'} after {10 * (block + 1)} graph steps: {e}")
            worst[i] = np.maximum(worst[i], e)
    ens.close()
    for c in ctxs:
        c.close()
    assert np.all(worst < bar), worst


@pytest.mark.parametrize("mixed", [False, True])
def test_ensemble_with_second_tiles_replays_match_eager_steps(torch_cuda, numa_mod, mixed):
    """Every domain on its second tile shape (set by hand, no autotuner):
    the captured graph's replays equal eager steps of the same contexts."""
    doms = [_domain(torch_cuda, numa_mod, *d) for d in DOMAINS]
    ctxs = [c for c, _ in doms]
    for c in ctxs:
        numa_mod.set_rhs_config(c.ctx, 1, 0)
        assert numa_mod.get_rhs_config(c.ctx)["tile"] == 1
    states = [q for _, q in doms]
    refs = [q.clone() for q in states]
    ens = numa_mod.Ensemble(ctxs, states, mixed=mixed, tune=False)
    for replay in range(2):
        ens.step(1)
        ens.sync()
        for c, r in zip(ctxs, refs):
            c.step(r, 1, mixed=mixed)
            c.check()
        for i, (q, r) in enumerate(zip(states, refs)):
            assert torch_cuda.equal(q, r), f"domain {i}, replay {replay}"
    assert [numa_mod.get_rhs_config(c.ctx)["tile"] for c in ctxs] == [1] * len(ctxs)
    ens.close()
    for c in ctxs:
        c.close()
