"""GPU parity of the learned correction of the 3D-IMEX preconditioner
(FP32 network, hand-written forward, backward and Adam kernels) against the
CPU oracle's FP64 network, element gather and flexible GMRES.

Bars: FP32 arithmetic against FP64, so features and network outputs to
1e-6 relative, gradients to 1e-4 relative (sums over a batch), targets to
1e-5 (they include a GMRES solution at tol 1e-12); flexible GMRES solves at
tol 1e-12 to 1e-9 per variable."""
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


def _oracle(O, g, bg=None):
    bg = bg or W.Background()
    return O.Oracle(g.lx, g.ly, g.lz, g.nex, g.ney, g.nez, g.N, theta0=bg.theta0, p00=bg.p00, cp=bg.cp,
                    rgas=bg.rgas, grav=bg.grav, zface=g.zface)


def _grid(N=3, nex=3, ney=2, nez=2):
    return W.Grid(625.0 * nex, 700.0 * ney, 2500.0 * nez, nex, ney, nez, N)


def _dt(g):
    return min(W.dt_for_courant(g, 15.0, "x"), W.dt_for_courant(g, 15.0, "y"), W.dt_for_courant(g, 15.0, "z"))


def _setup(numa, g, o=None, order=2, hidden=16, cap=None, seed=3):
    """Context, dt and PBNO interval: the oracle's interval (o given), set on
    the GPU solver too, so that both sides use the same polynomial."""
    ctx = numa.Context(g)
    dt = _dt(g)
    bd = ctx.imex3d_setup(dt, restart=30, pbno_order=order, power_steps=30, maxit=5000)
    if o is not None:
        bd = o.schur_bounds((1.0 - 1.0 / np.sqrt(2.0)) * dt, 30)
        numa.imex3d_set_bounds(ctx.ctx, *bd)
    nelem = g.nex * g.ney * g.nez
    numa.learned_setup(ctx.ctx, hidden=hidden, max_samples=cap or 4 * nelem, seed=seed)
    return ctx, dt, bd


def _mlp_from_theta(O, theta, nin, nh):
    th = theta.astype(np.float64)
    W1 = th[:nh * nin].reshape(nh, nin)
    b1 = th[nh * nin:nh * nin + nh]
    W2 = th[nh * nin + nh:nh * nin + nh + nin * nh].reshape(nin, nh)
    b2 = th[nh * nin + nh + nin * nh:]
    return O.Mlp(W1, b1, W2, b2)


def _dense_schur(o, lam, shape):
    n = int(np.prod(shape))
    S = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        S[:, j] = o.schur_apply(e.reshape(shape), lam).reshape(-1)
    return S


def test_samples_parity(torch_cuda, numa_mod, oracle_mod):
    g = _grid()
    o = _oracle(oracle_mod, g)
    ctx, dt, bd = _setup(numa_mod, g, o)
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * dt
    rng = np.random.default_rng(5)
    r = rng.standard_normal(g.shape[1:]) * 100.0
    numa_mod.learned_add_samples(ctx.ctx, torch_cuda.from_numpy(r).cuda().data_ptr(), 1e-12)
    info = numa_mod.learned_info(ctx.ctx)
    nelem, nin = g.nex * g.ney * g.nez, (g.N + 1) ** 3
    assert info["samples"] == nelem and info["nin"] == nin
    X = torch_cuda.empty(nelem * nin, dtype=torch_cuda.float32, device="cuda")
    T = torch_cuda.empty_like(X)
    numa_mod.learned_samples(ctx.ctx, 0, nelem, X.data_ptr(), T.data_ptr())
    Xo, so = o.element_features(r)
    assert np.max(np.abs(X.cpu().numpy().reshape(nelem, nin) - Xo)) < 1e-6 * np.max(np.abs(Xo))
    e = np.linalg.solve(_dense_schur(o, lam, g.shape[1:]), r.reshape(-1)).reshape(g.shape[1:])
    pb = o.pbno_apply(r, lam, 2, bd)
    To, _ = o.element_features(e - pb)
    # targets are scaled by the features' s_e, not by their own RMS
    _, s_e = o.element_features(r)
    _, s_t = o.element_features(e - pb)
    To = To * (s_t / s_e)[:, None]
    got = T.cpu().numpy().reshape(nelem, nin)
    assert np.max(np.abs(got - To)) < 1e-5 * np.max(np.abs(To))
    ctx.close()


def test_loss_gradient_parity(torch_cuda, numa_mod, oracle_mod):
    g = _grid(N=2)
    ctx, dt, bd = _setup(numa_mod, g, hidden=12)
    info = numa_mod.learned_info(ctx.ctx)
    nin, nh, npar = info["nin"], info["hidden"], info["nparam"]
    rng = np.random.default_rng(6)
    theta = (0.2 * rng.standard_normal(npar)).astype(np.float32)
    numa_mod.learned_params(ctx.ctx, theta_in=theta)
    back = np.zeros(npar, dtype=np.float32)
    numa_mod.learned_params(ctx.ctx, theta_out=back)
    assert np.array_equal(back, theta)
    B = 9
    X = rng.standard_normal((B, nin)).astype(np.float32)
    T = rng.standard_normal((B, nin)).astype(np.float32)
    Xd, Td = torch_cuda.from_numpy(X).cuda(), torch_cuda.from_numpy(T).cuda()
    gd = torch_cuda.empty(npar, dtype=torch_cuda.float32, device="cuda")
    loss = numa_mod.learned_loss_grad(ctx.ctx, Xd.data_ptr(), Td.data_ptr(), B, gd.data_ptr())
    m = _mlp_from_theta(oracle_mod, theta, nin, nh)
    lo, go = m.loss_grad(X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) < 1e-5 * lo
    gref = np.concatenate([a.reshape(-1) for a in go])
    assert np.linalg.norm(gd.cpu().numpy() - gref) < 1e-4 * np.linalg.norm(gref)
    ctx.close()


def test_learned_apply_parity(torch_cuda, numa_mod, oracle_mod):
    g = _grid(N=3, nex=1, ney=3, nez=2)  # a single element along x: the node gather wraps onto itself
    o = _oracle(oracle_mod, g)
    ctx, dt, bd = _setup(numa_mod, g, o, order=1, hidden=10)
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * dt
    info = numa_mod.learned_info(ctx.ctx)
    theta = np.zeros(info["nparam"], dtype=np.float32)
    numa_mod.learned_params(ctx.ctx, theta_out=theta)
    theta[-info["nin"]:] = 0.3  # nonzero b2 as well
    numa_mod.learned_params(ctx.ctx, theta_in=theta)
    m = _mlp_from_theta(oracle_mod, theta, info["nin"], info["hidden"])
    r = np.random.default_rng(7).standard_normal(g.shape[1:])
    z = torch_cuda.empty(g.shape[1:], dtype=torch_cuda.float64, device="cuda")
    numa_mod.learned_apply(ctx.ctx, torch_cuda.from_numpy(r).cuda().data_ptr(), z.data_ptr())
    zo = o.learned_apply(r, lam, 1, bd, m)
    corr = o.mlp_correction(m, r)
    assert np.max(np.abs(z.cpu().numpy() - zo)) < 1e-5 * np.max(np.abs(corr))
    ctx.close()


def test_training_and_flexible_solve(torch_cuda, numa_mod, oracle_mod):
    """Train on the solver's own pairs (Schur right-hand sides of stage-like
    states and seeded random fields, the residuals GMRES meets): the loss
    falls; the flexible solve with the network matches the oracle's flexible
    solve with the same weights (fallback rule included); switching the
    network off restores the polynomial path.  The iteration counts with and
    without the network are what the network gains (printed)."""
    wl = W.box_imex3d("small")
    g = wl.grid
    o = _oracle(oracle_mod, g)
    ne = g.nex * g.ney * g.nez
    ctx = numa_mod.Context(g)
    ctx.imex3d_setup(wl.dt, restart=30, pbno_order=2, power_steps=30, maxit=5000)
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * wl.dt
    bd = o.schur_bounds(lam, 30)
    numa_mod.imex3d_set_bounds(ctx.ctx, *bd)
    nfields = 72
    numa_mod.learned_setup(ctx.ctx, hidden=16, max_samples=nfields * ne, seed=3)
    q0 = W.make_initial_state(wl)
    R = o.rhs(q0)
    fields = [o.schur_rhs(q0 + (0.3 + 0.2 * k) * wl.dt * R, lam) for k in range(8)]
    rng = np.random.default_rng(11)
    fields += [rng.standard_normal(g.shape[1:]) for _ in range(nfields - 8)]
    for f in fields:
        numa_mod.learned_add_samples(ctx.ctx, torch_cuda.from_numpy(f).cuda().data_ptr(), 1e-10)
    lf, ll = numa_mod.learned_train(ctx.ctx, 2000, batch=128, lr=1e-3)
    assert ll < 0.7 * lf, (lf, ll)
    info = numa_mod.learned_info(ctx.ctx)
    theta = np.zeros(info["nparam"], dtype=np.float32)
    numa_mod.learned_params(ctx.ctx, theta_out=theta)
    m = _mlp_from_theta(oracle_mod, theta, info["nin"], info["hidden"])
    y = q0 + 0.5 * wl.dt * R
    yd = torch_cuda.from_numpy(y).cuda()
    numa_mod.learned_enable(ctx.ctx, True)
    x_net, it_net = ctx.imex3d_solve(yd, 1e-10)
    xo, ito = o.solve3d_learned(y, lam, m, tol=1e-10, order=2, bounds=bd)
    xn = x_net.cpu().numpy()
    for f in range(5):
        assert np.linalg.norm(xn[f] - xo[f]) <= 1e-7 * np.linalg.norm(xo[f]) + 1e-300, f
    assert abs(it_net - ito) <= max(3, 0.15 * ito), (it_net, ito)
    numa_mod.learned_enable(ctx.ctx, False)
    x_pb, it_pb = ctx.imex3d_solve(yd, 1e-10)
    xp, itp = o.solve3d(y, lam, tol=1e-10, order=2, bounds=bd)
    assert abs(it_pb - itp) <= 1
    print(f"\nGMRES iterations to 1e-10: PBNO(2) {it_pb}, PBNO(2) + network {it_net} (oracle {ito})")
    # PBNO judges the trained network on the same system, as the oracle does
    xj = torch_cuda.empty_like(yd)
    jd = numa_mod.learned_judge(ctx.ctx, yd.data_ptr(), xj.data_ptr(), 1e-10)
    po, qo, acc_o = o.learned_judge(y, lam, m, tol=1e-10, order=2, bounds=bd)
    print(f"judge: {jd} (oracle {po}, {qo}, {acc_o})")
    assert jd["pbno_iters"] == it_pb and jd["net_iters"] == it_net
    assert jd["accepted"] == (it_net < it_pb)
    if abs(qo - po) > 3:
        assert jd["accepted"] == acc_o
    assert numa_mod.learned_info(ctx.ctx)["enabled"] == int(jd["accepted"])
    assert np.linalg.norm(xj.cpu().numpy() - x_pb.cpu().numpy()) <= 1e-12 * np.linalg.norm(x_pb.cpu().numpy())
    # what the judged configuration then costs: at most PBNO's iterations
    # (the network kept only where it took fewer)
    _, it_after = ctx.imex3d_solve(yd, 1e-10)
    assert it_after <= it_pb, (it_after, it_pb)
    ctx.close()


def _diagonal_mlp(O, o, g, lam, scale, eps=1e-3):
    """A network in its linear regime (tanh(eps t) = eps t to 1e-7) whose
    output is D x, D the mean over the elements of 1/diag(S) at each local
    node: a Jacobi-like correction added to the polynomial."""
    shape = g.shape[1:]
    n = int(np.prod(shape))
    diag = np.empty(n)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        diag[j] = o.schur_apply(e.reshape(shape), lam).reshape(-1)[j]
    diag = diag.reshape(shape)
    nq = g.N + 1
    nin = nq ** 3
    acc = np.zeros(nin)
    for ez in range(g.nez):
        for ey in range(g.ney):
            for ex in range(g.nex):
                for c in range(nq):
                    for b in range(nq):
                        for a in range(nq):
                            k, j, i = ez * g.N + c, (ey * g.N + b) % shape[1], (ex * g.N + a) % shape[2]
                            acc[a + nq * (b + nq * c)] += 1.0 / diag[k, j, i]
    d = scale * acc / (g.nex * g.ney * g.nez)
    return O.Mlp(eps * np.eye(nin), np.zeros(nin), np.diag(d) / eps, np.zeros(nin))


def _theta_of(m):
    return np.concatenate([m.W1.reshape(-1), m.b1, m.W2.reshape(-1), m.b2]).astype(np.float32)


@pytest.mark.parametrize("kind", ["diagonal", "zero", "random"])
def test_judge_matches_oracle(torch_cuda, numa_mod, oracle_mod, kind):
    """PBNO as the judge: the GPU's decision and both iteration counts agree
    with the oracle's judge on the same weights.  A diagonal correction
    (mean 1/diag(S) per local node) takes fewer iterations than PBNO(2) and
    is accepted; a zero network ties and large random weights lose: both are
    rejected and the solver is back on the polynomial alone."""
    g = W.Grid(3000.0, 2500.0, 2000.0, 2, 2, 2, 3)
    o = _oracle(oracle_mod, g)
    nin = (g.N + 1) ** 3
    ctx = numa_mod.Context(g)
    dt = W.dt_for_courant(g, 15.0, "x")
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * dt
    ctx.imex3d_setup(dt, restart=30, pbno_order=2, power_steps=30, maxit=5000)
    bd = o.schur_bounds(lam, 30)
    numa_mod.imex3d_set_bounds(ctx.ctx, *bd)
    numa_mod.learned_setup(ctx.ctx, hidden=nin, max_samples=8, seed=1)
    if kind == "diagonal":
        m = _diagonal_mlp(oracle_mod, o, g, lam, 0.5)
    elif kind == "zero":
        m = oracle_mod.Mlp(np.zeros((nin, nin)), np.zeros(nin), np.zeros((nin, nin)), np.zeros(nin))
    else:
        rng = np.random.default_rng(5)
        m = oracle_mod.Mlp(30.0 * rng.standard_normal((nin, nin)), 30.0 * rng.standard_normal(nin),
                           30.0 * rng.standard_normal((nin, nin)), 30.0 * rng.standard_normal(nin))
    theta = _theta_of(m)
    numa_mod.learned_params(ctx.ctx, theta_in=theta)
    m = _mlp_from_theta(oracle_mod, theta, nin, nin)  # the FP32 weights the GPU runs
    y = W.make_random_state(g, 3, smooth=False)
    yd = torch_cuda.from_numpy(y).cuda()
    x = torch_cuda.empty_like(yd)
    jd = numa_mod.learned_judge(ctx.ctx, yd.data_ptr(), x.data_ptr(), 1e-10)
    po, qo, acc_o = o.learned_judge(y, lam, m, tol=1e-10, order=2, bounds=bd)
    print(f"{kind}: GPU {jd}, oracle ({po}, {qo}, {acc_o})")
    assert abs(jd["pbno_iters"] - po) <= 1
    assert abs(jd["net_iters"] - qo) <= max(3, 0.15 * qo)
    assert jd["accepted"] == acc_o == (kind == "diagonal")
    assert numa_mod.learned_info(ctx.ctx)["enabled"] == int(acc_o)
    xo, _ = o.solve3d(y, lam, tol=1e-10, order=2, bounds=bd)
    xh = x.cpu().numpy()
    for f in range(5):
        assert np.linalg.norm(xh[f] - xo[f]) <= 1e-7 * np.linalg.norm(xo[f]) + 1e-300, f
    _, it_after = ctx.imex3d_solve(yd, 1e-10)
    assert it_after <= jd["pbno_iters"] + 1, (it_after, jd)
    ctx.close()


@pytest.mark.parametrize("kind", ["diagonal", "random"])
def test_judge_with_fp32_polynomial(torch_cuda, numa_mod, oracle_mod, kind):
    """The judge and the network on top of the FP32 polynomial (flexible
    GMRES either way): the decision and both iteration counts agree with the
    oracle's FP64 judge within two iterations, and the accepted network's
    solution meets the solve bar."""
    g = W.Grid(3000.0, 2500.0, 2000.0, 2, 2, 2, 3)
    o = _oracle(oracle_mod, g)
    nin = (g.N + 1) ** 3
    ctx = numa_mod.Context(g)
    dt = W.dt_for_courant(g, 15.0, "x")
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * dt
    ctx.imex3d_setup(dt, restart=30, pbno_order=2, power_steps=30, maxit=5000)
    bd = o.schur_bounds(lam, 30)
    numa_mod.imex3d_set_bounds(ctx.ctx, *bd)
    numa_mod.imex3d_set_precision(ctx.ctx, True)
    numa_mod.learned_setup(ctx.ctx, hidden=nin, max_samples=8, seed=1)
    if kind == "diagonal":
        m = _diagonal_mlp(oracle_mod, o, g, lam, 0.5)
    else:
        rng = np.random.default_rng(5)
        m = oracle_mod.Mlp(30.0 * rng.standard_normal((nin, nin)), 30.0 * rng.standard_normal(nin),
                           30.0 * rng.standard_normal((nin, nin)), 30.0 * rng.standard_normal(nin))
    theta = _theta_of(m)
    numa_mod.learned_params(ctx.ctx, theta_in=theta)
    m = _mlp_from_theta(oracle_mod, theta, nin, nin)
    y = W.make_random_state(g, 3, smooth=False)
    yd = torch_cuda.from_numpy(y).cuda()
    x = torch_cuda.empty_like(yd)
    jd = numa_mod.learned_judge(ctx.ctx, yd.data_ptr(), x.data_ptr(), 1e-10)
    po, qo, acc_o = o.learned_judge(y, lam, m, tol=1e-10, order=2, bounds=bd)
    print(f"{kind} over the FP32 polynomial: GPU {jd}, oracle FP64 ({po}, {qo}, {acc_o})")
    assert abs(jd["pbno_iters"] - po) <= 2 and abs(jd["net_iters"] - qo) <= max(3, 0.15 * qo)
    assert jd["accepted"] == acc_o == (kind == "diagonal")
    xn, _ = ctx.imex3d_solve(yd, 1e-10)
    xo, _ = o.solve3d(y, lam, tol=1e-10, order=2, bounds=bd)
    xh = xn.cpu().numpy()
    for f in range(5):
        assert np.linalg.norm(xh[f] - xo[f]) <= 1e-7 * np.linalg.norm(xo[f]) + 1e-300, f
    ctx.close()


def test_fallback_keeps_a_bad_network_harmless(torch_cuda, numa_mod, oracle_mod):
    """Large random weights: the first flexible cycle fails to reduce the
    residual tenfold, the network is switched off and the solve converges."""
    g = _grid(N=3, nex=3, ney=3, nez=2)
    o = _oracle(oracle_mod, g)
    ctx, dt, bd = _setup(numa_mod, g, o, order=2, hidden=8)
    lam = (1.0 - 1.0 / np.sqrt(2.0)) * dt
    info = numa_mod.learned_info(ctx.ctx)
    theta = (3.0 * np.random.default_rng(9).standard_normal(info["nparam"])).astype(np.float32)
    numa_mod.learned_params(ctx.ctx, theta_in=theta)
    numa_mod.learned_enable(ctx.ctx, True)
    y = W.make_random_state(g, 4, smooth=False)
    x, it = ctx.imex3d_solve(torch_cuda.from_numpy(y).cuda(), 1e-10)
    m = _mlp_from_theta(oracle_mod, theta, info["nin"], info["hidden"])
    xo, ito = o.solve3d_learned(y, lam, m, tol=1e-10, order=2, bounds=bd)
    res = x.cpu().numpy() - lam * o.lfull(x.cpu().numpy()) - y
    assert np.linalg.norm(res) < 1e-7 * np.linalg.norm(y)
    assert abs(it - ito) <= max(3, 0.15 * ito), (it, ito)
    ctx.close()
