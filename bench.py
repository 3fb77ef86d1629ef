"""Benchmark of the HEVI (1D-IMEX) ARK2 step on one MI355X.

Workload: 64 x 64 x 10 hexahedral elements at LGL order 4 (256 x 256 x 41 =
2,686,976 unique nodes, 65,536 columns of 41 levels), x and y periodic,
vertical Courant number 15 with the horizontal extent stretched to a
horizontal Courant number of 0.4 (2400 x 2400 x 10 km), FP64, eight seeded
potential-temperature bumps in hydrostatic pressure balance.

Prints ONE JSON line.  value = DOF-steps/s = 5 * unique nodes * steps / s,
with the state already resident in HBM, timed by the wall clock over exactly
`steps` steps bracketed by device synchronisation.  A second run of as many
steps records a HIP event around every kernel on the library's stream; the
roofline object uses the average duration of the dominant kernel there and
its algorithmic bytes.  The
right-hand sides' tile shape and vertical chunk come from the library's
autotuner, run before the warm-up steps.  The CPU baseline times the plain
FP64 oracle on the same workload for a few steps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(np_, ncol, nz, N, table_bytes=None, r1=8):
    """Algorithmic HBM bytes per launch of the five kernels of a step: whole
    unique-node field passes (reads + writes) and the column factor reads
    (one LU band shared by all columns).  r1: bytes per value of the
    first-stage tendency R1 (8; 4 in the precision form), every other field
    FP64."""
    F = nz * (4 * N + 1) * 8 if table_bytes is None else table_bytes
    f, r = 8 * np_, r1 * np_
    return [
        ("rhs_stage1", 5 * f + 5 * r),          # reads q^n (5), writes R1 (5)
        ("colsolve_stage2", 4 * f + 3 * r + F), # reads R1 rho/w/theta, q^n rho/w; writes Q2 rho/w; factors
        ("rhs_stage2", 17 * f + 5 * r),         # reads Q2 rho/w, q^n (5), R1 (5); writes E3 (5), ACC (5)
        ("colsolve_stage3", 10 * f + r + F),    # reads E3, q^n (rho/w/theta), Q2 rho/w, R1 theta; writes Q3 rho/w; factors
        ("rhs_stage3", 15 * f),                 # reads Q3 rho/w, E3 u/v/theta, ACC (5); writes q^{n+1} (5)
    ]


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1702_04316_amd", "csrc", f)
                  for f in ("kernels.hip", "rhs_kernel.h", "rhs_alt.hip", "numa_internal.h")]


def kernel_source_hash():
    """SHA-256 over the sources of the step's kernels, in a fixed order."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic():
    """Measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy calibration) from the committed rocprofv3 counter summary; None if
    there is none or the kernels changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernels_sha256") != kernel_source_hash():
        return None
    return t


def wall_and_kernels(numa, torch, ctx, q, dt, steps, mixed=False, prof_steps=None):
    """Wall-clock seconds per step over `steps` plain steps bracketed by
    device synchronisation, then the per-kernel milliseconds (HIP events on
    the library's stream) of a separate profiled run of prof_steps steps, so
    that creating the events stays out of the wall clock."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(q, steps, mixed=mixed)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    prof = numa.profile_steps_mixed if mixed else numa.profile_steps
    ms = prof(ctx.ctx, q.data_ptr(), dt, prof_steps or steps)
    torch.cuda.synchronize()
    return t, ms


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(steps=5, single_steps=1):
    """The plain FP64 oracle on the benchmarked workload itself (64x64x10,
    N=4, R1): factorisation untimed, then `steps` steps with every host
    thread and `single_steps` with one thread, timed."""
    from oracle import oracle as O
    from paper_1702_04316_amd import workloads as W
    wl = W.box_large("R1")
    g = wl.grid
    o = O.Oracle(g.lx, g.ly, g.lz, g.nex, g.ney, g.nez, g.N)
    q0 = W.make_initial_state(wl)
    o.factor_dt(wl.dt)
    threads = O.get_threads()
    t0 = time.perf_counter()
    q = o.step(q0, wl.dt, steps)
    t = time.perf_counter() - t0
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        o.step(q, wl.dt, single_steps)
        t1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    return {"value": 5.0 * g.n_unique * steps / t, "unit": "DOF-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"the benchmarked workload itself (64x64x10 elements, N=4, 256x256x41 unique nodes), "
                       f"{steps} steps on {threads} threads, factorisation not timed"),
            "seconds": t, "cpu_model": cpu_model(),
            "single_thread": {"value": 5.0 * g.n_unique * single_steps / t1, "steps": single_steps,
                              "seconds": t1}}


def precision_form(numa, torch, ctx, wl, args, t_fp64):
    """The precision form (the first-stage tendency R1 stored in FP32) on
    the same workload and GPU: throughput, simulated seconds per wall second
    against the FP64 step, its algorithmic bytes, and its relative L2
    difference per variable from the FP64 step after 100 steps (the FP64
    step matches the oracle to 1e-11; the tests check the form against the
    oracle itself)."""
    import numpy as np
    from paper_1702_04316_amd import workloads as W
    g = wl.grid
    q0 = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
    q = q0.clone()
    ctx.step(q, args.warmup, mixed=True)
    ctx.check()
    tm, ms = wall_and_kernels(numa, torch, ctx, q, wl.dt, args.steps, mixed=True)
    tm *= args.steps
    ctx.check()
    a, b = q0.clone(), q0.clone()
    ctx.step(a, 100)
    ctx.step(b, 100, mixed=True)
    ctx.check()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    err = {n: float(np.linalg.norm(b[f] - a[f]) / np.linalg.norm(a[f]))
           for f, n in enumerate(("rho'", "u", "v", "w", "theta'"))}
    info = ctx.info()
    kb = kernel_bytes(g.n_unique, info["ncol"], info["nz"], g.N, info["factor_bytes"], r1=4)
    step_bytes = sum(b for _, b in kb)
    names = [n for n, _ in kb]
    return {
        "entry": "numa_hevi_step_mixed",
        "algorithmic_bytes_per_step": step_bytes,
        "step_algorithmic_GBps": step_bytes * args.steps / tm / 1e9,
        "value": 5 * g.n_unique * args.steps / tm,
        "unit": "DOF-steps/s",
        "ms_per_step": 1e3 * tm / args.steps,
        "speedup_vs_fp64": t_fp64 / tm,
        "sim_s_per_wall_s": {"fp64": wl.dt * args.steps / t_fp64, "mixed": wl.dt * args.steps / tm},
        "rel_l2_vs_fp64_after_100_steps": err,
        "kernels": [{"kernel": n, "ms": m, "GB/s": bb / (m * 1e6)} for (n, bb), m in zip(kb, ms)],
    }


def precision_form_n7(numa, torch, steps=20, err_steps=100):
    """The precision-form workload at N=7: 28x28x28 elements of a stretched
    1 km cube (196x196x197 = 7,567,952 unique nodes), vertical Courant
    number 15.  FP64 and precision-form steps on the same GPU (per-kernel
    HIP events), simulated seconds per wall second of each, and the
    relative L2 difference per variable after err_steps steps (the FP64 step
    equals the oracle to 1e-11; the tests check the precision form against
    the oracle at N=7 on 4x4x4 elements)."""
    import numpy as np
    from paper_1702_04316_amd import workloads as W
    wl = W.box_precision("large")
    g = wl.grid
    ctx = numa.Context(g, wl.background)
    ctx.factor(wl.dt)
    q0 = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
    names = ["rhs_stage1", "colsolve_stage2", "rhs_stage2", "colsolve_stage3", "rhs_stage3"]
    out = {"workload": f"{wl.name}: 28x28x28 elements, LGL N=7, {g.nx}x{g.ny}x{g.nz} unique nodes, "
                       "vertical Courant 15", "unique_nodes": g.n_unique, "dt_s": wl.dt,
           "rhs_config": numa.autotune(ctx.ctx, q0.data_ptr(), reps=3)}
    for name, mixed in (("fp64", False), ("mixed", True)):
        q = q0.clone()
        ctx.step(q, 3, mixed=mixed)
        ctx.check()
        t, ms = wall_and_kernels(numa, torch, ctx, q, wl.dt, steps, mixed=mixed)
        ctx.check()
        out[name] = {"ms_per_step": 1e3 * t, "value": 5 * g.n_unique / t, "sim_s_per_wall_s": wl.dt / t,
                     "kernels": [{"kernel": n, "ms": m} for n, m in zip(names, ms)]}
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    a, b = q0.clone(), q0.clone()
    ctx.step(a, err_steps)
    ctx.step(b, err_steps, mixed=True)
    ctx.check()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    out["rel_l2_vs_fp64_after_%d_steps" % err_steps] = {
        n: float(np.linalg.norm(b[f] - a[f]) / np.linalg.norm(a[f]))
        for f, n in enumerate(("rho'", "u", "v", "w", "theta'"))}
    out["unit"] = "DOF-steps/s"
    ctx.close()
    return out


def step_leg(numa, torch, wl, solver=None, steps=20, tune=True):
    """FP64 steps of workload wl on its own context (optionally with a
    column-solver kind), after the autotuner: ms per step, per-kernel
    milliseconds (HIP events, launch order) and the step's algorithmic bytes
    and GB/s (the library's byte model, numa_get_info)."""
    from paper_1702_04316_amd import workloads as W
    ctx = numa.Context(wl.grid, wl.background)
    if solver is not None:
        ctx.set_column_solver(solver)
    t0 = time.perf_counter()
    ctx.factor(wl.dt)
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    q = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
    cfg = numa.autotune(ctx.ctx, q.data_ptr(), reps=5) if tune else numa.get_rhs_config(ctx.ctx)
    ctx.step(q, 3)
    ctx.check()
    t, ms = wall_and_kernels(numa, torch, ctx, q, wl.dt, steps)
    ctx.check()
    info = ctx.info()
    ctx.close()
    names = ["rhs_stage1", "colsolve_stage2", "rhs_stage2", "colsolve_stage3", "rhs_stage3"]
    gbs = info["step_bytes"] / t / 1e9
    return {"ms_per_step": 1e3 * t, "value": 5 * wl.grid.n_unique / t, "unit": "DOF-steps/s",
            "factor_s": t_factor, "factor_bytes": info["factor_bytes"], "step_bytes": info["step_bytes"],
            "step_GBps": gbs, "step_frac_of_8TBps": gbs / HBM_PEAK_GBS, "rhs_config": cfg,
            "kernels": [{"kernel": n, "ms": m} for n, m in zip(names, ms)]}


def per_column_factors(numa, torch, steps=20):
    """The benchmarked workload with every column's own factors
    (NUMA_SOLVER_PER_COLUMN, 365 MB read twice per step): the byte model of
    65 field passes plus 2F, F = 41 x 17 x 65,536 doubles."""
    from paper_1702_04316_amd import workloads as W
    out = step_leg(numa, torch, W.box_large("R1"), solver=numa.SOLVER_PER_COLUMN, steps=steps)
    out["entry"] = "numa_set_column_solver(NUMA_SOLVER_PER_COLUMN)"
    return out


def stratified_leg(numa, torch, steps=20):
    """The benchmarked grid over the stratified background (Nb = 0.01/s):
    the solves also write theta' (71 field passes)."""
    from paper_1702_04316_amd import workloads as W
    out = step_leg(numa, torch, W.box_stratified("large"), steps=steps)
    out["workload"] = ("box64x64x10_N4_strat: the 64x64x10, N=4 grid over theta0(z) = 300 K exp(Nb^2 z/g), "
                       "Nb = 0.01/s")
    return out


def standard_form_columns(numa, torch, ctx, wl, q, reps=20):
    """The column solve in its standard (rho', w) form against the Schur
    form on the benchmark grid: factor bytes, milliseconds per solve (HIP
    events around `reps` solves of the same right-hand side) and the
    relative L2 difference of the two solutions per variable."""
    import numpy as np
    y = q.clone()
    xs, xk = torch.empty_like(y), torch.empty_like(y)
    t0 = time.perf_counter()
    nbytes = numa.factor_columns_standard(ctx.ctx, wl.dt)
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_std = timed(lambda: numa.solve_columns_standard(ctx.ctx, y.data_ptr(), xs.data_ptr()))
    ms_schur = timed(lambda: numa.solve_columns(ctx.ctx, y.data_ptr(), xk.data_ptr()))
    ctx.check()
    a, b = xs.cpu().numpy(), xk.cpu().numpy()
    diff = {n: float(np.linalg.norm(a[f] - b[f]) / np.linalg.norm(b[f])) for f, n in ((0, "rho'"), (3, "w"))}
    info = ctx.info()
    # the Schur form with one lane per column, on a context of its own
    cb = numa.Context(wl.grid, wl.background)
    cb.set_column_solver(numa.SOLVER_BAND)
    cb.factor(wl.dt)
    ms_band = timed(lambda: numa.solve_columns(cb.ctx, y.data_ptr(), xk.data_ptr()))
    cb.check()
    band_bytes = cb.info()["factor_bytes"]
    cb.close()
    return {"entry": "numa_solve_columns_standard", "factor_bytes": nbytes,
            "schur_solver": "blocked" if info["column_solver"] == numa.SOLVER_BLOCKED else "band",
            "schur_factor_bytes": info["factor_bytes"], "factor_s": t_factor, "ms_per_solve": ms_std,
            "schur_ms_per_solve": ms_schur, "schur_speedup": ms_std / ms_schur, "rel_l2_vs_schur": diff,
            "schur_band_ms_per_solve": ms_band, "schur_band_factor_bytes": band_bytes}


def column_solver_ab(numa, torch, wl, q0, steps=50):
    """The HEVI step with the one-lane-per-column solve instead of the
    default: per-kernel milliseconds (HIP events, launch order) and ms per
    step, on its own context and a copy of the state."""
    c = numa.Context(wl.grid, wl.background)
    c.set_column_solver(numa.SOLVER_BAND)
    c.factor(wl.dt)
    q = q0.clone()
    c.step(q, 5)
    t, ms = wall_and_kernels(numa, torch, c, q, wl.dt, steps)
    c.check()
    c.close()
    return {"solver": "band", "ms_per_step": 1e3 * t, "kernels_ms": ms}


def batched_ensemble(numa, torch, steps=50):
    """Sixteen seeded domains of different sizes and orders (3..7), stepped
    (a) one after another with the eager FP64 step (the baseline), (b)
    together through the captured ensemble graph with tuned vertical
    chunks, FP64, and (c) the same in the precision form.  Aggregate
    DOF-steps/s over all domains; inputs resident in HBM."""
    from paper_1702_04316_amd import workloads as W
    doms = W.ensemble_domains()
    ctxs, q0 = [], []
    for wl in doms:
        c = numa.Context(wl.grid, wl.background)
        c.factor(wl.dt)
        ctxs.append(c)
        q0.append(torch.from_numpy(W.make_initial_state(wl)).to("cuda"))
    dof = sum(5 * wl.grid.n_unique for wl in doms)

    def timed(run):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    qs = [q.clone() for q in q0]
    for c, q in zip(ctxs, qs):
        c.step(q, 2)
    t_seq = timed(lambda: [c.step(q, steps) for c, q in zip(ctxs, qs)])
    for c in ctxs:
        c.check()
    out = {"domains": len(doms), "steps": steps, "dof_per_step": dof,
           "orders": sorted({wl.grid.N for wl in doms}),
           "unique_nodes_range": [min(wl.grid.n_unique for wl in doms), max(wl.grid.n_unique for wl in doms)],
           "sequential_fp64": {"value": dof * steps / t_seq, "ms_per_step": 1e3 * t_seq / steps}}
    for name, mixed in (("ensemble_fp64", False), ("ensemble_mixed", True)):
        qs = [q.clone() for q in q0]
        ens = numa.Ensemble(ctxs, qs, mixed=mixed, tune=True)
        ens.step(2)
        ens.sync()
        t = timed(lambda: ens.step(steps))
        ens.sync()
        out[name] = {"value": dof * steps / t, "ms_per_step": 1e3 * t / steps, "speedup_vs_sequential": t_seq / t}
        out["tuned_zchunks"] = ens.zchunks()
        out["tuned_tiles"] = [numa.get_rhs_config(c.ctx)["tile"] for c in ctxs]
        ens.close()
        if mixed:
            out[name]["rel_l2_vs_fp64_after_%d_steps" % (steps + 2)] = ensemble_rel_l2(torch, qs, fp64_states)
        else:
            fp64_states = [q.clone() for q in qs]
    out["unit"] = "DOF-steps/s"
    for c in ctxs:
        c.close()
    return out


def ensemble_rel_l2(torch, qs, refs):
    """Largest relative L2 difference per variable over the domains."""
    worst = [0.0] * 5
    for q, r in zip(qs, refs):
        for f in range(5):
            d = float(torch.linalg.vector_norm(q[f] - r[f]) / torch.linalg.vector_norm(r[f]))
            worst[f] = max(worst[f], d)
    return dict(zip(("rho'", "u", "v", "w", "theta'"), worst))


def imex3d(numa, torch, steps=10, order=6, restart=30, learned=True):
    """The 3D-IMEX step (all acoustics implicit, Schur-complement GMRES with
    PBNO) on 32x32x8 elements, N=5, at acoustic Courant number 15 in every
    direction, tol 1e-8: throughput, simulated seconds per wall second,
    GMRES iterations per step, the same with the FP32 polynomial (flexible
    GMRES), with PBNO order 1 and without a preconditioner, and the Schur
    operator kernel against the HBM roofline
    (HIP events on the context's stream around 50 launches)."""
    from paper_1702_04316_amd import workloads as W
    wl = W.box_imex3d("full")
    g = wl.grid
    ctx = numa.Context(g, wl.background)
    q0 = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
    out = {"entry": "numa_imex3d_step", "workload": f"{wl.name}: 32x32x8 elements, LGL N=5, "
           f"{g.nx}x{g.ny}x{g.nz} unique nodes, acoustic Courant 15 on the finest spacing, tol {W.IMEX3D_TOL}",
           "dt_s": wl.dt, "unique_nodes": g.n_unique}
    runs = {}
    for name, p, n, f32 in (("pbno%d" % order, order, steps, False), ("pbno%d_fp32" % order, order, steps, True),
                            ("pbno1", 1, 3, False), ("none", -1, 3, False)):
        t0 = time.perf_counter()
        bd = ctx.imex3d_setup(wl.dt, restart=restart, pbno_order=p, power_steps=30, maxit=5000)
        numa.imex3d_set_precision(ctx.ctx, f32)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        q = q0.clone()
        ctx.imex3d_step(q, W.IMEX3D_TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = [ctx.imex3d_step(q, W.IMEX3D_TOL) for _ in range(n)]
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n
        ctx.check()
        runs[name] = {"pbno_order": p, "pbno_fp32": f32, "restart": restart, "ms_per_step": 1e3 * t,
                      "value": 5 * g.n_unique / t, "sim_s_per_wall_s": wl.dt / t,
                      "gmres_iters_per_step": sum(its) / n, "setup_s": t_setup, "interval": list(bd)}
    if learned:
        runs["pbno%d_learned" % order] = imex3d_learned(numa, torch, ctx, wl, q0, order, restart, runs)
    out["runs"] = runs
    best = runs["pbno%d" % order]
    out.update({"value": best["value"], "unit": "DOF-steps/s", "ms_per_step": best["ms_per_step"],
                "sim_s_per_wall_s": best["sim_s_per_wall_s"],
                "pbno_speedup_vs_none": runs["none"]["ms_per_step"] / best["ms_per_step"],
                "fp32_pbno_speedup": best["ms_per_step"] / runs["pbno%d_fp32" % order]["ms_per_step"]})
    return imex3d_roofline(numa, torch, ctx, g, out)


def imex3d_learned(numa, torch, ctx, wl, q0, order, restart, runs):
    """The learned correction: trained on 3 fields' element patches (24,576
    samples: one Schur right-hand side of a stage-like state, two seeded
    random fields), judged by PBNO on a stage-like system (kept only if it
    needs fewer GMRES iterations), then the same steps with the judged
    configuration."""
    from paper_1702_04316_amd import workloads as W
    g = wl.grid
    ctx.imex3d_setup(wl.dt, restart=restart, pbno_order=order, power_steps=30, maxit=5000)
    ne = g.nex * g.ney * g.nez
    t0 = time.perf_counter()
    numa.learned_setup(ctx.ctx, hidden=16, max_samples=3 * ne, seed=1)
    R1 = ctx.rhs(q0)
    lam = (1.0 - 1.0 / 2 ** 0.5) * wl.dt
    fields = [ctx.schur_rhs(q0 + 0.5 * wl.dt * R1)]
    gen = torch.Generator(device="cuda").manual_seed(11)
    fields += [torch.randn(g.shape[1:], dtype=torch.float64, device="cuda", generator=gen) for _ in range(2)]
    sample_iters = [numa.learned_add_samples(ctx.ctx, f.data_ptr(), 1e-10) for f in fields]
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    nin = (g.N + 1) ** 3
    nparam = numa.learned_info(ctx.ctx)["nparam"]
    Xs = torch.empty(3 * ne * nin, dtype=torch.float32, device="cuda")
    Ts = torch.empty_like(Xs)
    gr = torch.empty(nparam, dtype=torch.float32, device="cuda")
    numa.learned_samples(ctx.ctx, 0, 3 * ne, Xs.data_ptr(), Ts.data_ptr())
    loss_before = numa.learned_loss_grad(ctx.ctx, Xs.data_ptr(), Ts.data_ptr(), 3 * ne, gr.data_ptr())
    t0 = time.perf_counter()
    lf, ll = numa.learned_train(ctx.ctx, 2000, batch=1024, lr=1e-3)
    t_train = time.perf_counter() - t0
    loss_after = numa.learned_loss_grad(ctx.ctx, Xs.data_ptr(), Ts.data_ptr(), 3 * ne, gr.data_ptr())
    del Xs, Ts, gr
    # PBNO judges the network on a stage-like system; the steps below run
    # with it only if it was accepted
    y = q0 + 0.5 * wl.dt * R1
    xj = torch.empty_like(y)
    t0 = time.perf_counter()
    judge = numa.learned_judge(ctx.ctx, y.data_ptr(), xj.data_ptr(), W.IMEX3D_TOL)
    judge["s"] = time.perf_counter() - t0
    del xj
    q = q0.clone()
    ctx.imex3d_step(q, W.IMEX3D_TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = [ctx.imex3d_step(q, W.IMEX3D_TOL) for _ in range(3)]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / 3
    ctx.check()
    numa.learned_enable(ctx.ctx, False)
    return {
        "pbno_order": order, "restart": restart, "ms_per_step": 1e3 * t, "value": 5 * g.n_unique / t,
        "sim_s_per_wall_s": wl.dt / t, "gmres_iters_per_step": sum(its) / 3,
        "network": "per-element perceptron %d-16-%d, tanh, FP32" % ((g.N + 1) ** 3, (g.N + 1) ** 3),
        "samples": 3 * ne, "sample_solve_iters": sample_iters, "sample_s": t_samples,
        "train_steps": 2000, "batch": 1024, "train_s": t_train, "loss_all_samples_before": loss_before,
        "loss_all_samples_after": loss_after, "judge": judge,
        "network_in_timed_steps": judge["accepted"],
        "gain_vs_polynomial": runs["pbno%d" % order]["ms_per_step"] / (1e3 * t)}


def imex3d_roofline(numa, torch, ctx, g, out):
    # Schur operator: 16 algorithmic bytes per node (read P, write S P)
    P = torch.randn(g.shape[1:], dtype=torch.float64, device="cuda")
    ctx.schur_apply(P)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(50):
        ctx.schur_apply(P)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 50
    achieved = 16 * g.n_unique / (ms * 1e-3) / 1e9
    traffic = None
    try:  # counter-measured bytes of the same kernel source, if profiled
        t = json.load(open(os.path.join(ROOT, "profiles", "traffic_imex3d.json")))
        src = os.path.join(ROOT, "paper_1702_04316_amd", "csrc", "imex3d.hip")
        if t.get("kernels_sha256") == hashlib.sha256(open(src, "rb").read()).hexdigest():
            traffic = t["bytes_per_launch"]["k_schur_apply"]
    except (OSError, ValueError, KeyError):
        traffic = None
    out["roofline"] = {"bound": "hbm", "kernel": "k_schur_apply", "achieved": achieved, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                       "algorithmic_bytes_per_launch": 16 * g.n_unique, "avg_launch_ms": ms}
    ctx.close()
    return out


def copy_probe(nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of known size: the achievable HBM rate,
    and the calibration program for the FETCH_SIZE/WRITE_SIZE counters."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
            "ms_per_copy": 1e3 * t, "copy_GBps": 2 * nbytes / t / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble measurement")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-form measurement")
    ap.add_argument("--copy-probe", action="store_true", help="only time a plain 1 GiB device copy")
    ap.add_argument("--no-imex3d", action="store_true", help="skip the 3D-IMEX measurement")
    ap.add_argument("--imex3d-only", action="store_true", help="only run the 3D-IMEX measurement (printed alone)")
    ap.add_argument("--no-learned", action="store_true", help="3D-IMEX without the learned-correction run")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline FP64 measurement (the other legs and the CPU baseline skipped)")
    ap.add_argument("--precision-only", action="store_true",
                    help="only the headline workload's FP64 and precision-form steps (printed alone)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the batched-ensemble measurement (printed alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_probe:
        print(json.dumps(copy_probe()), flush=True)
        return

    import numpy as np
    import torch
    from paper_1702_04316_amd import numa
    from paper_1702_04316_amd import workloads as W

    torch.cuda.set_device(0)
    if args.imex3d_only:
        print(json.dumps(imex3d(numa, torch, learned=not args.no_learned)), flush=True)
        return
    if args.ensemble_only:
        print(json.dumps(batched_ensemble(numa, torch, steps=args.steps)), flush=True)
        return
    wl = W.box_large("R1")
    g = wl.grid
    if args.precision_only:
        ctx = numa.Context(g, wl.background)
        ctx.factor(wl.dt)
        q = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
        cfg = numa.autotune(ctx.ctx, q.data_ptr(), reps=5)
        ctx.step(q, args.warmup)
        t, ms = wall_and_kernels(numa, torch, ctx, q, wl.dt, args.steps)
        ctx.check()
        out = {"workload": "box 64x64x10 elements, N=4, 256x256x41 unique nodes", "rhs_config": cfg,
               "fp64": {"ms_per_step": 1e3 * t, "kernels_ms": ms},
               "precision_form": precision_form(numa, torch, ctx, wl, args, t * args.steps)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    ctx = numa.Context(g, wl.background)
    t0 = time.perf_counter()
    ctx.factor(wl.dt)
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    q = torch.from_numpy(W.make_initial_state(wl)).to("cuda")
    rhs_config = numa.autotune(ctx.ctx, q.data_ptr(), reps=5)

    ctx.step(q, args.warmup)
    ctx.check()
    # value: the wall clock over exactly `steps` steps; the per-kernel
    # durations (roofline) come from a separate profiled run of as many steps
    t, ms = wall_and_kernels(numa, torch, ctx, q, wl.dt, args.steps)
    t *= args.steps
    ctx.check()

    info = ctx.info()
    dof = 5 * g.n_unique
    value = dof * args.steps / t
    kb = kernel_bytes(g.n_unique, info["ncol"], info["nz"], g.N, info["factor_bytes"])
    per = [{"kernel": n, "ms": m, "GB/s": b / (m * 1e-3) / 1e9} for (n, b), m in zip(kb, ms)]
    dom = max(range(5), key=lambda i: ms[i])
    achieved = kb[dom][1] / (ms[dom] * 1e-3) / 1e9
    traffic = load_traffic()
    t_bytes = None
    if traffic:
        t_bytes = traffic.get("bytes_per_launch", {}).get(kb[dom][0])
    step_bytes = info["step_bytes"]
    out = {
        "metric": "HEVI DOF-steps/s on 1 GPU; speedup vs plain FP64 at fixed rel. L2 error",
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "HEVI ARK2 step, box 64x64x10 elements, LGL N=4, 256x256x41 unique nodes, "
                        "vertical Courant 15 (horizontal 0.4, 2400x2400x10 km), 8 seeded theta' bumps, FP64",
            "unique_nodes": g.n_unique,
            "element_local_nodes": g.n_local,
            "dof_per_step": dof,
            "dt_s": wl.dt,
            "element_local_dof_steps_per_s": 5 * g.n_local * args.steps / t,
            "factor_s": t_factor,
            "rhs_config": rhs_config,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kb[dom][0],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": t_bytes,
            "algorithmic_bytes_per_launch": kb[dom][1],
            "avg_launch_ms": ms[dom],
        },
        "kernels": per,
        "step_algorithmic_GBps": step_bytes * args.steps / t / 1e9,
    }
    if args.headline_only:
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    out["standard_form_columns"] = standard_form_columns(numa, torch, ctx, wl, q)
    out["column_solver"] = {"in_use": "blocked" if info["column_solver"] == numa.SOLVER_BLOCKED else "band",
                            "band_substitution": column_solver_ab(numa, torch, wl,
                                                                  torch.from_numpy(W.make_initial_state(wl)).to("cuda"))}
    out["per_column_factors"] = per_column_factors(numa, torch)
    out["stratified"] = stratified_leg(numa, torch)
    if not args.no_precision:
        out["precision_form"] = precision_form(numa, torch, ctx, wl, args, t)
        out["precision_form_n7"] = precision_form_n7(numa, torch)
    if not args.no_ensemble:
        out["batched_ensemble"] = batched_ensemble(numa, torch)
    if not args.no_imex3d:
        out["imex3d"] = imex3d(numa, torch, learned=not args.no_learned)
    cp = copy_probe()
    out["copy_probe"] = cp
    out["roofline"]["frac_of_copy"] = achieved / cp["copy_GBps"]
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline()
        except Exception as e:  # the baseline must not hide the GPU line
            out["cpu_baseline"] = {"error": str(e)}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
