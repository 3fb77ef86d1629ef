"""Thin ctypes binding of the HEVI C ABI (include/numa.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libnuma_hevi.so``.  PyTorch supplies device memory (the state tensor)
and the stream.  If the library has not been built this module raises on
first use; there is no fallback implementation.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnuma_hevi.so")

NUMA_OK = 0
NUMA_E_ARG = -1
NUMA_E_NOT_FACTORED = -2
NUMA_E_DT_MISMATCH = -3
NUMA_E_HIP = -4
NUMA_E_NOMEM = -5
NUMA_E_NONFINITE = -6
NUMA_E_NOT_CONVERGED = -7
NUMA_E_UNSUPPORTED = -8
SOLVER_AUTO, SOLVER_BAND, SOLVER_BLOCKED, SOLVER_PER_COLUMN = 0, 1, 2, 3

ERROR_NAMES = {
    NUMA_E_ARG: "NUMA_E_ARG",
    NUMA_E_NOT_FACTORED: "NUMA_E_NOT_FACTORED",
    NUMA_E_DT_MISMATCH: "NUMA_E_DT_MISMATCH",
    NUMA_E_HIP: "NUMA_E_HIP",
    NUMA_E_NOMEM: "NUMA_E_NOMEM",
    NUMA_E_NONFINITE: "NUMA_E_NONFINITE",
    NUMA_E_NOT_CONVERGED: "NUMA_E_NOT_CONVERGED",
    NUMA_E_UNSUPPORTED: "NUMA_E_UNSUPPORTED",
}


class numa_grid(C.Structure):
    _fields_ = [("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("nex", C.c_int32), ("ney", C.c_int32), ("nez", C.c_int32),
                ("zface", C.POINTER(C.c_double))]


class numa_background(C.Structure):
    _fields_ = [("theta0", C.c_double), ("p00", C.c_double), ("cp", C.c_double),
                ("rgas", C.c_double), ("grav", C.c_double), ("nbv", C.c_double)]


class numa_info(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64), ("ncol", C.c_int64),
                ("factor_bytes", C.c_int64), ("scratch_bytes", C.c_int64), ("step_bytes", C.c_int64),
                ("order", C.c_int32), ("factored", C.c_int32), ("dt_factored", C.c_double),
                ("column_solver", C.c_int32), ("reserved", C.c_int32)]


class NumaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libnuma_hevi.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python __graft_entry__.py` or "
                          f"`python paper_1702_04316_amd/build.py` to build the HIP library")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.numa_setup.argtypes = [C.POINTER(numa_grid), C.c_int32, C.POINTER(numa_background), vp, C.POINTER(vp)]
    lib.numa_state_shape.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.numa_get_info.argtypes = [vp, C.POINTER(numa_info)]
    lib.numa_set_stream.argtypes = [vp, vp]
    lib.numa_factor_columns.argtypes = [vp, C.c_double]
    lib.numa_set_column_solver.argtypes = [vp, C.c_int32]
    lib.numa_autotune.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int32)]
    lib.numa_set_rhs_config.argtypes = [vp, C.c_int32, C.c_int32]
    lib.numa_get_rhs_config.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.numa_hevi_step.argtypes = [vp, vp, C.c_double, C.c_int32]
    lib.numa_profile_steps.argtypes = [vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_double)]
    lib.numa_hevi_step_mixed.argtypes = [vp, vp, C.c_double, C.c_int32]
    lib.numa_hevi_step_mixed_noalloc.argtypes = [vp, vp, C.c_double, C.c_int32]
    lib.numa_ensemble_create.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                         C.c_int32, vp, C.POINTER(vp)]
    lib.numa_ensemble_step.argtypes = [vp, C.c_int32]
    lib.numa_ensemble_sync.argtypes = [vp]
    lib.numa_ensemble_zchunks.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.numa_ensemble_destroy.argtypes = [vp]
    lib.numa_ensemble_last_error.argtypes = [vp]
    lib.numa_ensemble_last_error.restype = C.c_char_p
    lib.numa_profile_steps_mixed.argtypes = [vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_double)]
    lib.numa_rhs.argtypes = [vp, vp, vp]
    lib.numa_solve_columns.argtypes = [vp, vp, vp]
    lib.numa_imex3d_setup.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    lib.numa_imex3d_bounds.argtypes = [vp, C.POINTER(C.c_double)]
    lib.numa_imex3d_set_bounds.argtypes = [vp, C.c_double, C.c_double]
    lib.numa_imex3d_set_precision.argtypes = [vp, C.c_int32]
    lib.numa_schur_apply.argtypes = [vp, vp, vp]
    lib.numa_schur_rhs.argtypes = [vp, vp, vp]
    lib.numa_pbno_apply.argtypes = [vp, vp, vp]
    lib.numa_imex3d_solve.argtypes = [vp, vp, vp, C.c_double, C.POINTER(C.c_int32)]
    lib.numa_imex3d_step.argtypes = [vp, vp, C.c_double, C.c_double, C.POINTER(C.c_int32)]
    lib.numa_factor_columns_standard.argtypes = [vp, C.c_double, C.POINTER(C.c_int64)]
    lib.numa_solve_columns_standard.argtypes = [vp, vp, vp]
    lib.numa_learned_setup.argtypes = [vp, C.c_int32, C.c_int64, C.c_uint64]
    lib.numa_learned_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.numa_learned_add_samples.argtypes = [vp, vp, C.c_double, C.POINTER(C.c_int32)]
    lib.numa_learned_samples.argtypes = [vp, C.c_int64, C.c_int64, vp, vp]
    lib.numa_learned_params.argtypes = [vp, vp, vp]
    lib.numa_learned_loss_grad.argtypes = [vp, vp, vp, C.c_int64, vp, C.POINTER(C.c_double)]
    lib.numa_learned_train.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_uint64, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
    lib.numa_learned_enable.argtypes = [vp, C.c_int32]
    lib.numa_learned_apply.argtypes = [vp, vp, vp]
    lib.numa_learned_judge.argtypes = [vp, vp, vp, C.c_double, C.POINTER(C.c_int32)]
    lib.numa_check.argtypes = [vp]
    lib.numa_destroy.argtypes = [vp]
    lib.numa_last_error.argtypes = [vp]
    lib.numa_last_error.restype = C.c_char_p
    lib.numa_lgl_basis.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.numa_line_operators.argtypes = [C.POINTER(numa_grid), C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
    for name in ("numa_setup", "numa_state_shape", "numa_get_info", "numa_set_stream", "numa_factor_columns",
                 "numa_hevi_step", "numa_profile_steps", "numa_hevi_step_mixed", "numa_hevi_step_mixed_noalloc", "numa_profile_steps_mixed",
                 "numa_rhs", "numa_solve_columns", "numa_imex3d_step", "numa_check", "numa_destroy",
                 "numa_lgl_basis", "numa_line_operators", "numa_ensemble_create", "numa_ensemble_step",
                 "numa_ensemble_sync", "numa_ensemble_zchunks", "numa_ensemble_destroy", "numa_imex3d_setup",
                 "numa_imex3d_bounds", "numa_imex3d_set_bounds", "numa_schur_apply", "numa_schur_rhs",
                 "numa_pbno_apply", "numa_imex3d_solve", "numa_learned_setup", "numa_learned_info",
                 "numa_learned_add_samples", "numa_learned_samples", "numa_learned_params", "numa_learned_loss_grad",
                 "numa_learned_train", "numa_learned_enable", "numa_learned_apply", "numa_learned_judge",
                 "numa_imex3d_set_precision", "numa_factor_columns_standard",
                 "numa_solve_columns_standard", "numa_set_column_solver", "numa_autotune",
                 "numa_set_rhs_config", "numa_get_rhs_config"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def last_error(ctx=None):
    return load().numa_last_error(ctx).decode()


def _check(rc, ctx=None):
    if rc != NUMA_OK:
        raise NumaError(rc, last_error(ctx))
    return rc


def _dptr(arr):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(lx, ly, lz, nex, ney, nez, zface=None):
    """numa_grid plus the host array that keeps zface alive."""
    g = numa_grid(lx, ly, lz, nex, ney, nez, None)
    keep = None
    if zface is not None:
        keep, g.zface = _dptr(zface)
    return g, keep


# ---------------------------------------------------------------------------
# Functions with the ABI's names (raw: return codes, pointers as integers)
# ---------------------------------------------------------------------------

def setup(grid, order, background, stream=None):
    ctx = C.c_void_p()
    rc = load().numa_setup(C.byref(grid), int(order), C.byref(background),
                           C.c_void_p(stream) if stream else None, C.byref(ctx))
    _check(rc, None)
    return ctx.value


def state_shape(ctx):
    s = (C.c_int64 * 4)()
    _check(load().numa_state_shape(ctx, s), ctx)
    return tuple(int(v) for v in s)


def get_info(ctx):
    info = numa_info()
    _check(load().numa_get_info(ctx, C.byref(info)), ctx)
    return {f: getattr(info, f) for f, _ in numa_info._fields_}


def set_stream(ctx, stream):
    return _check(load().numa_set_stream(ctx, C.c_void_p(stream) if stream else None), ctx)


def factor_columns(ctx, dt):
    return _check(load().numa_factor_columns(ctx, float(dt)), ctx)


def set_column_solver(ctx, kind):
    return _check(load().numa_set_column_solver(ctx, int(kind)), ctx)


def autotune(ctx, state_ptr, reps=3):
    """Autotune the right-hand sides on the state; returns {tile, TX, TY, zchunk}."""
    out = (C.c_int32 * 4)()
    _check(load().numa_autotune(ctx, C.c_void_p(state_ptr), int(reps), out), ctx)
    return dict(zip(("tile", "TX", "TY", "zchunk"), (int(v) for v in out)))


def set_rhs_config(ctx, tile, zchunk=0):
    return _check(load().numa_set_rhs_config(ctx, int(tile), int(zchunk)), ctx)


def get_rhs_config(ctx):
    out = (C.c_int32 * 4)()
    _check(load().numa_get_rhs_config(ctx, out), ctx)
    return dict(zip(("tile", "TX", "TY", "zchunk"), (int(v) for v in out)))


def hevi_step(ctx, state_ptr, dt, nsteps):
    return _check(load().numa_hevi_step(ctx, C.c_void_p(state_ptr), float(dt), int(nsteps)), ctx)


def hevi_step_mixed(ctx, state_ptr, dt, nsteps):
    """The precision form of hevi_step (the first-stage tendency R1 stored in FP32)."""
    return _check(load().numa_hevi_step_mixed(ctx, C.c_void_p(state_ptr), float(dt), int(nsteps)), ctx)


def hevi_step_mixed_noalloc(ctx, state_ptr, dt, nsteps):
    """hevi_step_mixed with the library's fixed stage buffers (no allocation)."""
    return _check(load().numa_hevi_step_mixed_noalloc(ctx, C.c_void_p(state_ptr), float(dt), int(nsteps)), ctx)


def profile_steps_mixed(ctx, state_ptr, dt, nsteps):
    """profile_steps for the precision form."""
    ms = (C.c_double * 5)()
    _check(load().numa_profile_steps_mixed(ctx, C.c_void_p(state_ptr), float(dt), int(nsteps), ms), ctx)
    return [float(v) for v in ms]


def ensemble_last_error(ens=None):
    return (load().numa_ensemble_last_error(ens) or b"").decode()


def _echeck(rc, ens=None):
    if rc != NUMA_OK:
        raise NumaError(rc, ensemble_last_error(ens))
    return rc


def ensemble_create(ctxs, state_ptrs, dts, mixed=False, tune=True, stream=None):
    """numa_ensemble_create: one captured step over the n contexts."""
    n = len(ctxs)
    carr = (C.c_void_p * n)(*ctxs)
    sarr = (C.c_void_p * n)(*state_ptrs)
    darr = (C.c_double * n)(*[float(d) for d in dts])
    out = C.c_void_p()
    _echeck(load().numa_ensemble_create(carr, sarr, darr, n, 1 if mixed else 0, 1 if tune else 0,
                                        C.c_void_p(stream) if stream else None, C.byref(out)))
    return out.value


def ensemble_step(ens, nsteps):
    return _echeck(load().numa_ensemble_step(ens, int(nsteps)), ens)


def ensemble_sync(ens):
    return _echeck(load().numa_ensemble_sync(ens), ens)


def ensemble_zchunks(ens, n):
    z = (C.c_int32 * n)()
    _echeck(load().numa_ensemble_zchunks(ens, z), ens)
    return [int(v) for v in z]


def ensemble_destroy(ens):
    return load().numa_ensemble_destroy(ens)


class Ensemble:
    """Several contexts (each factored with its dt) and their device states
    stepped together through one captured graph per step."""

    def __init__(self, contexts, states, mixed=False, tune=True):
        for c, st in zip(contexts, states):
            c._check_state(st)
        self.contexts = list(contexts)
        self.states = list(states)  # keep the tensors alive
        self.ens = ensemble_create([c.ctx for c in contexts], [st.data_ptr() for st in states],
                                   [c.dt for c in contexts], mixed=mixed, tune=tune)

    def step(self, nsteps=1):
        ensemble_step(self.ens, nsteps)

    def sync(self):
        ensemble_sync(self.ens)

    def zchunks(self):
        return ensemble_zchunks(self.ens, len(self.contexts))

    def close(self):
        if getattr(self, "ens", None):
            ensemble_destroy(self.ens)
            self.ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_steps(ctx, state_ptr, dt, nsteps):
    """Average milliseconds of each of the 5 kernels of a step (launch order)."""
    ms = (C.c_double * 5)()
    _check(load().numa_profile_steps(ctx, C.c_void_p(state_ptr), float(dt), int(nsteps), ms), ctx)
    return [float(v) for v in ms]


def rhs(ctx, state_ptr, out_ptr):
    return _check(load().numa_rhs(ctx, C.c_void_p(state_ptr), C.c_void_p(out_ptr)), ctx)


def solve_columns(ctx, y_ptr, x_ptr):
    return _check(load().numa_solve_columns(ctx, C.c_void_p(y_ptr), C.c_void_p(x_ptr)), ctx)


def imex3d_setup(ctx, dt, restart=30, pbno_order=1, power_steps=30, maxit=5000):
    return _check(load().numa_imex3d_setup(ctx, float(dt), int(restart), int(pbno_order), int(power_steps),
                                           int(maxit)), ctx)


def imex3d_bounds(ctx):
    out = (C.c_double * 2)()
    _check(load().numa_imex3d_bounds(ctx, out), ctx)
    return float(out[0]), float(out[1])


def imex3d_set_bounds(ctx, lmin, lmax):
    return _check(load().numa_imex3d_set_bounds(ctx, float(lmin), float(lmax)), ctx)


def imex3d_set_precision(ctx, pbno_fp32):
    """pbno_fp32=True: the PBNO recurrence in FP32 (flexible GMRES)."""
    return _check(load().numa_imex3d_set_precision(ctx, 1 if pbno_fp32 else 0), ctx)


def schur_apply(ctx, p_ptr, out_ptr):
    return _check(load().numa_schur_apply(ctx, C.c_void_p(p_ptr), C.c_void_p(out_ptr)), ctx)


def schur_rhs(ctx, y_ptr, b_ptr):
    return _check(load().numa_schur_rhs(ctx, C.c_void_p(y_ptr), C.c_void_p(b_ptr)), ctx)


def pbno_apply(ctx, r_ptr, z_ptr):
    return _check(load().numa_pbno_apply(ctx, C.c_void_p(r_ptr), C.c_void_p(z_ptr)), ctx)


def imex3d_solve(ctx, y_ptr, x_ptr, tol):
    it = C.c_int32(0)
    _check(load().numa_imex3d_solve(ctx, C.c_void_p(y_ptr), C.c_void_p(x_ptr), float(tol), C.byref(it)), ctx)
    return it.value


def factor_columns_standard(ctx, dt):
    nb = C.c_int64(0)
    _check(load().numa_factor_columns_standard(ctx, float(dt), C.byref(nb)), ctx)
    return nb.value


def solve_columns_standard(ctx, y_ptr, x_ptr):
    return _check(load().numa_solve_columns_standard(ctx, C.c_void_p(y_ptr), C.c_void_p(x_ptr)), ctx)


def learned_setup(ctx, hidden=64, max_samples=24576, seed=1):
    return _check(load().numa_learned_setup(ctx, int(hidden), int(max_samples), int(seed)), ctx)


def learned_info(ctx):
    info = (C.c_int64 * 6)()
    _check(load().numa_learned_info(ctx, info), ctx)
    return dict(zip(("nparam", "nin", "hidden", "samples", "max_samples", "enabled"), (int(v) for v in info)))


def learned_add_samples(ctx, r_ptr, tol):
    it = C.c_int32(0)
    _check(load().numa_learned_add_samples(ctx, C.c_void_p(r_ptr), float(tol), C.byref(it)), ctx)
    return it.value


def learned_samples(ctx, first, n, x_ptr, t_ptr):
    return _check(load().numa_learned_samples(ctx, int(first), int(n), C.c_void_p(x_ptr), C.c_void_p(t_ptr)), ctx)


def learned_params(ctx, theta_out=None, theta_in=None):
    """theta_out / theta_in: host float32 numpy arrays (nparam) or None."""
    po = theta_out.ctypes.data_as(C.c_void_p) if theta_out is not None else None
    pi = theta_in.ctypes.data_as(C.c_void_p) if theta_in is not None else None
    return _check(load().numa_learned_params(ctx, po, pi), ctx)


def learned_loss_grad(ctx, x_ptr, t_ptr, n, grad_ptr):
    loss = C.c_double(0.0)
    _check(load().numa_learned_loss_grad(ctx, C.c_void_p(x_ptr), C.c_void_p(t_ptr), int(n), C.c_void_p(grad_ptr),
                                         C.byref(loss)), ctx)
    return loss.value


def learned_train(ctx, steps, batch=1024, lr=1e-3, seed=7):
    lf, ll = C.c_double(0.0), C.c_double(0.0)
    _check(load().numa_learned_train(ctx, int(steps), int(batch), float(lr), int(seed), C.byref(lf), C.byref(ll)),
           ctx)
    return lf.value, ll.value


def learned_enable(ctx, on):
    return _check(load().numa_learned_enable(ctx, 1 if on else 0), ctx)


def learned_judge(ctx, y_ptr, x_ptr, tol):
    """PBNO judges the network on (I - lambda L) x = y; returns
    {pbno_iters, net_iters, accepted} (the network stays on if accepted)."""
    out = (C.c_int32 * 3)()
    _check(load().numa_learned_judge(ctx, C.c_void_p(y_ptr), C.c_void_p(x_ptr), float(tol), out), ctx)
    return {"pbno_iters": int(out[0]), "net_iters": int(out[1]), "accepted": bool(out[2])}


def learned_apply(ctx, r_ptr, z_ptr):
    return _check(load().numa_learned_apply(ctx, C.c_void_p(r_ptr), C.c_void_p(z_ptr)), ctx)


def imex3d_step(ctx, state_ptr, dt, tol):
    it = C.c_int32(0)
    _check(load().numa_imex3d_step(ctx, C.c_void_p(state_ptr), float(dt), float(tol), C.byref(it)), ctx)
    return it.value


def check(ctx):
    return _check(load().numa_check(ctx), ctx)


def destroy(ctx):
    return load().numa_destroy(ctx)


def lgl_basis(order):
    import numpy as np
    xi = np.zeros(order + 1)
    D = np.zeros((order + 1) ** 2)
    _check(load().numa_lgl_basis(int(order), xi.ctypes.data_as(C.POINTER(C.c_double)),
                                 D.ctypes.data_as(C.POINTER(C.c_double))))
    return xi, D.reshape(order + 1, order + 1)


def line_operators(grid, order):
    import numpy as np
    ns = 2 * order + 1
    nz = grid.nez * order + 1
    wxy = np.zeros(2 * order * ns)
    dzb = np.zeros(nz * ns)
    _check(load().numa_line_operators(C.byref(grid), int(order), wxy.ctypes.data_as(C.POINTER(C.c_double)),
                                      dzb.ctypes.data_as(C.POINTER(C.c_double))))
    return wxy.reshape(2, order, ns), dzb.reshape(nz, ns)


# ---------------------------------------------------------------------------
# Convenience wrapper around one context (torch tensors for the state)
# ---------------------------------------------------------------------------

class Context:
    """One HEVI context on the current CUDA (HIP) device and stream."""

    def __init__(self, grid, background=None, stream=None):
        import torch
        from . import workloads as W
        bg = background or W.Background()
        self.grid = grid
        self._g, self._zkeep = make_grid(grid.lx, grid.ly, grid.lz, grid.nex, grid.ney, grid.nez,
                                         grid.zface)
        self._bg = numa_background(bg.theta0, bg.p00, bg.cp, bg.rgas, bg.grav, getattr(bg, "nbv", 0.0))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.ctx = setup(self._g, grid.N, self._bg, stream)
        self.shape = state_shape(self.ctx)
        self.dt = None

    def close(self):
        if getattr(self, "ctx", None):
            destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return get_info(self.ctx)

    def factor(self, dt):
        factor_columns(self.ctx, dt)
        self.dt = float(dt)

    def set_column_solver(self, kind):
        """SOLVER_AUTO, SOLVER_BAND or SOLVER_BLOCKED; call factor() again after."""
        set_column_solver(self.ctx, kind)
        self.dt = None

    def _check_state(self, t):
        import torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous(), "state: contiguous float64 cuda"
        assert tuple(t.shape) == self.shape, (tuple(t.shape), self.shape)

    def step(self, state, nsteps=1, dt=None, mixed=False):
        """nsteps HEVI steps in place; mixed=True runs the precision form."""
        self._check_state(state)
        (hevi_step_mixed if mixed else hevi_step)(self.ctx, state.data_ptr(), self.dt if dt is None else dt, nsteps)
        return state

    def rhs(self, state, out=None):
        import torch
        self._check_state(state)
        out = torch.empty_like(state) if out is None else out
        self._check_state(out)
        rhs(self.ctx, state.data_ptr(), out.data_ptr())
        return out

    def solve(self, y, out=None):
        import torch
        self._check_state(y)
        out = torch.empty_like(y) if out is None else out
        self._check_state(out)
        solve_columns(self.ctx, y.data_ptr(), out.data_ptr())
        return out

    # --- 3D-IMEX -------------------------------------------------------------
    def imex3d_setup(self, dt, restart=30, pbno_order=1, power_steps=30, maxit=5000):
        imex3d_setup(self.ctx, dt, restart, pbno_order, power_steps, maxit)
        self.dt3d = float(dt)
        return imex3d_bounds(self.ctx)

    def imex3d_step(self, state, tol, nsteps=1):
        """nsteps 3D-IMEX steps in place; returns the GMRES iterations."""
        self._check_state(state)
        return sum(imex3d_step(self.ctx, state.data_ptr(), self.dt3d, tol) for _ in range(nsteps))

    def imex3d_solve(self, y, tol, out=None):
        import torch
        self._check_state(y)
        out = torch.empty_like(y) if out is None else out
        self._check_state(out)
        it = imex3d_solve(self.ctx, y.data_ptr(), out.data_ptr(), tol)
        return out, it

    def _scalar(self, t):
        import torch
        assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        assert tuple(t.shape) == self.shape[1:], (tuple(t.shape), self.shape)

    def schur_apply(self, P):
        import torch
        self._scalar(P)
        out = torch.empty_like(P)
        schur_apply(self.ctx, P.data_ptr(), out.data_ptr())
        return out

    def schur_rhs(self, y):
        import torch
        self._check_state(y)
        out = torch.empty(self.shape[1:], dtype=torch.float64, device=y.device)
        schur_rhs(self.ctx, y.data_ptr(), out.data_ptr())
        return out

    def pbno_apply(self, r):
        import torch
        self._scalar(r)
        out = torch.empty_like(r)
        pbno_apply(self.ctx, r.data_ptr(), out.data_ptr())
        return out

    def check(self):
        return check(self.ctx)
