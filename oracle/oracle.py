"""ctypes binding of the plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It loads ``oracle/libnuma_oracle.so`` (built by
``oracle/build.py``) and shares nothing with the GPU library.

Arrays are numpy float64, C-contiguous.  The state is (5, nz, ny, nx) with
fields (rho', u, v, w, theta').
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libnuma_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB)
    lib.orc_lgl.argtypes = [C.c_int, _dp, _dp]
    lib.orc_dmat.argtypes = [C.c_int, _dp, _dp]
    lib.orc_setup.restype = C.c_void_p
    lib.orc_setup.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                              C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_double, C.c_double]
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_get_threads.restype = C.c_int
    lib.orc_sizes.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")]
    lib.orc_coords.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.orc_mass.argtypes = [C.c_void_p, _dp]
    lib.orc_background.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    lib.orc_background_theta.argtypes = [C.c_void_p, _dp, _dp]
    for name in ("orc_rhs", "orc_lv", "orc_lfull", "orc_solve"):
        f = getattr(lib, name)
        f.argtypes = [C.c_void_p, _dp, _dp]
        f.restype = C.c_int
    lib.orc_pressure_perturbation.argtypes = [C.c_void_p, _dp, _dp]
    lib.orc_pressure_perturbation.restype = C.c_int
    lib.orc_factor.argtypes = [C.c_void_p, C.c_double]
    lib.orc_factor.restype = C.c_int
    lib.orc_column_matrix.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int, _dp]
    lib.orc_column_matrix.restype = C.c_int
    lib.orc_step.argtypes = [C.c_void_p, _dp, C.c_double, C.c_int, C.c_int]
    lib.orc_step.restype = C.c_int
    lib.orc_ark2_tableau.argtypes = [_dp, _dp, _dp]
    lib.orc_schur_apply.argtypes = [C.c_void_p, _dp, _dp, C.c_double]
    lib.orc_schur_rhs.argtypes = [C.c_void_p, _dp, _dp, C.c_double]
    lib.orc_pbno_apply.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_double, C.c_double]
    lib.orc_schur_bounds.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp]
    lib.orc_solve3d.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _dp,
                                C.POINTER(C.c_int)]
    lib.orc_solve3d_standard.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                         C.POINTER(C.c_int)]
    lib.orc_step3d.argtypes = [C.c_void_p, _dp, C.c_double, C.c_int, C.c_int, C.c_double, C.c_int, _dp,
                               C.POINTER(C.c_int)]
    lib.orc_mlp_loss_grad.argtypes = [C.POINTER(OrcMlp), C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_mlp_loss_grad.restype = C.c_double
    lib.orc_element_features.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.orc_mlp_correction.argtypes = [C.c_void_p, C.POINTER(OrcMlp), _dp, _dp]
    lib.orc_learned_apply.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, _dp, C.POINTER(OrcMlp)]
    lib.orc_solve3d_learned.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                        _dp, C.POINTER(OrcMlp), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.orc_learned_judge.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _dp,
                                      C.POINTER(OrcMlp), C.POINTER(C.c_int)]
    for name in ("orc_schur_apply", "orc_schur_rhs", "orc_pbno_apply", "orc_schur_bounds", "orc_solve3d",
                 "orc_solve3d_standard", "orc_step3d", "orc_element_features", "orc_mlp_correction",
                 "orc_learned_apply", "orc_solve3d_learned", "orc_learned_judge"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


class OrcMlp(C.Structure):
    _fields_ = [("nin", C.c_int), ("nh", C.c_int), ("W1", C.POINTER(C.c_double)), ("b1", C.POINTER(C.c_double)),
                ("W2", C.POINTER(C.c_double)), ("b2", C.POINTER(C.c_double))]


class Mlp:
    """Weights of the per-element perceptron (float64 copies): W1[nh][nin],
    b1[nh], W2[nin][nh], b2[nin]."""

    def __init__(self, W1, b1, W2, b2):
        self.W1 = np.ascontiguousarray(W1, dtype=np.float64)
        self.b1 = np.ascontiguousarray(b1, dtype=np.float64)
        self.W2 = np.ascontiguousarray(W2, dtype=np.float64)
        self.b2 = np.ascontiguousarray(b2, dtype=np.float64)
        nh, nin = self.W1.shape
        assert self.W2.shape == (nin, nh) and self.b1.shape == (nh,) and self.b2.shape == (nin,)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self.s = OrcMlp(nin, nh, p(self.W1), p(self.b1), p(self.W2), p(self.b2))

    def loss_grad(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        g = [np.zeros_like(self.W1), np.zeros_like(self.b1), np.zeros_like(self.W2), np.zeros_like(self.b2)]
        loss = _load().orc_mlp_loss_grad(C.byref(self.s), X.shape[0], X.reshape(-1), T.reshape(-1),
                                         *[a.reshape(-1) for a in g])
        return loss, g


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def lgl(N):
    lib = _load()
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    lib.orc_lgl(N, xi, w)
    return xi, w


def dmat(N):
    lib = _load()
    xi, _ = lgl(N)
    D = np.zeros((N + 1) * (N + 1))
    lib.orc_dmat(N, xi, D)
    return D.reshape(N + 1, N + 1)


def ark2_tableau():
    lib = _load()
    a = np.zeros(9)
    at = np.zeros(9)
    b = np.zeros(3)
    lib.orc_ark2_tableau(a, at, b)
    return a.reshape(3, 3), at.reshape(3, 3), b


def set_threads(n):
    _load().orc_set_threads(int(n))


def get_threads():
    return int(_load().orc_get_threads())


class Oracle:
    """One grid + background; mirrors the GPU library's set-up contract."""

    def __init__(self, lx, ly, lz, nex, ney, nez, N, theta0=300.0, p00=1.0e5,
                 cp=1004.67, rgas=287.17, grav=9.80616, zface=None, nbv=0.0):
        lib = _load()
        self._zf = None if zface is None else np.ascontiguousarray(zface, dtype=np.float64)
        zp = None if self._zf is None else self._zf.ctypes.data_as(C.c_void_p)
        self.h = lib.orc_setup(lx, ly, lz, nex, ney, nez, zp, N, theta0, p00, cp, rgas, grav, nbv)
        self.nvar = 3 if nbv > 0.0 else 2
        if not self.h:
            raise OracleError("orc_setup rejected its arguments")
        sz = np.zeros(4, dtype=np.int64)
        lib.orc_sizes(self.h, sz)
        self.nx, self.ny, self.nz, self.nelem = (int(v) for v in sz)
        self.N = N
        self.shape = (5, self.nz, self.ny, self.nx)
        self.lam = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self.h = None

    def coords(self):
        x = np.zeros(self.nx)
        y = np.zeros(self.ny)
        z = np.zeros(self.nz)
        _lib.orc_coords(self.h, x, y, z)
        return x, y, z

    def mass(self):
        M = np.zeros(self.shape[1:])
        _lib.orc_mass(self.h, M.reshape(-1))
        return M

    def background(self):
        out = [np.zeros(self.nz) for _ in range(4)]
        _lib.orc_background(self.h, *out)
        th = [np.zeros(self.nz) for _ in range(2)]
        _lib.orc_background_theta(self.h, *th)
        return dict(zip(("rho0", "P0", "G0", "H0", "theta0", "dtheta0dz"), out + th))

    def _op(self, name, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == self.shape, (q.shape, self.shape)
        out = np.zeros(self.shape)
        _check(getattr(_lib, name)(self.h, q.reshape(-1), out.reshape(-1)), name)
        return out

    def pressure_perturbation(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(self.shape[1:])
        _check(_lib.orc_pressure_perturbation(self.h, q.reshape(-1), out.reshape(-1)), "orc_pressure_perturbation")
        return out

    def rhs(self, q):
        return self._op("orc_rhs", q)

    def lv(self, q):
        return self._op("orc_lv", q)

    def lfull(self, q):
        return self._op("orc_lfull", q)

    def factor(self, lam):
        _check(_lib.orc_factor(self.h, float(lam)), "orc_factor")
        self.lam = float(lam)

    def factor_dt(self, dt):
        self.factor((1.0 - 1.0 / np.sqrt(2.0)) * dt)

    def solve(self, y):
        return self._op("orc_solve", y)

    def column_matrix(self, lam, i, j):
        n2 = self.nvar * self.nz
        A = np.zeros(n2 * n2)
        _check(_lib.orc_column_matrix(self.h, float(lam), i, j, A), "orc_column_matrix")
        return A.reshape(n2, n2)

    def step(self, q, dt, nsteps=1, linear=False):
        q = np.array(q, dtype=np.float64, order="C", copy=True)
        assert q.shape == self.shape
        _check(_lib.orc_step(self.h, q.reshape(-1), float(dt), int(nsteps), 1 if linear else 0), "orc_step")
        return q

    # --- 3D-IMEX (Schur form, GMRES, PBNO) ---------------------------------
    def schur_apply(self, P, lam):
        P = np.ascontiguousarray(P, dtype=np.float64)
        assert P.shape == self.shape[1:]
        out = np.zeros(self.shape[1:])
        _check(_lib.orc_schur_apply(self.h, P.reshape(-1), out.reshape(-1), float(lam)), "orc_schur_apply")
        return out

    def schur_rhs(self, y, lam):
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert y.shape == self.shape
        out = np.zeros(self.shape[1:])
        _check(_lib.orc_schur_rhs(self.h, y.reshape(-1), out.reshape(-1), float(lam)), "orc_schur_rhs")
        return out

    def pbno_apply(self, r, lam, order, bounds):
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(self.shape[1:])
        _check(_lib.orc_pbno_apply(self.h, r.reshape(-1), out.reshape(-1), float(lam), int(order),
                                   float(bounds[0]), float(bounds[1])), "orc_pbno_apply")
        return out

    def schur_bounds(self, lam, k=30):
        out = np.zeros(2)
        _check(_lib.orc_schur_bounds(self.h, float(lam), int(k), out), "orc_schur_bounds")
        return out

    def solve3d(self, y, lam, tol=1e-12, restart=30, maxit=100000, order=-1, bounds=None, allow_unconverged=False):
        """(I - lam L)^{-1} y through the Schur form; returns (x, iterations)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert y.shape == self.shape
        x = np.zeros(self.shape)
        it = C.c_int(0)
        bd = np.ascontiguousarray(bounds if bounds is not None else (1.0, 2.0), dtype=np.float64)
        rc = _lib.orc_solve3d(self.h, y.reshape(-1), x.reshape(-1), float(lam), float(tol), int(restart), int(maxit),
                              int(order), bd, C.byref(it))
        if not (allow_unconverged and rc == -6):
            _check(rc, "orc_solve3d")
        return x, it.value

    def solve3d_standard(self, y, lam, tol=1e-12, restart=40, maxit=100000):
        y = np.ascontiguousarray(y, dtype=np.float64)
        x = np.zeros(self.shape)
        it = C.c_int(0)
        _check(_lib.orc_solve3d_standard(self.h, y.reshape(-1), x.reshape(-1), float(lam), float(tol), int(restart),
                                         int(maxit), C.byref(it)), "orc_solve3d_standard")
        return x, it.value

    def step3d(self, q, dt, nsteps=1, tol=1e-12, linear=False, order=-1, bounds=None):
        """nsteps 3D-IMEX ARK2 steps; returns (state, GMRES iterations)."""
        q = np.array(q, dtype=np.float64, order="C", copy=True)
        assert q.shape == self.shape
        it = C.c_int(0)
        bd = np.ascontiguousarray(bounds if bounds is not None else (1.0, 2.0), dtype=np.float64)
        _check(_lib.orc_step3d(self.h, q.reshape(-1), float(dt), int(nsteps), 1 if linear else 0, float(tol),
                               int(order), bd, C.byref(it)), "orc_step3d")
        return q, it.value

    # --- learned preconditioner (project addition) --------------------------
    def element_features(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        nq3 = (self.N + 1) ** 3
        ne = self.nelem
        X = np.zeros((ne, nq3))
        sc = np.zeros(ne)
        _check(_lib.orc_element_features(self.h, r.reshape(-1), X.reshape(-1), sc), "orc_element_features")
        return X, sc

    def mlp_correction(self, mlp, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(self.shape[1:])
        _check(_lib.orc_mlp_correction(self.h, C.byref(mlp.s), r.reshape(-1), out.reshape(-1)), "orc_mlp_correction")
        return out

    def learned_apply(self, r, lam, order, bounds, mlp):
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(self.shape[1:])
        bd = np.ascontiguousarray(bounds if bounds is not None else (1.0, 2.0), dtype=np.float64)
        _check(_lib.orc_learned_apply(self.h, r.reshape(-1), out.reshape(-1), float(lam), int(order), bd,
                                      C.byref(mlp.s) if mlp is not None else None), "orc_learned_apply")
        return out

    def solve3d_learned(self, y, lam, mlp, tol=1e-12, restart=30, maxit=100000, order=-1, bounds=None,
                        with_cycles=False):
        """Flexible GMRES with PBNO + the network; returns (x, iterations), and
        with with_cycles also the number of restart cycles that ran with the
        network (the fallback switches it off after a cycle that does not cut
        the residual tenfold)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        x = np.zeros(self.shape)
        it = C.c_int(0)
        nc = C.c_int(0)
        bd = np.ascontiguousarray(bounds if bounds is not None else (1.0, 2.0), dtype=np.float64)
        _check(_lib.orc_solve3d_learned(self.h, y.reshape(-1), x.reshape(-1), float(lam), float(tol), int(restart),
                                        int(maxit), int(order), bd, C.byref(mlp.s) if mlp is not None else None,
                                        C.byref(it), C.byref(nc)), "orc_solve3d_learned")
        return (x, it.value, nc.value) if with_cycles else (x, it.value)

    def learned_judge(self, y, lam, mlp, tol=1e-12, restart=30, maxit=100000, order=-1, bounds=None):
        """The polynomial judges the network on (I - lam L) x = y: returns
        (polynomial iterations, network iterations, accepted)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert y.shape == self.shape
        out = (C.c_int * 3)()
        bd = np.ascontiguousarray(bounds if bounds is not None else (1.0, 2.0), dtype=np.float64)
        _check(_lib.orc_learned_judge(self.h, y.reshape(-1), float(lam), float(tol), int(restart), int(maxit),
                                      int(order), bd, C.byref(mlp.s), out), "orc_learned_judge")
        return int(out[0]), int(out[1]), bool(out[2])
