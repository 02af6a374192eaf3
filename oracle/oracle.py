"""Python face of the CPU oracle (test infrastructure only).

Wraps ``liboracle.so`` (plain C, see ``ace_oracle.c``) with numpy arrays.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this module.  Nothing here is shared with the GPU library.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

BC_HN, BC_HD, BC_P = 0, 1, 2
BC_NAMES = {"HN": BC_HN, "HD": BC_HD, "P": BC_P}

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_L = ctypes.POINTER(ctypes.c_long)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_nodes_per_axis.argtypes = [ctypes.c_long, ctypes.c_int]
        L.oracle_nodes_per_axis.restype = ctypes.c_long
        L.oracle_node_coord.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_long]
        L.oracle_node_coord.restype = ctypes.c_double
        L.oracle_kappa.argtypes = [ctypes.c_double] * 3
        L.oracle_kappa.restype = ctypes.c_double
        L.oracle_root.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_root.restype = ctypes.c_double
        L.oracle_root_array.argtypes = [ctypes.c_long, _D, ctypes.c_double, _D]
        L.oracle_root_array.restype = None
        L.oracle_xi.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_xi.restype = None
        L.oracle_step.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_step.restype = None
        L.oracle_bulk_sum.argtypes = [ctypes.c_long, _D]
        L.oracle_bulk_sum.restype = ctypes.c_double
        L.oracle_grad_sum.argtypes = [ctypes.c_int, _L, ctypes.c_int, _D]
        L.oracle_grad_sum.restype = ctypes.c_double
        L.oracle_energy.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.oracle_energy.restype = ctypes.c_double
        L.oracle_maxnorm.argtypes = [ctypes.c_long, _D]
        L.oracle_maxnorm.restype = ctypes.c_double
        L.oracle_run.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _D, ctypes.c_long, ctypes.c_long, _D, _D]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_step_fex.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_step_fex.restype = None
        L.oracle_run_scheme.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _D, ctypes.c_long, ctypes.c_long, _D, _D, ctypes.c_int]
        L.oracle_run_scheme.restype = ctypes.c_int
        L.oracle_phase_volume.argtypes = [ctypes.c_int, _L, ctypes.c_double, _D]
        L.oracle_phase_volume.restype = ctypes.c_double
        L.oracle_adjoint.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     _D, ctypes.c_long, _D, _D, _D]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_pop_moment.argtypes = [ctypes.c_int, _L, _D, _D]
        L.oracle_pop_moment.restype = None
        L.oracle_pop_equilibrium.argtypes = [ctypes.c_int, _L, ctypes.c_double, _D, _D]
        L.oracle_pop_equilibrium.restype = None
        L.oracle_pop_step.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_pop_step.restype = None
        L.oracle_pop_run.argtypes = [ctypes.c_int, _L, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, _D, ctypes.c_long]
        L.oracle_pop_run.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's parallel loops (0 leaves them); returns the
    previous maximum.  Results do not depend on it."""
    return lib().oracle_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _bc(bc):
    return BC_NAMES[bc] if isinstance(bc, str) else int(bc)


def root(xi, h):
    """Unique real root of theta + h(theta^3 - theta) = xi, elementwise."""
    xi = _f64(np.atleast_1d(xi))
    out = np.empty_like(xi)
    lib().oracle_root_array(xi.size, _dp(xi), float(h), _dp(out))
    return out


class Problem:
    """One Allen-Cahn problem: d, N[], L[], R[], eps, dt, bc (Sec. 2)."""

    def __init__(self, d, N, L, R, eps, dt, bc, scheme=0):
        self.d = int(d)
        self.N = [int(n) for n in N][: self.d]
        self.L = [float(x) for x in L][: self.d]
        self.R = [float(x) for x in R][: self.d]
        self.eps = float(eps)
        self.dt = float(dt)
        self.bc = _bc(bc)
        self.h = 0.5 * self.dt
        # Delta x = X / N (square mesh: all axes share one spacing)
        self.dx = (self.R[0] - self.L[0]) / self.N[0]
        self.kappa = lib().oracle_kappa(self.eps, self.dt, self.dx)
        self.M = [int(lib().oracle_nodes_per_axis(n, self.bc)) for n in self.N]
        self.shape = tuple(self.M)
        self._Marr = (ctypes.c_long * 3)(*(self.M + [1] * (3 - self.d)))
        self.scheme = int(scheme)  # 0: RLB-MIE-FD, 1: FEX-FD (Remark 2)

    # Theorem 2 hypothesis on the step: dt <= 1 - 2 d kappa, 0 < kappa < 1/(2d);
    # for FEX-FD Remark 2's dt <= (1 - 2 d kappa) / 2
    def conditions_ok(self, rel=1e-12):
        bound = 1.0 - 2 * self.d * self.kappa
        if self.scheme == 1:
            bound *= 0.5
        return self.dt <= bound * (1.0 + rel) and 0.0 < self.kappa < 1.0 / (2 * self.d)

    def coords(self, axis):
        return np.array([lib().oracle_node_coord(self.bc, self.L[axis], self.dx, i)
                         for i in range(self.M[axis])])

    def xi(self, phi):
        phi = _f64(phi).reshape(self.shape)
        out = np.empty_like(phi)
        lib().oracle_xi(self.d, self._Marr, self.bc, self.kappa, self.h, _dp(phi), _dp(out))
        return out

    def step(self, phi):
        phi = _f64(phi).reshape(self.shape)
        out = np.empty_like(phi)
        if self.scheme == 1:
            lib().oracle_step_fex(self.d, self._Marr, self.bc, self.kappa, self.dt, _dp(phi), _dp(out))
        else:
            lib().oracle_step(self.d, self._Marr, self.bc, self.kappa, self.h, _dp(phi), _dp(out))
        return out

    def run(self, phi0, nsteps, every=0):
        """Returns (phi after nsteps, E series, max-norm series)."""
        phi = _f64(phi0).reshape(self.shape).copy()
        nmon = nsteps // every + 1 if every > 0 else 0
        E = np.empty(max(nmon, 1))
        mx = np.empty(max(nmon, 1))
        rc = lib().oracle_run_scheme(self.d, self._Marr, self.bc, self.kappa, self.dt, self.dx,
                                     _dp(phi), int(nsteps), int(every), _dp(E), _dp(mx), self.scheme)
        if rc != 0:
            raise MemoryError("oracle_run")
        return phi, E[:nmon], mx[:nmon]

    def energy(self, phi):
        phi = _f64(phi).reshape(self.shape)
        return lib().oracle_energy(self.d, self._Marr, self.bc, self.kappa, self.dt, self.dx, _dp(phi))

    def grad_sum(self, phi):
        phi = _f64(phi).reshape(self.shape)
        return lib().oracle_grad_sum(self.d, self._Marr, self.bc, _dp(phi))

    def phase_volume(self, phi):
        phi = _f64(phi).reshape(self.shape)
        return lib().oracle_phase_volume(self.d, self._Marr, self.dx, _dp(phi))

    def equivalent_radius(self, phi):
        """Radius of the disc (d = 2) or ball (d = 3) with the phase volume."""
        V = self.phase_volume(phi)
        if self.d == 2:
            return math.sqrt(V / math.pi)
        return (3 * V / (4 * math.pi)) ** (1.0 / 3.0)

    def maxnorm(self, phi):
        phi = _f64(phi)
        return lib().oracle_maxnorm(phi.size, _dp(phi))

    # ---- mesoscopic form (Sec. 2): 2d+1 populations per node ----
    def default_omega1(self):
        """The weight the paper's experiments use: 1/3, 1/5, 1/6 for d = 1, 2, 3."""
        return {1: 1 / 3, 2: 1 / 5, 3: 1 / 6}[self.d]

    def relaxation(self, omega1=None):
        """s = omega_1 / kappa (kappa = omega_1 / s, Sec. 2)."""
        omega1 = self.default_omega1() if omega1 is None else float(omega1)
        return omega1 / self.kappa

    def pop_equilibrium(self, phi, omega1=None):
        omega1 = self.default_omega1() if omega1 is None else float(omega1)
        phi = _f64(phi).reshape(self.shape)
        f = np.empty((2 * self.d + 1,) + self.shape)
        lib().oracle_pop_equilibrium(self.d, self._Marr, omega1, _dp(phi), _dp(f))
        return f

    def pop_moment(self, f):
        f = _f64(f).reshape((2 * self.d + 1,) + self.shape)
        phi = np.empty(self.shape)
        lib().oracle_pop_moment(self.d, self._Marr, _dp(f), _dp(phi))
        return phi

    def pop_step(self, f, omega1=None):
        omega1 = self.default_omega1() if omega1 is None else float(omega1)
        f = _f64(f).reshape((2 * self.d + 1,) + self.shape)
        out = np.empty_like(f)
        lib().oracle_pop_step(self.d, self._Marr, self.bc, omega1, self.relaxation(omega1),
                              self.dt, self.dx, _dp(f), _dp(out))
        return out

    def pop_run(self, f0, nsteps, omega1=None):
        omega1 = self.default_omega1() if omega1 is None else float(omega1)
        f = _f64(f0).reshape((2 * self.d + 1,) + self.shape).copy()
        lib().oracle_pop_run(self.d, self._Marr, self.bc, omega1, self.relaxation(omega1),
                             self.dt, self.dx, _dp(f), int(nsteps))
        return f

    def adjoint(self, phi0, nsteps, lambdaT):
        """(dL/dphi0, dL/dkappa, dL/d(eps^2)) for a given dL/dphi_T."""
        phi0 = _f64(phi0).reshape(self.shape)
        lam = _f64(lambdaT).reshape(self.shape)
        g = np.empty_like(phi0)
        gk = ctypes.c_double(0.0)
        rc = lib().oracle_adjoint(self.d, self._Marr, self.bc, self.kappa, self.dt,
                                  _dp(phi0), int(nsteps), _dp(lam), _dp(g), ctypes.byref(gk))
        if rc != 0:
            raise MemoryError("oracle_adjoint")
        # kappa = eps^2 dt / dx^2, so dL/d(eps^2) = (dt / dx^2) dL/dkappa
        return g, gk.value, gk.value * self.dt / (self.dx * self.dx)
