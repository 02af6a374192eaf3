"""Python binding of libace.so (the C ABI in include/ace.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  Host arrays are numpy float64 in C order; device arrays are
torch tensors on the GPU (float64, contiguous), passed by pointer together
with torch's current HIP stream.  There is no CPU fallback: if the library
is missing, loading fails with an error.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libace.so")

ACE_OK = 0
ACE_E_ARG, ACE_E_SIZE, ACE_E_ANISO, ACE_E_DT = -1, -2, -3, -4
ACE_E_HIP, ACE_E_NOMEM, ACE_E_NONFINITE, ACE_E_STATE = -5, -6, -7, -8
ACE_W_CONDITIONS, ACE_W_PHI0_GT1, ACE_W_MAXPRINCIPLE, ACE_W_ENERGY_UP = 1, 2, 3, 4


def warn_bit(w):
    """Bit of warning w in a warning mask (ACE_WARN_BIT)."""
    return 1 << int(w)


ACE_BC_HN, ACE_BC_HD, ACE_BC_P = 0, 1, 2
BC = {"HN": ACE_BC_HN, "HD": ACE_BC_HD, "P": ACE_BC_P}
ACE_HOST, ACE_DEVICE = 0, 1
ACE_KERNEL_AUTO, ACE_KERNEL_DIRECT, ACE_KERNEL_MARCH = 0, 1, 2
ACE_KERNEL_RESIDENT, ACE_KERNEL_TBLOCK = 3, 4
ACE_SCHEME_RLB_MIE, ACE_SCHEME_FEX = 0, 1
ACE_POP_AUTO, ACE_POP_DIRECT, ACE_POP_FUSED, ACE_POP_SPLIT, ACE_POP_CARRY = 0, 1, 2, 3, 4

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_vp = ctypes.c_void_p
_P = ctypes.POINTER


class AceError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class Params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("bc", ctypes.c_int), ("N", _i64 * 3), ("M", _i64 * 3),
                ("total", _i64), ("dx", _dbl), ("dt", _dbl), ("eps", _dbl), ("kappa", _dbl),
                ("h", _dbl), ("dt_bound", _dbl), ("omega1", _dbl), ("s", _dbl),
                ("conditions_ok", ctypes.c_int), ("newton_iters", ctypes.c_int),
                ("scheme", ctypes.c_int)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class InstanceDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("bc", ctypes.c_int), ("N", _i64 * 3), ("L", _dbl * 3),
                ("R", _dbl * 3), ("eps", _dbl), ("dt", _dbl)]


_SIGS = {
    "ace_version": (ctypes.c_char_p, []),
    "ace_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ace_create": (ctypes.c_int, [ctypes.c_int, _P(_i64), _P(_dbl), _P(_dbl), _dbl, _dbl,
                                  ctypes.c_int, _P(_vp)]),
    "ace_destroy": (ctypes.c_int, [_vp]),
    "ace_shape": (ctypes.c_int, [_vp, _P(_i64), _P(_i64)]),
    "ace_node_coords": (ctypes.c_int, [_vp, ctypes.c_int, _P(_dbl)]),
    "ace_params": (ctypes.c_int, [_vp, _P(Params)]),
    "ace_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ace_bind_fields": (ctypes.c_int, [_vp, _vp, _vp]),
    "ace_set_kernel": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "ace_set_plane_chunk": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_set_region3d": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ace_get_region3d": (ctypes.c_int, [_vp, _P(ctypes.c_int), _P(ctypes.c_int), _P(ctypes.c_int)]),
    "ace_set_region2d": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "ace_get_region2d": (ctypes.c_int, [_vp, _P(ctypes.c_int), _P(ctypes.c_int)]),
    "ace_get_plane_chunk": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "ace_set_eps": (ctypes.c_int, [_vp, _dbl]),
    "ace_set_scheme": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_set_graph_launches": (ctypes.c_int, [_vp, _i64]),
    "ace_get_kernel": (ctypes.c_int, [_vp, _P(ctypes.c_int), _P(ctypes.c_int)]),
    "ace_set_phi0": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_step": (ctypes.c_int, [_vp, _i64]),
    "ace_run_monitored": (ctypes.c_int, [_vp, _i64, _i64, _P(_dbl), _P(_dbl)]),
    "ace_energy": (ctypes.c_int, [_vp, _P(_dbl)]),
    "ace_maxnorm": (ctypes.c_int, [_vp, _P(_dbl)]),
    "ace_get_phi": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_phase_volume": (ctypes.c_int, [_vp, _P(_dbl)]),
    "ace_equivalent_radius": (ctypes.c_int, [_vp, _P(_dbl)]),
    "ace_get_warnings": (ctypes.c_int, [_vp, _P(ctypes.c_int)]),
    "ace_monitor_status": (ctypes.c_int, [_i64, _P(_dbl), _P(_dbl), ctypes.c_int, _P(ctypes.c_int)]),
    "ace_monitor_noalloc": (ctypes.c_int, [_vp, _vp, _vp]),
    "ace_ckpt_generation": (_i64, [_vp]),
    "ace_step_count": (_i64, [_vp]),
    "ace_field_ptr": (_vp, [_vp]),
    "ace_adjoint": (ctypes.c_int, [_vp, _vp, _i64, _i64, _vp, _vp, _P(_dbl), ctypes.c_int]),
    "ace_forward_ckpt": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _i64, _i64]),
    "ace_backward": (ctypes.c_int, [_vp, _vp, _vp, _P(_dbl), ctypes.c_int]),
    "ace_batch_create": (ctypes.c_int, [ctypes.c_int, _P(InstanceDesc), _P(_vp), _P(ctypes.c_int)]),
    "ace_batch_destroy": (ctypes.c_int, [_vp]),
    "ace_batch_shape": (ctypes.c_int, [_vp, ctypes.c_int, _P(_i64), _P(_i64), _P(_i64)]),
    "ace_batch_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ace_batch_set_phi0": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "ace_batch_set_all": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_batch_step": (ctypes.c_int, [_vp, _i64]),
    "ace_batch_set_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_batch_set_region": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_batch_monitor": (ctypes.c_int, [_vp, _P(_dbl), _P(_dbl)]),
    "ace_batch_get_phi": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "ace_batch_get_all": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_batch_set_resident_limit": (ctypes.c_int, [_vp, _i64]),
    "ace_batch_set_depth": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_batch_autotune": (ctypes.c_int, [_vp, _i64, ctypes.c_char_p, ctypes.c_size_t]),
    "ace_autotune": (ctypes.c_int, [_vp, _i64, ctypes.c_char_p, ctypes.c_size_t]),
    "ace_pop_create": (ctypes.c_int, [ctypes.c_int, _P(_i64), _P(_dbl), _P(_dbl), _dbl, _dbl,
                                      ctypes.c_int, _dbl, _P(_vp)]),
    "ace_pop_destroy": (ctypes.c_int, [_vp]),
    "ace_pop_info": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(ctypes.c_int), _P(_dbl), _P(_dbl),
                                    _P(_i64)]),
    "ace_pop_set_stream": (ctypes.c_int, [_vp, _vp]),
    "ace_pop_set_kernel": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ace_pop_set_phi0": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_pop_set_populations": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_pop_get_populations": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_pop_step": (ctypes.c_int, [_vp, _i64]),
    "ace_pop_get_phi": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "ace_pop_step_count": (_i64, [_vp]),
}

_lib = None


def lib():
    """Loads libace.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2312_07010_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code):
    return lib().ace_strerror(int(code)).decode()


def _check(code, where):
    if code < 0:
        raise AceError(code, where)
    return code


def _host(a, n=None):
    """Contiguous float64 copy (or view) and its address; n: required size."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"array has {a.size} elements, {n} expected")
    return a, a.ctypes.data


def _is_device(x):
    return hasattr(x, "is_cuda") and x.is_cuda


def _dev(t, n=None):
    """Address of a contiguous float64 device tensor; n: required element
    count (the library reads or writes exactly that many)."""
    import torch
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous float64 tensors")
    if n is not None and t.numel() != n:
        raise ValueError(f"tensor has {t.numel()} elements, {n} expected")
    return t.data_ptr()


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Solver:
    """One problem of the paper (Sec. 1): d, N[], L[], R[], eps, dt, bc."""

    def __init__(self, d, N, L, R, eps, dt, bc):
        bc = BC[bc] if isinstance(bc, str) else int(bc)
        n = (_i64 * 3)(*[int(v) for v in list(N) + [1] * (3 - len(N))])
        lo = (_dbl * 3)(*[float(v) for v in list(L) + [0.0] * (3 - len(L))])
        hi = (_dbl * 3)(*[float(v) for v in list(R) + [1.0] * (3 - len(R))])
        h = _vp()
        self.status = _check(lib().ace_create(int(d), n, lo, hi, float(eps), float(dt), bc,
                                              ctypes.byref(h)), "ace_create")
        self._h = h
        M = (_i64 * 3)()
        tot = _i64()
        _check(lib().ace_shape(h, M, ctypes.byref(tot)), "ace_shape")
        self.d = int(d)
        self.shape = tuple(int(M[j]) for j in range(self.d))
        self.total = int(tot.value)
        self.last_status = self.status

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def params(self):
        p = Params()
        _check(lib().ace_params(self._h, ctypes.byref(p)), "ace_params")
        return p.as_dict()

    def coords(self, axis):
        x = np.empty(self.shape[axis])
        _check(lib().ace_node_coords(self._h, int(axis), x.ctypes.data_as(_P(_dbl))), "ace_node_coords")
        return x

    def set_stream(self, stream):
        _check(lib().ace_set_stream(self._h, stream), "ace_set_stream")

    def use_torch_stream(self):
        self.set_stream(current_stream())

    def bind_fields(self, a, b):
        pa = _dev(a, self.total) if a is not None else None
        pb = _dev(b, self.total) if b is not None else None
        _check(lib().ace_bind_fields(self._h, pa, pb), "ace_bind_fields")

    def set_eps(self, eps):
        self.last_status = _check(lib().ace_set_eps(self._h, float(eps)), "ace_set_eps")
        return self.last_status

    def set_scheme(self, scheme):
        self.last_status = _check(lib().ace_set_scheme(self._h, int(scheme)), "ace_set_scheme")
        return self.last_status

    def set_graph_launches(self, launches):
        _check(lib().ace_set_graph_launches(self._h, int(launches)), "ace_set_graph_launches")

    def set_kernel(self, kernel, depth=0):
        _check(lib().ace_set_kernel(self._h, int(kernel), int(depth)), "ace_set_kernel")

    def set_plane_chunk(self, planes):
        _check(lib().ace_set_plane_chunk(self._h, int(planes)), "ace_set_plane_chunk")

    def set_region3d(self, depth, rows=0, rows_per_thread=0):
        _check(lib().ace_set_region3d(self._h, int(depth), int(rows), int(rows_per_thread)),
               "ace_set_region3d")

    def get_region3d(self):
        """(depth, rows, rows per thread) of the 3D blocked kernel."""
        v = [ctypes.c_int() for _ in range(3)]
        _check(lib().ace_get_region3d(self._h, *[ctypes.byref(x) for x in v]), "ace_get_region3d")
        return tuple(x.value for x in v)

    def set_region2d(self, rows=0, rows_per_thread=0):
        _check(lib().ace_set_region2d(self._h, int(rows), int(rows_per_thread)), "ace_set_region2d")

    def get_region2d(self):
        """(rows, rows per thread) of the 2D blocked kernel ((0, 0): the LDS-plane kernel)."""
        v = [ctypes.c_int() for _ in range(2)]
        _check(lib().ace_get_region2d(self._h, *[ctypes.byref(x) for x in v]), "ace_get_region2d")
        return tuple(x.value for x in v)

    def get_plane_chunk(self):
        p = ctypes.c_int()
        _check(lib().ace_get_plane_chunk(self._h, ctypes.byref(p)), "ace_get_plane_chunk")
        return p.value

    def get_kernel(self):
        """(kernel id, steps per launch) that ace_step will use."""
        k = ctypes.c_int()
        n = ctypes.c_int()
        _check(lib().ace_get_kernel(self._h, ctypes.byref(k), ctypes.byref(n)), "ace_get_kernel")
        return k.value, n.value

    def set_phi0(self, phi0):
        if _is_device(phi0):
            rc = lib().ace_set_phi0(self._h, _dev(phi0, self.total), ACE_DEVICE)
        else:
            a, p = _host(phi0)
            if a.size != self.total:
                raise ValueError("phi0 has the wrong size")
            rc = lib().ace_set_phi0(self._h, p, ACE_HOST)
        self.last_status = _check(rc, "ace_set_phi0")
        return self.last_status

    def step(self, nsteps):
        self.last_status = _check(lib().ace_step(self._h, int(nsteps)), "ace_step")
        return self.last_status

    def run_monitored(self, nsteps, every):
        # invalid counts go to the library, which rejects them (ACE_E_ARG)
        n = int(nsteps) // int(every) + 1 if int(every) >= 1 and int(nsteps) >= 0 else 1
        E = np.empty(n)
        mx = np.empty(n)
        rc = lib().ace_run_monitored(self._h, int(nsteps), int(every), E.ctypes.data_as(_P(_dbl)),
                                     mx.ctypes.data_as(_P(_dbl)))
        self.last_status = _check(rc, "ace_run_monitored")
        return E, mx

    def energy(self):
        v = _dbl()
        _check(lib().ace_energy(self._h, ctypes.byref(v)), "ace_energy")
        return v.value

    def maxnorm(self):
        v = _dbl()
        _check(lib().ace_maxnorm(self._h, ctypes.byref(v)), "ace_maxnorm")
        return v.value

    def phase_volume(self):
        v = _dbl()
        _check(lib().ace_phase_volume(self._h, ctypes.byref(v)), "ace_phase_volume")
        return v.value

    def equivalent_radius(self):
        """Radius of the disc (d = 2) or ball (d = 3) holding the phase volume
        (half the phase length for d = 1)."""
        v = _dbl()
        _check(lib().ace_equivalent_radius(self._h, ctypes.byref(v)), "ace_equivalent_radius")
        return v.value

    def warnings(self):
        """Mask of every warning the last run_monitored saw (warn_bit)."""
        m = ctypes.c_int()
        _check(lib().ace_get_warnings(self._h, ctypes.byref(m)), "ace_get_warnings")
        return m.value

    def monitor_noalloc(self, out, phi=None):
        """Energy and max-norm into the device tensor out[0:2] (float64),
        stream-ordered, allocating nothing; phi: a device field of the
        handle's shape, or None for the current field."""
        po = _dev(out, 2)
        pf = _dev(phi, self.total) if phi is not None else None
        _check(lib().ace_monitor_noalloc(self._h, pf, po), "ace_monitor_noalloc")
        return out

    def get_phi(self, out=None):
        if out is not None and _is_device(out):
            _check(lib().ace_get_phi(self._h, _dev(out, self.total), ACE_DEVICE), "ace_get_phi")
            return out
        a = np.empty(self.shape)
        _check(lib().ace_get_phi(self._h, a.ctypes.data, ACE_HOST), "ace_get_phi")
        return a

    @property
    def step_count(self):
        return int(lib().ace_step_count(self._h))

    def field_ptr(self):
        return lib().ace_field_ptr(self._h)

    # reverse mode ---------------------------------------------------------
    def forward_ckpt(self, phi0, nsteps, ckpt_every):
        if _is_device(phi0):
            rc = lib().ace_forward_ckpt(self._h, _dev(phi0, self.total), ACE_DEVICE, int(nsteps),
                                        int(ckpt_every))
        else:
            a, p = _host(phi0, self.total)
            rc = lib().ace_forward_ckpt(self._h, p, ACE_HOST, int(nsteps), int(ckpt_every))
        return _check(rc, "ace_forward_ckpt")

    @property
    def ckpt_generation(self):
        return int(lib().ace_ckpt_generation(self._h))

    def backward(self, lambdaT, dphi0=None):
        g = _dbl()
        if _is_device(lambdaT):
            import torch
            out = dphi0 if dphi0 is not None else torch.empty_like(lambdaT)
            rc = lib().ace_backward(self._h, _dev(lambdaT, self.total), _dev(out, self.total),
                                    ctypes.byref(g), ACE_DEVICE)
        else:
            lam, p = _host(lambdaT, self.total)
            out = np.empty(self.shape)
            rc = lib().ace_backward(self._h, p, out.ctypes.data, ctypes.byref(g), ACE_HOST)
        _check(rc, "ace_backward")
        return out, g.value

    def adjoint(self, phi0, nsteps, ckpt_every, lambdaT):
        """Host arrays in, (dL/dphi0, dL/d(eps^2)) out."""
        a, pa = _host(phi0, self.total)
        lam, pl = _host(lambdaT, self.total)
        out = np.empty(self.shape)
        g = _dbl()
        rc = lib().ace_adjoint(self._h, pa, int(nsteps), int(ckpt_every), pl, out.ctypes.data,
                               ctypes.byref(g), ACE_HOST)
        _check(rc, "ace_adjoint")
        return out, g.value

    def autotune(self, trial_steps=20):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().ace_autotune(self._h, int(trial_steps), buf, 1 << 16), "ace_autotune")
        return buf.value.decode()


def monitor_status(E, maxn, conditions_ok=True):
    """The library's check of a monitor series (host only): (status, mask)."""
    E, _ = _host(E)
    mx, _ = _host(maxn, E.size)
    m = ctypes.c_int()
    rc = lib().ace_monitor_status(E.size, E.ctypes.data_as(_P(_dbl)), mx.ctypes.data_as(_P(_dbl)),
                                  int(bool(conditions_ok)), ctypes.byref(m))
    return rc, m.value


class Batch:
    """Many independent 1D/2D instances stepped by one persistent launch.

    instances: sequence of (d, N, L, R, eps, dt, bc) tuples (N, L, R per axis).
    """

    def __init__(self, instances):
        n = len(instances)
        descs = (InstanceDesc * n)()
        for i, (d, N, L, R, eps, dt, bc) in enumerate(instances):
            D = descs[i]
            D.d = int(d)
            D.bc = BC[bc] if isinstance(bc, str) else int(bc)
            for j in range(3):
                D.N[j] = int(N[j]) if j < len(N) else 1
                D.L[j] = float(L[j]) if j < len(L) else 0.0
                D.R[j] = float(R[j]) if j < len(R) else 1.0
            D.eps = float(eps)
            D.dt = float(dt)
        st = (ctypes.c_int * n)()
        h = _vp()
        rc = lib().ace_batch_create(n, descs, ctypes.byref(h), st)
        self.status = list(st)
        _check(rc, "ace_batch_create")
        self._h = h
        self.count = n
        self.shapes, self.totals, self.offsets = [], [], []
        for i in range(n):
            M = (_i64 * 3)()
            tot = _i64()
            off = _i64()
            _check(lib().ace_batch_shape(h, i, M, ctypes.byref(tot), ctypes.byref(off)), "ace_batch_shape")
            d = int(instances[i][0])
            self.shapes.append(tuple(int(M[j]) for j in range(d)))
            self.totals.append(int(tot.value))
            self.offsets.append(int(off.value))

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(lib().ace_batch_set_stream(self._h, stream), "ace_batch_set_stream")

    def use_torch_stream(self):
        self.set_stream(current_stream())

    def set_phi0(self, i, phi0):
        a, p = _host(phi0)
        if a.size != self.totals[i]:
            raise ValueError("phi0 has the wrong size")
        return _check(lib().ace_batch_set_phi0(self._h, int(i), p, ACE_HOST), "ace_batch_set_phi0")

    def set_all(self, fields):
        flat = np.concatenate([np.ascontiguousarray(f, dtype=np.float64).ravel() for f in fields])
        if flat.size != sum(self.totals):
            raise ValueError("fields have the wrong total size")
        return _check(lib().ace_batch_set_all(self._h, flat.ctypes.data, ACE_HOST), "ace_batch_set_all")

    def step(self, nsteps):
        return _check(lib().ace_batch_step(self._h, int(nsteps)), "ace_batch_step")

    def monitor(self):
        E = np.empty(self.count)
        mx = np.empty(self.count)
        _check(lib().ace_batch_monitor(self._h, E.ctypes.data_as(_P(_dbl)), mx.ctypes.data_as(_P(_dbl))),
               "ace_batch_monitor")
        return E, mx

    def get_phi(self, i):
        a = np.empty(self.shapes[i])
        _check(lib().ace_batch_get_phi(self._h, int(i), a.ctypes.data, ACE_HOST), "ace_batch_get_phi")
        return a

    def get_all(self):
        flat = np.empty(sum(self.totals))
        _check(lib().ace_batch_get_all(self._h, flat.ctypes.data, ACE_HOST), "ace_batch_get_all")
        out, o = [], 0
        for shp, t in zip(self.shapes, self.totals):
            out.append(flat[o:o + t].reshape(shp))
            o += t
        return out

    def set_resident_limit(self, limit):
        _check(lib().ace_batch_set_resident_limit(self._h, int(limit)), "ace_batch_set_resident_limit")

    def set_depth(self, depth):
        _check(lib().ace_batch_set_depth(self._h, int(depth)), "ace_batch_set_depth")

    def set_region(self, rows):
        _check(lib().ace_batch_set_region(self._h, int(rows)), "ace_batch_set_region")

    def set_graphs(self, enable):
        _check(lib().ace_batch_set_graphs(self._h, int(bool(enable))), "ace_batch_set_graphs")

    def autotune(self, trial_steps=20):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().ace_batch_autotune(self._h, int(trial_steps), buf, 1 << 16), "ace_batch_autotune")
        return buf.value.decode()


class Pop:
    """The mesoscopic form (Sec. 2): 2d+1 populations per node under the
    regularized evolution equation.  omega1 = 0 selects the weights of the
    paper's experiments (1/3, 1/5, 1/6 for d = 1, 2, 3)."""

    def __init__(self, d, N, L, R, eps, dt, bc, omega1=0.0):
        bc = BC[bc] if isinstance(bc, str) else int(bc)
        n = (_i64 * 3)(*[int(v) for v in list(N) + [1] * (3 - len(N))])
        lo = (_dbl * 3)(*[float(v) for v in list(L) + [0.0] * (3 - len(L))])
        hi = (_dbl * 3)(*[float(v) for v in list(R) + [1.0] * (3 - len(R))])
        h = _vp()
        self.status = _check(lib().ace_pop_create(int(d), n, lo, hi, float(eps), float(dt), bc,
                                                  float(omega1), ctypes.byref(h)), "ace_pop_create")
        self._h = h
        M = (_i64 * 3)()
        tot = _i64()
        q = ctypes.c_int()
        w1 = _dbl()
        sr = _dbl()
        nb = _i64()
        _check(lib().ace_pop_info(h, M, ctypes.byref(tot), ctypes.byref(q), ctypes.byref(w1),
                                  ctypes.byref(sr), ctypes.byref(nb)), "ace_pop_info")
        self.d = int(d)
        self.shape = tuple(int(M[j]) for j in range(self.d))
        self.total = int(tot.value)
        self.q = int(q.value)
        self.omega1 = float(w1.value)
        self.s = float(sr.value)
        self.device_bytes = int(nb.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_pop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(lib().ace_pop_set_stream(self._h, _vp(stream)), "ace_pop_set_stream")

    def use_torch_stream(self):
        self.set_stream(current_stream())

    def set_kernel(self, kernel):
        _check(lib().ace_pop_set_kernel(self._h, int(kernel)), "ace_pop_set_kernel")

    def set_phi0(self, phi0):
        if _is_device(phi0):
            rc = lib().ace_pop_set_phi0(self._h, _dev(phi0, self.total), ACE_DEVICE)
        else:
            a, p = _host(phi0)
            if a.size != self.total:
                raise ValueError("phi0 has the wrong size")
            rc = lib().ace_pop_set_phi0(self._h, p, ACE_HOST)
        return _check(rc, "ace_pop_set_phi0")

    def set_populations(self, f):
        if _is_device(f):
            return _check(lib().ace_pop_set_populations(self._h, _dev(f, self.q * self.total), ACE_DEVICE),
                          "ace_pop_set_populations")
        a, p = _host(f)
        if a.size != self.q * self.total:
            raise ValueError("populations have the wrong size")
        return _check(lib().ace_pop_set_populations(self._h, p, ACE_HOST), "ace_pop_set_populations")

    def get_populations(self, out=None):
        if out is not None and _is_device(out):
            _check(lib().ace_pop_get_populations(self._h, _dev(out, self.q * self.total), ACE_DEVICE),
                   "ace_pop_get_populations")
            return out
        a = np.empty((self.q,) + self.shape)
        _check(lib().ace_pop_get_populations(self._h, a.ctypes.data, ACE_HOST), "ace_pop_get_populations")
        return a

    def step(self, nsteps):
        return _check(lib().ace_pop_step(self._h, int(nsteps)), "ace_pop_step")

    def get_phi(self, out=None):
        if out is not None and _is_device(out):
            _check(lib().ace_pop_get_phi(self._h, _dev(out, self.total), ACE_DEVICE), "ace_pop_get_phi")
            return out
        a = np.empty(self.shape)
        _check(lib().ace_pop_get_phi(self._h, a.ctypes.data, ACE_HOST), "ace_pop_get_phi")
        return a

    @property
    def step_count(self):
        return int(lib().ace_pop_step_count(self._h))
