"""FP64 CPU oracle for the voxel cardiac-EP step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  The arithmetic
lives in ``ep_oracle.c`` (plain C, FP64); this wrapper only marshals numpy
arrays.  Problem instances come from :mod:`ep_inputs`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ep_oracle.c")
_LIB = os.path.join(_HERE, "libep_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Stim(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("center", C.c_double * 3),
                ("radius", C.c_double), ("amp", C.c_double), ("t_on", C.c_double),
                ("t_off", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("dt", C.c_double),
                ("theta", C.c_double), ("tau_in", C.c_double), ("tau_out", C.c_double),
                ("tau_open", C.c_double), ("tau_close", C.c_double), ("v_gate", C.c_double),
                ("exc", C.c_double), ("model", C.c_int32), ("diff", C.c_int32),
                ("cg_rtol", C.c_double), ("cg_maxit", C.c_int32), ("n_stim", C.c_int32),
                ("stim", C.POINTER(Stim)), ("mask", C.c_void_p), ("Di", C.c_void_p),
                ("De", C.c_void_p), ("jacobi_sweeps", C.c_int32), ("bath", C.c_void_p),
                ("sig_bath", C.c_double)]


class State(C.Structure):
    _fields_ = [("v", C.c_void_p), ("w", C.c_void_p), ("phi", C.c_void_p),
                ("tact", C.c_void_p), ("step", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("cg_iters", C.c_int64), ("cg_max", C.c_int32), ("cg_fail", C.c_int32),
                ("q_stim", C.c_double), ("mass", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _lib.orc_run.restype = C.c_int
        _lib.orc_solve_elliptic.restype = C.c_int
        _lib.orc_adjoint.restype = C.c_int
        _lib.orc_threads.restype = C.c_int
    return _lib


def threads() -> int:
    """Threads the oracle's OpenMP loops run with."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle's OpenMP loops on n threads from now on."""
    lib().orc_set_threads(C.c_int(int(n)))


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or '' if unknown."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _n3(n):
    return (C.c_int32 * 3)(*[int(k) for k in n])


def tensors(n, mask, fibre, scale, sig_l, sig_t):
    """Per-voxel conductivity tensors s*(sT I + (sL-sT) f f^T), shape (6, N)."""
    N = int(np.prod(n))
    D = np.zeros((6, N))
    fib = _f64(fibre).reshape(N, 3)
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    sc = None if scale is None else _f64(scale).ravel()
    lib().orc_tensors(_n3(n), _p(m), _p(fib), None if sc is None else _p(sc),
                      C.c_double(sig_l), C.c_double(sig_t), _p(D))
    return D


def apply(n, h, mask, D, v):
    """(A v) with the energy-form operator; returns an array shaped like v."""
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    vv = _f64(v).ravel()
    out = np.zeros_like(vv)
    lib().orc_apply(_n3(n), C.c_double(h), _p(m), _p(_f64(D)), _p(vv), _p(out))
    return out.reshape(np.shape(v))


def apply27(n, h, mask, D, v):
    """(A27 v) with the thesis's corner-gradient operator."""
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    vv = _f64(v).ravel()
    out = np.zeros_like(vv)
    lib().orc_apply27(_n3(n), C.c_double(h), _p(m), _p(_f64(D)), _p(vv), _p(out))
    return out.reshape(np.shape(v))


def diag(n, h, mask, D):
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    out = np.zeros(int(np.prod(n)))
    lib().orc_diag(_n3(n), C.c_double(h), _p(m), _p(_f64(D)), _p(out))
    return out.reshape(tuple(n))


def dA_ds(n, h, mask, D0, mu, v):
    """out_q = mu^T (dA/ds_q) v for voxel tensors s_q * D0_q."""
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    out = np.zeros(int(np.prod(n)))
    lib().orc_dA_ds(_n3(n), C.c_double(h), _p(m), _p(_f64(D0)), _p(_f64(mu).ravel()),
                    _p(_f64(v).ravel()), _p(out))
    return out.reshape(tuple(n))


def dense_matrix(n, h, mask, D, op=None):
    """Dense A (or of op, e.g. apply27) by applying the operator to unit
    vectors (tiny grids only)."""
    op = apply if op is None else op
    N = int(np.prod(n))
    A = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = op(n, h, mask, D, e.reshape(tuple(n))).ravel()
        e[j] = 0.0
    return A


class Oracle:
    """Holds one problem instance and its FP64 state, and advances it."""

    def __init__(self, inst, cg_rtol=1e-13, cg_maxit=20000, scale=None):
        self.inst = inst
        self.n = tuple(int(k) for k in inst.n)
        self.N = int(np.prod(self.n))
        self.mask = np.ascontiguousarray(inst.mask, dtype=np.uint8).ravel()
        sc = inst.scale if scale is None else scale
        self.Di = tensors(self.n, inst.mask, inst.fibre, sc, inst.sigma_l, inst.sigma_t)
        self.De = (tensors(self.n, inst.mask, inst.fibre, sc, inst.sigma_el, inst.sigma_et)
                   if inst.model == "bido" else None)
        st = inst.stims
        self._stims = (Stim * max(1, len(st)))()
        for k, s in enumerate(st):
            self._stims[k].lo[:] = [int(v) for v in s.lo]
            self._stims[k].hi[:] = [int(v) for v in s.hi]
            self._stims[k].center[:] = [float(v) for v in s.center]
            self._stims[k].radius = float(s.radius)
            self._stims[k].amp = float(s.amp)
            self._stims[k].t_on = float(s.t_on)
            self._stims[k].t_off = float(s.t_off)
        io = inst.ionic
        self.P = Problem()
        self.P.n[:] = list(self.n)
        self.P.h, self.P.dt, self.P.theta = inst.h, inst.dt, inst.theta
        self.P.tau_in, self.P.tau_out = io["tau_in"], io["tau_out"]
        self.P.tau_open, self.P.tau_close = io["tau_open"], io["tau_close"]
        self.P.v_gate, self.P.exc = io["v_gate"], io["exc"]
        self.P.model = 1 if inst.model == "bido" else 0
        self.P.diff = {"explicit": 0, "be_pcg": 1, "be_jacobi": 2,
                       "explicit27": 3}[inst.diff]
        self.P.jacobi_sweeps = int(getattr(inst, "jacobi_sweeps", 0))
        self.P.cg_rtol, self.P.cg_maxit = cg_rtol, cg_maxit
        self.P.n_stim = len(st)
        self.P.stim = C.cast(self._stims, C.POINTER(Stim))
        self.P.mask = _p(self.mask)
        self.P.Di = _p(self.Di)
        self.P.De = _p(self.De) if self.De is not None else None
        bath = getattr(inst, "bath", None)
        self.bath = (None if bath is None
                     else np.ascontiguousarray(bath, dtype=np.uint8).ravel())
        self.P.bath = _p(self.bath) if self.bath is not None else None
        self.P.sig_bath = float(getattr(inst, "sigma_bath", 0.0))
        m = inst.mask.astype(bool)
        self.v = np.zeros(self.N)
        self.w = np.where(m.ravel(), 1.0, 0.0)
        self.phi = np.zeros(self.N)
        self.tact = np.where(m.ravel(), np.inf, np.inf)
        self.step = 0
        self.last_info = None

    def set_state(self, v=None, w=None, phi=None, tact=None, step=None):
        m = self.mask.astype(bool)
        if v is not None:
            self.v = np.where(m, _f64(v).ravel(), 0.0)
        if w is not None:
            self.w = np.where(m, _f64(w).ravel(), 0.0)
        if phi is not None:
            dom = m if self.bath is None else (m | (self.bath > 0))
            self.phi = np.where(dom, _f64(phi).ravel(), 0.0)
        if tact is not None:
            self.tact = _f64(tact).ravel().copy()
        if step is not None:
            self.step = int(step)

    def run(self, nsteps):
        S = State(_p(self.v), _p(self.w), _p(self.phi), _p(self.tact), self.step)
        info = Info()
        rc = lib().orc_run(C.byref(self.P), C.byref(S), C.c_int32(nsteps), C.byref(info))
        self.step = int(S.step)
        self.last_info = info
        return rc, info

    def field(self, name):
        return getattr(self, name).reshape(self.n)

    def ionic(self, v, w, jstim=None):
        vs = np.zeros(self.N)
        ws = np.zeros(self.N)
        j = None if jstim is None else _f64(jstim).ravel()
        lib().orc_ionic(C.byref(self.P), _p(_f64(v).ravel()), _p(_f64(w).ravel()),
                        None if j is None else _p(j), _p(vs), _p(ws))
        return vs.reshape(self.n), ws.reshape(self.n)

    def solve_elliptic(self, b, phi0=None, rtol=1e-13, maxit=20000):
        phi = np.zeros(self.N) if phi0 is None else _f64(phi0).ravel().copy()
        it = lib().orc_solve_elliptic(C.byref(self.P), _p(_f64(b).ravel()), _p(phi),
                                      C.c_double(rtol), C.c_int(maxit))
        return phi.reshape(self.n), it

    def ecg(self, electrodes=None):
        """The six limb leads (I, II, III, aVR, aVL, aVF) from phi at the
        RA, LA, LL voxels."""
        e = self.inst.electrodes if electrodes is None else electrodes
        ee = (C.c_int32 * 9)(*[int(k) for xyz in e for k in xyz])
        out = np.zeros(6)
        lib().orc_ecg(_n3(self.n), _p(self.phi), ee, _p(out))
        return out

    def adjoint(self, D0, nsteps, tstar, v0=None, w0=None, step0=0):
        """Loss and gradient wrt the per-voxel scale (explicit monodomain)."""
        v0 = self.v if v0 is None else _f64(v0).ravel()
        w0 = self.w if w0 is None else _f64(w0).ravel()
        grad = np.zeros(self.N)
        tact = np.zeros(self.N)
        loss = C.c_double(0.0)
        used = C.c_int64(0)
        rc = lib().orc_adjoint(C.byref(self.P), _p(_f64(D0)), _p(_f64(v0)), _p(_f64(w0)),
                               C.c_int64(step0), C.c_int32(nsteps), _p(_f64(tstar).ravel()),
                               _p(grad), C.byref(loss), C.byref(used), _p(tact))
        if rc != 0:
            raise MemoryError("oracle adjoint: out of memory")
        return loss.value, grad.reshape(self.n), int(used.value), tact.reshape(self.n)
