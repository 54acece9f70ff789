"""ctypes binding of the HIP voxel-EP library (include/ep.h).

Argument marshalling only: every step of the method runs in the HIP library
``libep_hip.so`` built in this package directory.  If the library is missing
the import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch ships its own HIP runtime.  When this library's runtime (ROCm from
# /opt/rocm) is loaded into a process before torch's, and torch then
# initialises the device, this library's first HIP call finds no device; in
# the opposite order both work.  Load torch first whenever it is installed.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is optional for the binding
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libep_hip.so")

EP_OK, EP_ERR_ARG, EP_ERR_OOM, EP_ERR_HIP, EP_ERR_NOCONV, EP_ERR_NONFINITE, EP_ERR_STATE, \
    EP_ERR_UNSUPPORTED = range(8)
EP_F64, EP_F32 = 0, 1
EP_MONO, EP_BIDO = 0, 1
EP_DIFF_EXPLICIT, EP_DIFF_BE_PCG, EP_DIFF_BE_JACOBI, EP_DIFF_EXPLICIT27 = 0, 1, 2, 3
FIELDS = {"v": 0, "w": 1, "phi": 2, "tact": 3}
KERNELS = {"stencil": 0, "cg_setup": 1, "parabolic": 2, "resid": 3, "cg_tail": 4, "adjoint": 5,
           "be_init": 6, "cg_update": 7, "coarse": 8, "multistep": 9}


class EPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Ionic(C.Structure):
    _fields_ = [("tau_in", C.c_double), ("tau_out", C.c_double), ("tau_open", C.c_double),
                ("tau_close", C.c_double), ("v_gate", C.c_double), ("exc", C.c_double)]


class Stim(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("center", C.c_double * 3),
                ("radius", C.c_double), ("amp", C.c_double), ("t_on", C.c_double),
                ("t_off", C.c_double)]


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("mask", C.c_void_p),
                ("model", C.c_int), ("prec", C.c_int), ("diff", C.c_int), ("dt", C.c_double),
                ("ionic", Ionic), ("stim", C.POINTER(Stim)), ("n_stim", C.c_int32),
                ("act_threshold", C.c_double), ("pcg_rtol", C.c_double),
                ("pcg_maxit", C.c_int32), ("jacobi_sweeps", C.c_int32), ("ell_rtol", C.c_double),
                ("ell_max_outer", C.c_int32), ("ell_inner_maxit", C.c_int32),
                ("stream", C.c_void_p), ("arena", C.c_void_p), ("arena_bytes", C.c_int64),
                ("bath", C.c_void_p), ("sig_bath", C.c_double), ("ell_precond", C.c_int32),
                ("persistent_blocks", C.c_int32), ("steps_per_launch", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("step", C.c_int64), ("t", C.c_double),
                ("cg_iters", C.c_int64), ("cg_max", C.c_int32), ("ell_outer", C.c_int32),
                ("q_stim", C.c_double), ("mass", C.c_double), ("relres", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("outer", C.c_int32), ("inner_iters", C.c_int64), ("relres", C.c_double),
                ("precond", C.c_int32)]


class BatchDesc(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_slots", C.c_int32),
                ("steps_per_launch", C.c_int32), ("stream", C.c_void_p)]


class BatchStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("finished", C.c_int64),
                ("released", C.c_int64), ("resident", C.c_int32), ("queued", C.c_int32),
                ("arena_used", C.c_int64), ("arena_peak", C.c_int64),
                ("graph_launches", C.c_int64), ("voxel_steps", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.ep_create_grid.argtypes = [C.POINTER(GridDesc), C.POINTER(vp)]
    lib.ep_set_conductivity_fibres.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                               C.c_double]
    lib.ep_set_conductivity_fibres_noalloc.argtypes = [vp, vp, vp, C.c_double, C.c_double,
                                                       C.c_double, C.c_double]
    lib.ep_step.argtypes = [vp, C.c_int32, C.POINTER(StepInfo)]
    lib.ep_solve_elliptic.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(SolveInfo)]
    lib.ep_read_state.argtypes = [vp, C.c_int, vp, C.c_size_t]
    lib.ep_read_state_device.argtypes = [vp, C.c_int, vp, C.c_int32]
    lib.ep_write_state.argtypes = [vp, C.c_int, vp, C.c_size_t]
    lib.ep_ecg_leads.argtypes = [vp, vp, vp]
    lib.ep_get_step.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.ep_set_step.argtypes = [vp, C.c_int64]
    lib.ep_grid_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]
    lib.ep_kernel_timing.argtypes = [vp, C.c_int32]
    lib.ep_kernel_time.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.ep_kernel_timing_period.argtypes = [vp, C.c_int32]
    lib.ep_adjoint_scale.argtypes = [vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_double), vp,
                                     C.POINTER(C.c_int64)]
    lib.ep_stream_bandwidth.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
    lib.ep_destroy_grid.argtypes = [vp]
    lib.ep_status_string.argtypes = [C.c_int]
    lib.ep_status_string.restype = C.c_char_p
    lib.ep_last_error.argtypes = [vp]
    lib.ep_last_error.restype = C.c_char_p
    lib.ep_batch_create.argtypes = [C.POINTER(BatchDesc), C.POINTER(vp)]
    lib.ep_batch_submit.argtypes = [vp, C.POINTER(GridDesc), vp, vp, C.c_double, C.c_double,
                                    C.c_int64, C.POINTER(C.c_int64)]
    lib.ep_batch_advance.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.ep_batch_finished.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32,
                                      C.POINTER(C.c_int32)]
    lib.ep_batch_read.argtypes = [vp, C.c_int64, C.c_int, vp, C.c_size_t]
    lib.ep_batch_release.argtypes = [vp, C.c_int64]
    lib.ep_batch_get_stats.argtypes = [vp, C.POINTER(BatchStats)]
    lib.ep_batch_destroy.argtypes = [vp]
    lib.ep_batch_last_error.argtypes = [vp]
    lib.ep_batch_last_error.restype = C.c_char_p
    for name in ("ep_create_grid", "ep_set_conductivity_fibres",
                 "ep_set_conductivity_fibres_noalloc", "ep_step", "ep_solve_elliptic",
                 "ep_read_state", "ep_read_state_device", "ep_write_state", "ep_ecg_leads",
                 "ep_get_step",
                 "ep_set_step",
                 "ep_grid_stats", "ep_kernel_timing", "ep_kernel_timing_period",
                 "ep_kernel_time", "ep_destroy_grid",
                 "ep_adjoint_scale", "ep_stream_bandwidth",
                 "ep_batch_create", "ep_batch_submit", "ep_batch_advance", "ep_batch_finished",
                 "ep_batch_read", "ep_batch_release", "ep_batch_get_stats", "ep_batch_destroy"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def make_desc(n, h, dt, mask=None, model="mono", prec="f32", diff="explicit", ionic=None,
              stims=(), theta=0.5, pcg_rtol=1e-6, pcg_maxit=50, ell_rtol=1e-8,
              ell_max_outer=8, ell_inner_maxit=4000, stream=None, arena=None,
              jacobi_sweeps=10, bath=None, sig_bath=0.0, ell_precond=0,
              persistent_blocks=0, steps_per_launch=0):
    """Fill an ep_grid_desc; returns it and the arrays it points into (keep
    them alive while the descriptor is used).  arena: optional caller-owned
    device memory, a torch CUDA tensor whose bytes the grid carves its
    arrays from (kept alive by the returned list)."""
    n = tuple(int(k) for k in n)
    N = int(np.prod(n))
    d = GridDesc()
    d.n[:] = list(n)
    d.h = float(h)
    keep = []
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
        if m.size != N:
            raise ValueError("mask size does not match n")
        keep.append(m)
        d.mask = _p(m)
    d.model = EP_BIDO if model == "bido" else EP_MONO
    d.prec = EP_F64 if prec == "f64" else EP_F32
    d.diff = {"explicit": EP_DIFF_EXPLICIT, "be_pcg": EP_DIFF_BE_PCG,
              "be_jacobi": EP_DIFF_BE_JACOBI, "explicit27": EP_DIFF_EXPLICIT27}[diff]
    d.dt = float(dt)
    keys = ("tau_in", "tau_out", "tau_open", "tau_close", "v_gate", "exc")
    if ionic is None or any(k not in ionic for k in keys):
        raise ValueError(f"ionic must give {', '.join(keys)}")
    for k in keys:
        setattr(d.ionic, k, float(ionic[k]))
    stims = list(stims)
    arr = (Stim * max(1, len(stims)))()
    for k, s in enumerate(stims):
        arr[k].lo[:] = [int(v) for v in s.lo]
        arr[k].hi[:] = [int(v) for v in s.hi]
        arr[k].center[:] = [float(v) for v in s.center]
        arr[k].radius = float(s.radius)
        arr[k].amp = float(s.amp)
        arr[k].t_on = float(s.t_on)
        arr[k].t_off = float(s.t_off)
    keep.append(arr)
    d.stim = C.cast(arr, C.POINTER(Stim))
    d.n_stim = len(stims)
    d.act_threshold = float(theta)
    d.pcg_rtol, d.pcg_maxit = float(pcg_rtol), int(pcg_maxit)
    d.jacobi_sweeps = int(jacobi_sweeps)
    d.ell_rtol, d.ell_max_outer = float(ell_rtol), int(ell_max_outer)
    d.ell_inner_maxit = int(ell_inner_maxit)
    d.stream = stream
    if arena is not None:
        if not getattr(arena, "is_cuda", False) or not arena.is_contiguous():
            raise ValueError("arena must be a contiguous CUDA tensor")
        keep.append(arena)
        d.arena = C.c_void_p(arena.data_ptr())
        d.arena_bytes = int(arena.numel() * arena.element_size())
    if bath is not None:
        b = np.ascontiguousarray(bath, dtype=np.uint8).ravel()
        if b.size != N:
            raise ValueError("bath size does not match n")
        keep.append(b)
        d.bath = _p(b)
        d.sig_bath = float(sig_bath)
    d.ell_precond = int(ell_precond)
    d.persistent_blocks = int(persistent_blocks)
    d.steps_per_launch = int(steps_per_launch)
    return d, keep


def stream_bandwidth(nbytes=1 << 30, reps=5):
    """ep_stream_bandwidth: (copy GB/s, read-only GB/s) of plain HIP kernels
    over `nbytes` buffers on the current device."""
    cp, rd = C.c_double(), C.c_double()
    st = lib.ep_stream_bandwidth(int(nbytes), int(reps), C.byref(cp), C.byref(rd))
    if st != EP_OK:
        raise EPError(st, "ep_stream_bandwidth: " + lib.ep_status_string(st).decode())
    return cp.value, rd.value


class Grid:
    """One simulation grid on the GPU (see include/ep.h for the semantics)."""

    def __init__(self, n, h, dt, mask=None, model="mono", prec="f32", diff="explicit",
                 ionic=None, stims=(), theta=0.5, pcg_rtol=1e-6, pcg_maxit=50,
                 ell_rtol=1e-8, ell_max_outer=8, ell_inner_maxit=4000, stream=None,
                 arena=None, jacobi_sweeps=10, bath=None, sig_bath=0.0, ell_precond=0,
                 persistent_blocks=0, steps_per_launch=0):
        self._desc, keep = make_desc(n, h, dt, mask, model, prec, diff, ionic, stims, theta,
                                     pcg_rtol, pcg_maxit, ell_rtol, ell_max_outer,
                                     ell_inner_maxit, stream, arena, jacobi_sweeps, bath,
                                     sig_bath, ell_precond, persistent_blocks,
                                     steps_per_launch)
        self._keep = keep
        self.n = tuple(int(k) for k in n)
        self.N = int(np.prod(self.n))
        self._h = C.c_void_p()
        self._check(lib.ep_create_grid(C.byref(self._desc), C.byref(self._h)), "ep_create_grid",
                    handle=False)

    @classmethod
    def from_instance(cls, inst, prec=None, **kw):
        """Create from a problem-instance object (attributes n, h, dt, mask,
        model, prec, diff, ionic, stims, theta, tolerances) and set its
        conductivity."""
        g = cls(inst.n, inst.h, inst.dt, mask=inst.mask, model=inst.model,
                prec=prec or inst.prec, diff=inst.diff, ionic=inst.ionic, stims=inst.stims,
                theta=inst.theta, pcg_rtol=inst.pcg_rtol, pcg_maxit=inst.pcg_maxit,
                ell_rtol=inst.ell_rtol,
                jacobi_sweeps=getattr(inst, "jacobi_sweeps", 10),
                bath=getattr(inst, "bath", None), sig_bath=getattr(inst, "sigma_bath", 0.0),
                **kw)
        try:
            g.set_conductivity(inst.fibre, inst.scale, inst.sigma_l, inst.sigma_t,
                               inst.sigma_el, inst.sigma_et)
        except Exception:
            g.close()
            raise
        return g

    def _check(self, st, what, handle=True):
        if st != EP_OK:
            msg = lib.ep_last_error(self._h if handle else None).decode()
            name = lib.ep_status_string(st).decode()
            raise EPError(st, f"{what}: {name} {msg}".strip())

    def set_conductivity(self, fibre, scale, sig_l, sig_t, sig_el=0.0, sig_et=0.0):
        f = np.ascontiguousarray(fibre, dtype=np.float64).reshape(self.N * 3)
        s = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64).ravel()
        self._check(lib.ep_set_conductivity_fibres(self._h, _p(f), None if s is None else _p(s),
                                                   sig_l, sig_t, sig_el, sig_et),
                    "ep_set_conductivity_fibres")

    def set_conductivity_noalloc(self, fibre, scale, sig_l, sig_t, sig_el=0.0, sig_et=0.0):
        """ep_set_conductivity_fibres_noalloc: the same set-up with its device
        temporaries in the library's fixed scratch (no device allocation)."""
        f = np.ascontiguousarray(fibre, dtype=np.float64).reshape(self.N * 3)
        s = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64).ravel()
        self._check(lib.ep_set_conductivity_fibres_noalloc(
            self._h, _p(f), None if s is None else _p(s), sig_l, sig_t, sig_el, sig_et),
            "ep_set_conductivity_fibres_noalloc")

    def step(self, nsteps, check=True):
        info = StepInfo()
        st = lib.ep_step(self._h, int(nsteps), C.byref(info))
        if check:
            self._check(st, "ep_step")
        out = {k: getattr(info, k) for k, _ in StepInfo._fields_}
        out["status"] = st
        return out

    def solve_elliptic(self, rtol=1e-8, max_outer=8, check=True):
        info = SolveInfo()
        st = lib.ep_solve_elliptic(self._h, float(rtol), int(max_outer), C.byref(info))
        if check:
            self._check(st, "ep_solve_elliptic")
        out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        out["status"] = st
        return out

    def adjoint_scale(self, tstar, nsteps, ckpt_every=0, grad=True):
        """Run ``nsteps`` explicit steps with a fresh T_act and return
        (loss, dL/dscale in box layout, voxels in the loss); with
        ``grad=False`` only the forward run and the loss (gradient None)."""
        t = np.ascontiguousarray(tstar, dtype=np.float64).ravel()
        if t.size != self.N:
            raise ValueError("tstar size does not match n")
        g = np.empty(self.N, dtype=np.float64) if grad else None
        loss, used = C.c_double(), C.c_int64()
        self._check(lib.ep_adjoint_scale(self._h, int(nsteps), int(ckpt_every), _p(t),
                                         C.byref(loss), None if g is None else _p(g),
                                         C.byref(used)),
                    "ep_adjoint_scale")
        return loss.value, (None if g is None else g.reshape(self.n)), used.value

    def read(self, field):
        out = np.empty(self.N, dtype=np.float64)
        self._check(lib.ep_read_state(self._h, FIELDS[field], _p(out), self.N), "ep_read_state")
        return out.reshape(self.n)

    def read_tensor(self, field, dtype=None):
        """The field as a torch tensor on the GPU (box layout, shape n),
        copied device to device by the library; FP32 unless dtype is
        torch.float64.  Waits for the copy before returning."""
        import torch
        dtype = torch.float32 if dtype is None else dtype
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        out = torch.empty(self.n, dtype=dtype, device="cuda")
        self._check(lib.ep_read_state_device(self._h, FIELDS[field], C.c_void_p(out.data_ptr()),
                                             0 if dtype == torch.float64 else 1),
                    "ep_read_state_device")
        torch.cuda.synchronize()
        return out

    def write(self, field, values):
        a = np.ascontiguousarray(values, dtype=np.float64).ravel()
        if a.size != self.N:
            raise ValueError("size mismatch")
        self._check(lib.ep_write_state(self._h, FIELDS[field], _p(a), self.N), "ep_write_state")

    @property
    def step_index(self):
        s = C.c_int64()
        self._check(lib.ep_get_step(self._h, C.byref(s)), "ep_get_step")
        return s.value

    @step_index.setter
    def step_index(self, v):
        self._check(lib.ep_set_step(self._h, int(v)), "ep_set_step")

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib.ep_grid_stats(self._h, C.byref(a), C.byref(b), C.byref(c)),
                    "ep_grid_stats")
        return {"n_tissue": a.value, "n_bricks": b.value, "device_bytes": c.value}

    def ecg(self, electrodes):
        """Leads I, II, III, aVR, aVL, aVF from phi at the RA, LA, LL voxels
        (three (x, y, z) triples)."""
        e = np.ascontiguousarray(np.asarray(electrodes, dtype=np.int32).reshape(9))
        out = np.zeros(6)
        self._check(lib.ep_ecg_leads(self._h, _p(e), _p(out)), "ep_ecg_leads")
        return out

    def kernel_timing(self, enable=True, kernels=None, every=1):
        """Time launches with HIP events: all kernels, or only those named in
        `kernels` (keys of KERNELS), in every step or (every > 1) only in
        the steps whose index is a multiple of `every`; resets the totals."""
        self._check(lib.ep_kernel_timing_period(self._h, int(every)), "ep_kernel_timing_period")
        if not enable:
            mask = 0
        elif kernels is None:
            mask = -1
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNELS[k]
        self._check(lib.ep_kernel_timing(self._h, mask), "ep_kernel_timing")

    def kernel_time(self, kernel):
        ms, cnt = C.c_double(), C.c_int64()
        self._check(lib.ep_kernel_time(self._h, KERNELS[kernel], C.byref(ms), C.byref(cnt)),
                    "ep_kernel_time")
        return ms.value, cnt.value

    def close(self):
        if self._h:
            lib.ep_destroy_grid(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Continuous-batching server state on the GPU (ep_batch_* of include/ep.h)."""

    def __init__(self, hbm_budget, max_slots=64, steps_per_launch=16, stream=None):
        d = BatchDesc(int(hbm_budget), int(max_slots), int(steps_per_launch), stream)
        self._b = C.c_void_p()
        st = lib.ep_batch_create(C.byref(d), C.byref(self._b))
        if st != EP_OK:
            raise EPError(st, f"ep_batch_create: {lib.ep_status_string(st).decode()}")
        self._sizes = {}

    def _check(self, st, what):
        if st != EP_OK:
            raise EPError(st, f"{what}: {lib.ep_status_string(st).decode()} "
                              f"{lib.ep_batch_last_error(self._b).decode()}".strip())

    def submit(self, n, h, dt, mask, ionic, stims, theta, fibre, scale, sig_l, sig_t, n_steps):
        d, keep = make_desc(n, h, dt, mask, "mono", "f32", "explicit", ionic, stims, theta)
        N = int(np.prod(n))
        f = np.ascontiguousarray(fibre, dtype=np.float64).reshape(N * 3)
        sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64).ravel()
        rid = C.c_int64()
        self._check(lib.ep_batch_submit(self._b, C.byref(d), _p(f), None if sc is None else _p(sc),
                                        float(sig_l), float(sig_t), int(n_steps), C.byref(rid)),
                    "ep_batch_submit")
        self._sizes[rid.value] = tuple(int(k) for k in n)
        return rid.value

    def submit_instance(self, inst, n_steps=None):
        return self.submit(inst.n, inst.h, inst.dt, inst.mask, inst.ionic, inst.stims, inst.theta,
                           inst.fibre, inst.scale, inst.sigma_l, inst.sigma_t,
                           inst.steps if n_steps is None else n_steps)

    def advance(self):
        nf = C.c_int32()
        self._check(lib.ep_batch_advance(self._b, C.byref(nf)), "ep_batch_advance")
        return nf.value

    def finished(self, cap=1024):
        ids = (C.c_int64 * cap)()
        n = C.c_int32()
        self._check(lib.ep_batch_finished(self._b, ids, cap, C.byref(n)), "ep_batch_finished")
        return [ids[i] for i in range(n.value)]

    def read(self, rid, field):
        n = self._sizes[rid]
        out = np.empty(int(np.prod(n)), dtype=np.float64)
        self._check(lib.ep_batch_read(self._b, int(rid), FIELDS[field], _p(out), out.size),
                    "ep_batch_read")
        return out.reshape(n)

    def release(self, rid):
        self._check(lib.ep_batch_release(self._b, int(rid)), "ep_batch_release")
        self._sizes.pop(rid, None)

    def stats(self):
        s = BatchStats()
        self._check(lib.ep_batch_get_stats(self._b, C.byref(s)), "ep_batch_get_stats")
        return {k: getattr(s, k) for k, _ in BatchStats._fields_}

    def close(self):
        if self._b:
            lib.ep_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
