"""Seeded synthetic problem instances for the voxel cardiac-EP step.

This module is the ONE input path shared by the GPU library's tests/bench and
by the CPU oracle.  It builds problem *instances* only: a tissue mask, a unit
fibre field, an optional per-voxel conductivity scale, stimulus regions and the
constants of each workload.  It holds none of the method's arithmetic (no ionic
model, no conductivity tensor, no stencil, no solver); each side computes those
itself from these inputs.

Geometry follows the thesis's signed-distance encoding (Geometry section of
the Discretization and Solver chapter, "Primitives" and the set operations after them): an ellipsoid primitive
``|p/r| - 1`` and the complement ``max(s1, -s2)`` carve a hollow, ventricle-like
shell out of the voxel box; a voxel is tissue when the SDF at its centre is
<= 0 (volume pass of the two-pass encoding).  The thesis's schematic heart is
not reproducible from its text (its parameters are not printed), so this shell
stands in for it; the conductivities are the thesis's (Whole-heart chapter,
"Fibre Directions": sigma_L = 0.20, sigma_T = 0.05) and the fibre angle rotates
transmurally from -60 to +60 degrees.

Index convention everywhere: flat index = (x*ny + y)*nz + z (z fastest);
arrays are numpy with shape (nx, ny, nz) in C order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Mitchell-Schaeffer constants (Cardiac Multiphysics chapter,
# Mitchell-Schaeffer Model subsection).  The thesis prints none; these are
# the values of the original 2003 model it cites.  Times in ms, v dimensionless.
MS_DEFAULT = dict(tau_in=0.3, tau_out=6.0, tau_open=120.0, tau_close=150.0,
                  v_gate=0.13, exc=1.0)

SHELL_RHO = 0.66559           # inner/outer radius ratio giving ~30 % tissue
SHELL_ROUT = (0.46, 0.46, 0.48)  # outer semi-axes as a fraction of the box edge


@dataclasses.dataclass
class Stim:
    """Stimulus region: voxels p with lo <= p < hi (per axis) that are also
    within ``radius`` mm of ``center`` (mm) when radius > 0, intersected with
    tissue.  Current ``amp`` (1/ms) for t_on <= t_n < t_off."""
    lo: Sequence[int]
    hi: Sequence[int]
    center: Sequence[float] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    amp: float = 1.0
    t_on: float = 0.0
    t_off: float = 1.0


@dataclasses.dataclass
class Instance:
    name: str
    n: tuple                      # (nx, ny, nz)
    h: float                      # mm
    dt: float                     # ms
    steps: int
    mask: np.ndarray              # uint8 (nx,ny,nz), 1 = tissue
    fibre: np.ndarray             # float64 (nx,ny,nz,3), unit vectors
    scale: Optional[np.ndarray]   # float64 (nx,ny,nz) or None (= 1)
    sigma_l: float
    sigma_t: float
    sigma_el: float = 0.0         # extracellular (bidomain only)
    sigma_et: float = 0.0
    stims: List[Stim] = dataclasses.field(default_factory=list)
    model: str = "mono"           # "mono" | "bido"
    diff: str = "explicit"        # "explicit" | "be_pcg" | "be_jacobi" | "explicit27"
    prec: str = "f32"             # "f32" | "f64"
    ionic: dict = dataclasses.field(default_factory=lambda: dict(MS_DEFAULT))
    theta: float = 0.5
    pcg_rtol: float = 1e-6
    pcg_maxit: int = 50
    ell_rtol: float = 1e-8
    jacobi_sweeps: int = 10       # "be_jacobi": fixed Jacobi sweeps per step
    bath: Optional[np.ndarray] = None   # uint8, 1 on conducting bath voxels (bidomain)
    sigma_bath: float = 0.0       # isotropic bath conductivity
    electrodes: Optional[tuple] = None  # voxel coordinates of RA, LA, LL

    @property
    def nb(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nt(self) -> int:
        return int(self.mask.sum())


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def _centres(n, h):
    """Voxel-centre coordinates (mm) relative to the box centre, as 3 open
    grids broadcastable to (nx, ny, nz)."""
    ax = [((np.arange(k, dtype=np.float64) + 0.5) * h - 0.5 * k * h) for k in n]
    return (ax[0][:, None, None], ax[1][None, :, None], ax[2][None, None, :])


def shell_mask(n, h, rout_frac=SHELL_ROUT, rho=SHELL_RHO):
    """Ellipsoidal shell: outer ellipsoid minus the inner one scaled by rho."""
    X, Y, Z = _centres(n, h)
    L = np.array(n, dtype=np.float64) * h
    R = np.asarray(rout_frac, dtype=np.float64) * L
    s_out = np.sqrt((X / R[0]) ** 2 + (Y / R[1]) ** 2 + (Z / R[2]) ** 2) - 1.0
    Ri = rho * R
    s_in = np.sqrt((X / Ri[0]) ** 2 + (Y / Ri[1]) ** 2 + (Z / Ri[2]) ** 2) - 1.0
    sdf = np.maximum(s_out, -s_in)
    return (sdf <= 0.0).astype(np.uint8), R


def transmural_fibres(n, h, R, rho, mask):
    """Fibre angle alpha(e) = -60deg + 120deg*e across the wall, e = 0 at the
    outer (epicardial) surface and 1 at the inner one; f = cos(a) c + sin(a) l
    with n the normalised gradient of the normalised radius, c = e_z x n
    (e_x where degenerate) and l = n x c.  Non-tissue voxels get (1,0,0)."""
    X, Y, Z = _centres(n, h)
    X, Y, Z = np.broadcast_arrays(X, Y, Z)
    qx, qy, qz = X / R[0], Y / R[1], Z / R[2]
    r = np.sqrt(qx * qx + qy * qy + qz * qz)
    rs = np.where(r > 0, r, 1.0)
    # gradient of r with respect to position
    gx, gy, gz = qx / (rs * R[0]), qy / (rs * R[1]), qz / (rs * R[2])
    gn = np.sqrt(gx * gx + gy * gy + gz * gz)
    gn = np.where(gn > 0, gn, 1.0)
    nx_, ny_, nz_ = gx / gn, gy / gn, gz / gn
    # c = e_z x n = (-n_y, n_x, 0)
    cx, cy, cz = -ny_, nx_, np.zeros_like(nx_)
    cn = np.sqrt(cx * cx + cy * cy)
    deg = cn < 1e-12
    cn = np.where(deg, 1.0, cn)
    cx, cy = cx / cn, cy / cn
    cx = np.where(deg, 1.0, cx)
    cy = np.where(deg, 0.0, cy)
    # l = n x c
    lx = ny_ * cz - nz_ * cy
    ly = nz_ * cx - nx_ * cz
    lz = nx_ * cy - ny_ * cx
    e = np.clip((1.0 - r) / (1.0 - rho), 0.0, 1.0)
    a = np.deg2rad(-60.0 + 120.0 * e)
    ca, sa = np.cos(a), np.sin(a)
    f = np.stack([ca * cx + sa * lx, ca * cy + sa * ly, ca * cz + sa * lz], axis=-1)
    f /= np.linalg.norm(f, axis=-1, keepdims=True)
    f[mask == 0] = (1.0, 0.0, 0.0)
    return f


def ball_stims(mask, h, count, rng, radius=1.0, amp=1.0, t_on=0.0, t_off=1.0):
    """``count`` balls of ``radius`` mm centred on tissue voxels drawn
    uniformly (seeded)."""
    n = mask.shape
    tissue = np.flatnonzero(mask.ravel())
    picks = rng.choice(tissue, size=count, replace=False)
    r_vox = int(math.ceil(radius / h))
    out = []
    for p in np.sort(picks):
        x, y, zz = np.unravel_index(int(p), n)
        c = tuple((np.array([x, y, zz], dtype=np.float64) + 0.5) * h)
        lo = [max(0, int(v) - r_vox) for v in (x, y, zz)]
        hi = [min(n[d], int(v) + r_vox + 1) for d, v in enumerate((x, y, zz))]
        out.append(Stim(lo=lo, hi=hi, center=c, radius=radius, amp=amp,
                        t_on=t_on, t_off=t_off))
    return out


def smooth_scale(n, seed, sigma_vox=8.0, amp=0.5):
    """s = 1 + amp * G / max|G|, G = Gaussian-filtered white noise (seeded)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = gaussian_filter(rng.standard_normal(n), sigma=sigma_vox, mode="reflect")
    return 1.0 + amp * g / np.max(np.abs(g))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def plain_box(n=32, steps=1000, prec="f64"):
    """Plain monodomain: n^3 all-tissue box (or an (nx, ny, nz) box), h = 0.25
    mm, isotropic 0.1 mm^2/ms, stimulus on the x = 0 layer for 1 ms, explicit
    Euler dt 0.01."""
    shape = (n, n, n) if np.isscalar(n) else tuple(int(k) for k in n)
    mask = np.ones(shape, np.uint8)
    fib = np.zeros(shape + (3,))
    fib[..., 0] = 1.0
    stims = [Stim(lo=(0, 0, 0), hi=(1,) + shape[1:], amp=1.0, t_on=0.0, t_off=1.0)]
    tag = str(n) if np.isscalar(n) else "x".join(str(k) for k in shape)
    return Instance(name=f"plain_box_{tag}", n=shape, h=0.25, dt=0.01, steps=steps,
                    mask=mask, fibre=fib, scale=None, sigma_l=0.1, sigma_t=0.1,
                    stims=stims, model="mono", diff="explicit", prec=prec)


def cuboid(dx, dt, t_end=60.0, prec="f32", diff="explicit", sigma=(0.2, 0.05)):
    """The thesis's electrophysiology benchmark geometry (Benchmark Studies
    section): a 20 x 7 x 3 mm all-tissue cuboid at voxel width dx (mm),
    fibres along its long axis, stimulated in the 1.5 mm cube at one corner
    for the first 1 ms.  The benchmark's own cell model and conductivities
    are not in the thesis; this stands in with Mitchell-Schaeffer and
    sigma = (0.2, 0.05) mm^2/ms (the shell workloads' values).  Steps cover
    t_end ms at dt."""
    shape = tuple(int(round(L / dx)) for L in (20.0, 7.0, 3.0))
    mask = np.ones(shape, np.uint8)
    fib = np.zeros(shape + (3,))
    fib[..., 0] = 1.0
    k = int(math.ceil(1.5 / dx - 1e-9))
    stims = [Stim(lo=(0, 0, 0), hi=(k, k, k), amp=1.0, t_on=0.0, t_off=1.0)]
    return Instance(name=f"cuboid_dx{dx:g}_dt{dt:g}", n=shape, h=float(dx), dt=float(dt),
                    steps=int(round(t_end / dt)), mask=mask, fibre=fib, scale=None,
                    sigma_l=sigma[0], sigma_t=sigma[1], stims=stims, model="mono", diff=diff,
                    prec=prec)


def shell(n, seed, n_stim, h=0.25, rout_frac=SHELL_ROUT, rho=SHELL_RHO):
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    mask, R = shell_mask(shape, h, rout_frac, rho)
    fib = transmural_fibres(shape, h, R, rho, mask)
    rng = np.random.default_rng(seed)
    stims = ball_stims(mask, h, n_stim, rng)
    return shape, mask, fib, stims


def aniso_be(n=256, steps=2000):
    """Anisotropic monodomain, FP32 state, backward-Euler diffusion by
    Jacobi-PCG: n^3 ventricle-like shell, sigma 0.2/0.05, 16 ball stimuli."""
    shape, mask, fib, stims = shell(n, 2001, 16)
    return Instance(name=f"aniso_be_{n}", n=shape, h=0.25, dt=0.05, steps=steps,
                    mask=mask, fibre=fib, scale=None, sigma_l=0.2, sigma_t=0.05,
                    stims=stims, model="mono", diff="be_pcg", prec="f32",
                    pcg_rtol=1e-6, pcg_maxit=50)


def bidomain(n=192, steps=500):
    """Bidomain, mixed-precision elliptic solve: n^3 shell, sigma_i 0.17/0.019,
    sigma_e 0.62/0.24, 16 ball stimuli, dt 0.05."""
    shape, mask, fib, stims = shell(n, 3001, 16)
    return Instance(name=f"bidomain_{n}", n=shape, h=0.25, dt=0.05, steps=steps,
                    mask=mask, fibre=fib, scale=None, sigma_l=0.17, sigma_t=0.019,
                    sigma_el=0.62, sigma_et=0.24, stims=stims, model="bido",
                    diff="explicit", prec="f32", ell_rtol=1e-8)


def bidomain_bath(n=128, steps=200, sigma_bath=1.0, rout_frac=(0.30, 0.30, 0.32)):
    """Bidomain with a conducting bath for the ECG: a smaller shell (the
    heart) inside an n^3 box whose every other voxel (cavity and
    surroundings) is bath of isotropic conductivity sigma_bath.  Electrodes
    at box corners: RA (0, 0, n-1) and LL (n-1, n-1, 0) diametrically
    opposite, LA (n-1, 0, n-1).  Heart conductivities and stimuli as in
    bidomain(); dt 0.05."""
    shape, mask, fib, stims = shell(n, 3001, 8, rout_frac=rout_frac)
    bath = (mask == 0).astype(np.uint8)
    e = ((0, 0, n - 1), (n - 1, 0, n - 1), (n - 1, n - 1, 0))
    return Instance(name=f"bidomain_bath_{n}", n=shape, h=0.25, dt=0.05, steps=steps,
                    mask=mask, fibre=fib, scale=None, sigma_l=0.17, sigma_t=0.019,
                    sigma_el=0.62, sigma_et=0.24, stims=stims, model="bido",
                    diff="explicit", prec="f32", ell_rtol=1e-8, bath=bath,
                    sigma_bath=float(sigma_bath), electrodes=e)


def adjoint_shell(n=128, steps=500, target=False):
    """Differentiation workload: n^3 shell, sigma 0.2/0.05 times a smooth
    per-voxel scale in [0.5, 1.5] (seed 5001; the target run uses 5002), 8
    ball stimuli, explicit dt 0.04."""
    shape, mask, fib, stims = shell(n, 5001, 8)
    scale = smooth_scale(shape, 5002 if target else 5001)
    return Instance(name=f"adjoint_{n}", n=shape, h=0.25, dt=0.04, steps=steps,
                    mask=mask, fibre=fib, scale=scale, sigma_l=0.2, sigma_t=0.05,
                    stims=stims, model="mono", diff="explicit", prec="f32")


def fd_directions(n, count=5, seed=5003):
    """Smooth seeded perturbation directions for finite-difference checks."""
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    return [smooth_scale(shape, seed * 100 + k) - 1.0 for k in range(count)]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                # s, relative to stream start
    inst: Instance


def serving_stream(count=64, seed_arrivals=4001, seed_params=4002, rate=None,
                   n_range=(48, 160), steps_range=(200, 1000), burst=False):
    """Serving workload: ``count`` requests with Poisson arrivals (``rate``
    per second; all at t = 0 when ``burst``), grid n ~ U{48..160}, outer
    semi-axes L*U[0.40, 0.48] per axis, rho ~ U[0.55, 0.75], conductivity
    scale c ~ U[0.5, 1.5] (on 0.2/0.05), excitability ~ U[0.8, 1.2], 4 ball
    stimuli, steps ~ U{200..1000}, explicit FP32, dt 0.04, h 0.25."""
    ra = np.random.default_rng(seed_arrivals)
    rp = np.random.default_rng(seed_params)
    if burst or rate is None:
        arrivals = np.zeros(count)
    else:
        arrivals = np.cumsum(ra.exponential(1.0 / rate, size=count))
    reqs = []
    for k in range(count):
        n = int(rp.integers(n_range[0], n_range[1] + 1))
        rout = tuple(float(v) for v in rp.uniform(0.40, 0.48, size=3))
        rho = float(rp.uniform(0.55, 0.75))
        c = float(rp.uniform(0.5, 1.5))
        exc = float(rp.uniform(0.8, 1.2))
        steps = int(rp.integers(steps_range[0], steps_range[1] + 1))
        sseed = int(rp.integers(1 << 30))
        shape = (n, n, n)
        mask, R = shell_mask(shape, 0.25, rout, rho)
        fib = transmural_fibres(shape, 0.25, R, rho, mask)
        stims = ball_stims(mask, 0.25, 4, np.random.default_rng(sseed))
        ionic = dict(MS_DEFAULT)
        ionic["exc"] = exc
        inst = Instance(name=f"req{k}", n=shape, h=0.25, dt=0.04, steps=steps,
                        mask=mask, fibre=fib, scale=None, sigma_l=0.2 * c,
                        sigma_t=0.05 * c, stims=stims, model="mono",
                        diff="explicit", prec="f32", ionic=ionic)
        reqs.append(Request(rid=k, arrival=float(arrivals[k]), inst=inst))
    return reqs


def resting_state(inst: Instance):
    """v = 0, w = 1 (the MS resting point) on tissue; zeros elsewhere."""
    v = np.zeros(inst.n)
    w = np.where(inst.mask > 0, 1.0, 0.0)
    return v, w


def random_state(inst: Instance, seed: int):
    """Seeded state with v, w in [0, 1] on tissue (for one-step parity)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 1.0, inst.n) * inst.mask
    w = rng.uniform(0.0, 1.0, inst.n) * inst.mask
    return v, w
