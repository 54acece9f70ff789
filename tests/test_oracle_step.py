"""Pins for the oracle's time step: conservation, exact moment growth, exact
eigenmodes, implicit solves against dense linear algebra, the bidomain ->
monodomain reduction, activation times and the discrete adjoint."""
import math

import numpy as np
import pytest

import ep_inputs as E

NO_IONIC = dict(E.MS_DEFAULT, exc=0.0, tau_out=math.inf)


def box(n, D=0.1, dt=0.01, stims=(), diff="explicit", fibre=None, sig=None, ionic=None):
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    fib = np.zeros(shape + (3,))
    fib[..., 0] = 1.0
    if fibre is not None:
        fib[...] = fibre
    sl, st = (D, D) if sig is None else sig
    inst = E.Instance(name="box", n=shape, h=0.25, dt=dt, steps=0,
                      mask=np.ones(shape, np.uint8), fibre=fib, scale=None,
                      sigma_l=sl, sigma_t=st, stims=list(stims), diff=diff, prec="f64")
    if ionic is not None:
        inst.ionic = dict(ionic)
    return inst


@pytest.mark.parametrize("diff", ["explicit", "be_pcg"])
def test_charge_conservation_with_stimulus(orc, diff):
    """Ionic currents off: the potential integral h^3 sum v changes only by
    the injected charge dt h^3 sum J_stim (no-flux boundaries)."""
    n = 12
    st = [E.Stim(lo=(0, 0, 0), hi=(1, n, n), amp=1.0, t_on=0.0, t_off=0.1),
          E.Stim(lo=(3, 3, 3), hi=(9, 9, 9), center=(1.5, 1.5, 1.5), radius=0.8,
                 amp=0.5, t_on=0.05, t_off=0.3)]
    inst = box(n, D=0.1, dt=0.01, stims=st, diff=diff, ionic=NO_IONIC,
               fibre=(0.6, 0.0, 0.8), sig=(0.2, 0.05))
    o = orc.Oracle(inst)
    rc, info = o.run(40)
    assert rc == 0
    # closed form of the injected charge: voxel counts times the windows
    h3 = 0.25 ** 3
    ball = 0
    for x in range(3, 9):
        for y in range(3, 9):
            for z in range(3, 9):
                d2 = ((x + .5) * .25 - 1.5) ** 2 + ((y + .5) * .25 - 1.5) ** 2 + ((z + .5) * .25 - 1.5) ** 2
                ball += d2 <= 0.64
    steps1 = sum(1 for k in range(40) if 0.0 <= k * 0.01 < 0.1)
    steps2 = sum(1 for k in range(40) if 0.05 <= k * 0.01 < 0.3)
    q = 0.01 * h3 * (n * n * 1.0 * steps1 + ball * 0.5 * steps2)
    assert abs(info.q_stim - q) <= 1e-14 * q
    tol = 1e-13 if diff == "explicit" else 1e-11
    assert abs(info.mass - q) <= tol * q, (info.mass, q)


def test_moment_tensor_grows_by_2D_dt_mass(orc):
    """Constant anisotropic D, ionic off, blob far from the walls: the first
    moments stay fixed and the second-moment tensor grows by exactly
    2 D dt mass per explicit step (the operator is exact on quadratics)."""
    n = 24
    f = np.array([0.48, 0.6, 0.64])
    f /= np.linalg.norm(f)
    sl, st = 0.2, 0.05
    inst = box(n, dt=0.01, ionic=NO_IONIC, fibre=f, sig=(sl, st))
    o = orc.Oracle(inst)
    h = 0.25
    ax = (np.arange(n) + 0.5) * h
    X = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
    c = X[n // 2, n // 2, n // 2]
    r2 = np.sum((X - c) ** 2, axis=-1)
    v0 = np.where(r2 <= (2 * h) ** 2, 1.0 + np.cos(r2), 0.0)
    o.set_state(v=v0, w=np.ones((n, n, n)))

    def moments(v):
        m = v.sum()
        m1 = np.einsum("xyzi,xyz->i", X, v)
        m2 = np.einsum("xyzi,xyzj,xyz->ij", X, X, v)
        return m, m1, m2

    Dt = st * np.eye(3) + (sl - st) * np.outer(f, f)
    m0, m10, m20 = moments(o.field("v"))
    k = 4
    o.run(k)
    m, m1, m2 = moments(o.field("v"))
    assert abs(m - m0) <= 1e-14 * m0
    assert np.abs(m1 - m10).max() <= 1e-13 * np.abs(m10).max()
    pred = m20 + 2.0 * Dt * 0.01 * k * m0
    assert np.abs(m2 - pred).max() <= 1e-13 * np.abs(m20).max()


@pytest.mark.parametrize("diff", ["explicit", "be_pcg"])
def test_cosine_modes_are_exact_eigenvectors(orc, diff):
    """Isotropic D on a full Neumann box: cell-centred cosines are eigenvectors
    with lambda_k = -(4D/h^2) sum_d sin^2(pi k_d / (2 n_d)); one explicit step
    multiplies by (1 + dt lambda), one implicit step by 1/(1 - dt lambda)."""
    n = (10, 8, 6)
    D, h, dt = 0.1, 0.25, 0.02
    inst = box(n, D=D, dt=dt, diff=diff, ionic=NO_IONIC)
    o = orc.Oracle(inst)
    k = (2, 3, 1)
    ax = [np.cos(np.pi * k[d] * (np.arange(n[d]) + 0.5) / n[d]) for d in range(3)]
    v0 = ax[0][:, None, None] * ax[1][None, :, None] * ax[2][None, None, :]
    lam = -(4 * D / h ** 2) * sum(math.sin(math.pi * k[d] / (2 * n[d])) ** 2 for d in range(3))
    o.set_state(v=v0, w=np.ones(n))
    o.run(1)
    fac = (1 + dt * lam) if diff == "explicit" else 1.0 / (1 - dt * lam)
    tol = 1e-14 if diff == "explicit" else 1e-12
    assert np.abs(o.field("v") - fac * v0).max() <= tol


def small_shell(n, model="mono", seed=9, sig=(0.2, 0.05), sig_e=(0.0, 0.0)):
    shape, mask, fib, stims = E.shell(n, seed, 2)
    return E.Instance(name="s", n=shape, h=0.25, dt=0.05, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=sig[0], sigma_t=sig[1], sigma_el=sig_e[0],
                      sigma_et=sig_e[1], stims=stims, model=model,
                      diff="be_pcg" if model == "mono" else "explicit")


def test_implicit_step_matches_dense_solve(orc):
    inst = small_shell(12)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 3)
    o.set_state(v=v0, w=w0, step=100)      # past the stimulus window
    vs, _ = o.ionic(o.field("v"), o.field("w"))
    o.run(1)
    A = orc.dense_matrix(inst.n, inst.h, inst.mask, o.Di)
    M = np.eye(A.shape[0]) - inst.dt * A
    x = np.linalg.solve(M, vs.ravel())
    assert np.abs(o.v - x).max() <= 1e-11 * np.abs(x).max()


def test_elliptic_matches_dense_least_squares(orc):
    inst = small_shell(12, model="bido", sig=(0.17, 0.019), sig_e=(0.62, 0.24))
    assert inst.nt < 1000
    o = orc.Oracle(inst)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(inst.n) * inst.mask
    b = orc.apply(inst.n, inst.h, inst.mask, o.Di, v)
    phi, it = o.solve_elliptic(b)
    assert it > 0
    t = inst.mask.ravel() > 0
    K = -(orc.dense_matrix(inst.n, inst.h, inst.mask, o.Di)
          + orc.dense_matrix(inst.n, inst.h, inst.mask, o.De))[np.ix_(t, t)]
    x, *_ = np.linalg.lstsq(K, b.ravel()[t], rcond=None)
    x -= x.mean()
    assert abs(phi.ravel()[t].sum()) <= 1e-12 * np.abs(x).sum()
    assert np.abs(phi.ravel()[t] - x).max() <= 1e-10 * np.abs(x).max()


def test_bidomain_reduces_to_monodomain(orc):
    """Sigma_e = lambda Sigma_i gives phi = -v*/(1+lambda) + const and the
    monodomain step with D = lambda/(1+lambda) Sigma_i (eqn:monodomain1)."""
    lam = 2.5
    si = (0.17, 0.019)
    bi = small_shell(14, model="bido", sig=si, sig_e=(lam * si[0], lam * si[1]))
    mo = small_shell(14, model="mono", sig=(lam / (1 + lam) * si[0], lam / (1 + lam) * si[1]))
    mo.diff = "explicit"
    ob, om = orc.Oracle(bi), orc.Oracle(mo)
    v0, w0 = E.random_state(bi, 8)
    for o in (ob, om):
        o.set_state(v=v0, w=w0, step=100)  # past the stimulus window
    vs, _ = ob.ionic(ob.field("v"), ob.field("w"))
    ob.run(1)
    om.run(1)
    t = bi.mask.ravel() > 0
    ref_phi = -vs.ravel()[t] / (1 + lam)
    ref_phi -= ref_phi.mean()
    assert np.abs(ob.phi[t] - ref_phi).max() <= 1e-9 * np.abs(ref_phi).max()
    assert np.abs(ob.v - om.v).max() <= 1e-10
    ob.run(3)
    om.run(3)
    assert np.abs(ob.v - om.v).max() <= 1e-9


def test_activation_mirror_symmetry_and_planar_speed(orc):
    """A stimulus on the x = 0 layer of an isotropic box gives a planar wave:
    T_act is the same across each layer (mirror symmetric in y and z) and
    grows linearly in x at constant speed away from the ends."""
    n = (48, 6, 6)
    inst = box(n, D=0.1, dt=0.02, stims=[E.Stim(lo=(0, 0, 0), hi=(1, 6, 6))])
    o = orc.Oracle(inst)
    o.run(2200)
    T = o.field("tact")
    assert np.all(np.isfinite(T))
    assert np.abs(T - T[:, ::-1, :]).max() <= 1e-12 * T.max()
    assert np.abs(T - T[:, :, ::-1]).max() <= 1e-12 * T.max()
    line = T[:, 3, 3]
    assert np.all(np.diff(line) > 0)
    cv = 0.25 / np.diff(line)[10:38]
    assert cv.std() / cv.mean() < 0.01
    assert 0.2 < cv.mean() < 0.6


@pytest.mark.parametrize("dt", [0.03, 0.01, 0.007, 0.05])
@pytest.mark.parametrize("diff", ["explicit", "be_pcg"])
def test_activation_time_closed_form(orc, dt, diff):
    """One tissue voxel, ionic currents off, a constant stimulus amp: then
    v_n = n dt amp and the potential reaches theta at exactly t = theta/amp,
    whatever dt.  The interpolated crossing time must give that to rounding;
    basing the interpolation on t_{n+1} instead of t_n, or interpolating
    from the wrong end, would be off by up to one dt."""
    amp, theta = 0.7, 0.5
    st = [E.Stim(lo=(0, 0, 0), hi=(1, 1, 1), amp=amp, t_on=0.0, t_off=1e9)]
    inst = box((1, 1, 1), dt=dt, stims=st, diff=diff, ionic=NO_IONIC)
    inst.theta = theta
    o = orc.Oracle(inst)
    nsteps = int(math.ceil(theta / amp / dt)) + 3
    rc, _ = o.run(nsteps)
    assert rc == 0
    T = float(o.tact[0])
    assert abs(T - theta / amp) <= 1e-12, (T, theta / amp)
    # the potential itself is the running sum n dt amp
    assert abs(o.v[0] - nsteps * dt * amp) <= 1e-12


def test_adjoint_matches_central_differences(orc):
    """Gradient of sum (T - T*)^2 with respect to the per-voxel conductivity
    scale, against central differences in FP64 along smooth directions."""
    n = (12, 12, 10)
    shape = n
    mask = np.ones(shape, np.uint8)
    mask[5:8, 5:8, :] = 0          # a hole so the mask matters
    f = np.zeros(shape + (3,))
    f[..., 0], f[..., 1] = np.cos(0.5), np.sin(0.5)
    st = [E.Stim(lo=(0, 0, 0), hi=(4, 4, 10), amp=1.0, t_on=0.0, t_off=1.0)]
    inst = E.Instance(name="adj", n=shape, h=0.25, dt=0.04, steps=0, mask=mask, fibre=f,
                      scale=None, sigma_l=0.2, sigma_t=0.05, stims=st, prec="f64")
    s = E.smooth_scale(shape, 11, sigma_vox=3.0)
    s_star = E.smooth_scale(shape, 12, sigma_vox=3.0)
    D0 = orc.tensors(shape, mask, f, None, 0.2, 0.05)
    steps = 260

    def run_loss(scale, tstar):
        o = orc.Oracle(inst, scale=scale)
        return o.adjoint(D0, steps, tstar)

    _, _, _, tstar = run_loss(s_star, np.full(shape, np.inf))
    tstar = np.where(np.isfinite(tstar), tstar, np.inf)
    L, g, used, tact = run_loss(s, tstar)
    assert used > 0.5 * mask.sum() and L > 0
    rng = np.random.default_rng(3)
    for k in range(3):
        d = E.smooth_scale(shape, 100 + k, sigma_vox=3.0) - 1.0
        eps = 1e-5
        Lp = run_loss(s + eps * d, tstar)[0]
        Lm = run_loss(s - eps * d, tstar)[0]
        fd = (Lp - Lm) / (2 * eps)
        ad = float(np.sum(g * d))
        assert abs(fd - ad) <= 1e-5 * abs(fd), (fd, ad)


def jacobi_shell(n, sweeps):
    inst = small_shell(n)
    inst.diff = "be_jacobi"
    inst.jacobi_sweeps = sweeps
    return inst


@pytest.mark.parametrize("sweeps", [1, 2, 5])
def test_jacobi_step_matches_dense_recurrence(orc, sweeps):
    """The fixed-sweep implicit step (eqn:iejac1) against the same recurrence
    on the dense matrix: M = I - dt A split into its diagonal and the rest,
    u^0 = v*, u^{k+1} = diag(M)^-1 (v* - (M - diag(M)) u^k)."""
    inst = jacobi_shell(12, sweeps)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 5)
    o.set_state(v=v0, w=w0, step=100)
    vs, _ = o.ionic(o.field("v"), o.field("w"))
    rc, info = o.run(1)
    A = orc.dense_matrix(inst.n, inst.h, inst.mask, o.Di)
    M = np.eye(A.shape[0]) - inst.dt * A
    d = np.diag(M)
    R = M - np.diag(d)
    b = vs.ravel()
    u = b.copy()
    for _ in range(sweeps):
        u = (b - R @ u) / d
    u = np.where(inst.mask.ravel() > 0, u, 0.0)
    assert rc == 0 and info.cg_iters == sweeps
    assert np.abs(o.v - u).max() <= 1e-13 * np.abs(u).max()


def test_jacobi_step_converges_to_the_implicit_solve(orc):
    """Enough sweeps reach the backward-Euler solution (dense solve), and the
    error shrinks monotonically with the sweep count."""
    errs = []
    for sweeps in (2, 8, 32):
        inst = jacobi_shell(12, sweeps)
        o = orc.Oracle(inst)
        v0, w0 = E.random_state(inst, 3)
        o.set_state(v=v0, w=w0, step=100)
        vs, _ = o.ionic(o.field("v"), o.field("w"))
        o.run(1)
        A = orc.dense_matrix(inst.n, inst.h, inst.mask, o.Di)
        x = np.linalg.solve(np.eye(A.shape[0]) - inst.dt * A, vs.ravel())
        errs.append(np.abs(o.v - x).max() / np.abs(x).max())
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-12
