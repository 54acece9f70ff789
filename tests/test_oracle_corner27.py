"""Pins for the oracle's corner-gradient operator A27 (the thesis's own
operator, Matrix-Free Assembly section, eqn:ass1 - eqn:ass3, with the
conductivity block of the Diffusion subsection), each from something other
than its own formula:

- exact on quadratics: A27 (x^T H x / 2) = tr(D H) away from the boundary;
- its Fourier symbol, worked out by hand: A27 e^{i th.p} = -lambda(th) e^{i th.p}
  with lambda = (4/h^2) S^T D S, S_d = sin(th_d/2) prod_{e != d} cos(th_e/2);
- hourglass null modes: (-1)^(i+j), (-1)^(i+k), (-1)^(j+k), (-1)^(i+j+k)
  are annihilated in the interior (the 19-point operator does not do that);
- on masked, heterogeneous tissue: symmetric, negative semidefinite, zero
  row sums, and lambda_max(-A27) <= 4 max_p lambda_max(D_p) / h^2 (each of
  a voxel's 8 corners adds at most lambda_max(D_c) / (2 h^2));
- one explicit step of the run equals the ionic step plus dt A27 v*.
"""
import numpy as np
import pytest

import ep_inputs as E


def uniform(shape, fibre, sl, st):
    f = np.asarray(fibre, float) / np.linalg.norm(fibre)
    fib = np.broadcast_to(f, tuple(shape) + (3,)).copy()
    return np.ones(shape, np.uint8), fib, f


def tensor(f, sl, st, s=1.0):
    return s * (st * np.eye(3) + (sl - st) * np.outer(f, f))


def interior(shape):
    return tuple(slice(1, k - 1) for k in shape)


def test_quadratic_exact(orc):
    shape, h, sl, st = (7, 8, 9), 0.4, 0.3, 0.07
    mask, fib, f = uniform(shape, (0.3, -0.5, 0.8), sl, st)
    D = orc.tensors(shape, mask, fib, None, sl, st)
    H = np.array([[0.7, -0.4, 0.25], [-0.4, -1.1, 0.6], [0.25, 0.6, 0.9]])
    X = np.stack(np.meshgrid(*[h * (np.arange(k) + 0.5) for k in shape], indexing="ij"), -1)
    v = 0.5 * np.einsum("...i,ij,...j->...", X, H, X)
    a = orc.apply27(shape, h, mask, D, v)
    want = np.trace(tensor(f, sl, st) @ H)
    got = a[interior(shape)]
    assert np.abs(got - want).max() <= 1e-11 * abs(want) + 1e-12


@pytest.mark.parametrize("th", [(0.7, 2.1, 1.3), (np.pi, 0.0, 0.0), (0.4, -2.9, 0.5)])
def test_plane_wave_symbol(orc, th):
    shape, h, sl, st = (9, 8, 10), 0.25, 0.2, 0.05
    mask, fib, f = uniform(shape, (0.6, 0.64, 0.48), sl, st)
    D = orc.tensors(shape, mask, fib, None, sl, st)
    th = np.asarray(th)
    I = np.stack(np.meshgrid(*[np.arange(k) for k in shape], indexing="ij"), -1)
    v = np.cos(I @ th)
    c, s = np.cos(th / 2), np.sin(th / 2)
    S = np.array([s[0] * c[1] * c[2], c[0] * s[1] * c[2], c[0] * c[1] * s[2]])
    lam = 4.0 / h**2 * S @ tensor(f, sl, st) @ S
    a = orc.apply27(shape, h, mask, D, v)
    sl_ = interior(shape)
    assert np.abs(a[sl_] + lam * v[sl_]).max() <= 1e-11 * max(lam, 1.0)


def test_hourglass_modes_are_null(orc):
    shape, h, sl, st = (8, 7, 9), 0.3, 0.25, 0.04
    mask, fib, f = uniform(shape, (0.2, 0.9, -0.4), sl, st)
    D = orc.tensors(shape, mask, fib, None, sl, st)
    i, j, k = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    sl_ = interior(shape)
    for mode in [(-1.0) ** (i + j), (-1.0) ** (i + k), (-1.0) ** (j + k), (-1.0) ** (i + j + k)]:
        a = orc.apply27(shape, h, mask, D, mode)
        assert np.abs(a[sl_]).max() <= 1e-12
    # the 19-point operator is not blind to the checkerboard
    a19 = orc.apply(shape, h, mask, D, (-1.0) ** (i + j + k))
    assert np.abs(a19[sl_]).min() > 1.0


def test_masked_heterogeneous_invariants(orc):
    rng = np.random.default_rng(27)
    shape, h, sl, st = (6, 5, 7), 0.5, 0.3, 0.08
    mask = (rng.random(shape) < 0.8).astype(np.uint8)
    fib = rng.normal(size=shape + (3,))
    fib /= np.linalg.norm(fib, axis=-1, keepdims=True)
    scale = 1.0 + rng.random(shape)
    D = orc.tensors(shape, mask, fib, scale, sl, st)
    A = orc.dense_matrix(shape, h, mask, D, op=orc.apply27)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * np.abs(A).max()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() <= 1e-12 * np.abs(ev).max()
    bound = 4.0 * (scale[mask.astype(bool)].max() * sl) / h**2
    assert -ev.min() <= bound * (1 + 1e-12)
    # non-tissue rows and columns are empty
    off = ~mask.astype(bool).ravel()
    assert np.abs(A[off]).max() == 0.0 and np.abs(A[:, off]).max() == 0.0
    # corners leaving the tissue carry no flux: a voxel whose 2x2x2 blocks
    # all hold non-tissue is decoupled from everything
    m = mask.astype(bool)
    blocks = np.ones((shape[0] - 1, shape[1] - 1, shape[2] - 1), bool)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                blocks &= m[a:shape[0] - 1 + a, b:shape[1] - 1 + b, c:shape[2] - 1 + c]
    touched = np.zeros(shape, bool)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                touched[a:shape[0] - 1 + a, b:shape[1] - 1 + b, c:shape[2] - 1 + c] |= blocks
    lone = (m & ~touched).ravel()
    if lone.any():
        assert np.abs(A[lone]).max() == 0.0


def test_bound_is_reached_on_uniform_tissue(orc):
    """The stability bound is the largest eigenvalue of the symbol, reached
    at th = (pi, 0, 0) along the fibre axis: a large uniform box gets within
    a few per cent (the no-flux walls hold the top mode slightly below it)."""
    shape, h, sl, st = (16, 12, 12), 0.5, 0.3, 0.08
    mask, fib, f = uniform(shape, (1.0, 0.0, 0.0), sl, st)
    D = orc.tensors(shape, mask, fib, None, sl, st)
    x = np.random.default_rng(3).normal(size=shape)
    for _ in range(600):
        x = -orc.apply27(shape, h, mask, D, x)
        x /= np.linalg.norm(x)
    lam = float(np.sum(x * -orc.apply27(shape, h, mask, D, x)))
    bound = 4.0 * sl / h**2
    assert 0.95 * bound <= lam <= bound


def test_run_step_is_ionic_plus_explicit27(orc):
    shape, sl, st = (6, 7, 5), 0.2, 0.05
    rng = np.random.default_rng(5)
    mask = np.ones(shape, np.uint8)
    mask[0, 0, :] = 0
    fib = rng.normal(size=shape + (3,))
    fib /= np.linalg.norm(fib, axis=-1, keepdims=True)
    inst = E.Instance(name="c27", n=shape, h=0.25, dt=0.01, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=sl, sigma_t=st, stims=[], diff="explicit27",
                      prec="f64")
    o = orc.Oracle(inst)
    v0 = np.where(mask > 0, rng.random(shape), 0.0)
    w0 = np.where(mask > 0, rng.random(shape), 0.0)
    o.set_state(v=v0, w=w0)
    vs, ws = o.ionic(v0, w0)
    o.run(1)
    want = vs + inst.dt * orc.apply27(shape, inst.h, mask, o.Di, vs)
    assert np.abs(o.field("v") - np.where(mask > 0, want, 0.0)).max() <= 1e-15


@pytest.mark.parametrize("diff", ["explicit", "explicit27"])
def test_second_moment_tensor_grows_by_2D(orc, diff):
    """Ionic currents off, a blob far from the walls, uniform anisotropic D:
    one explicit step changes sum v x_i x_j h^3 by exactly 2 D_ij dt mass,
    off-diagonal moments included (both operators are symmetric and exact on
    quadratics)."""
    import math
    shape, h, dt, sl, st = (24, 26, 22), 0.25, 0.01, 0.2, 0.05
    f = np.array([1.0, 2.0, 2.0]) / 3.0
    fib = np.broadcast_to(f, shape + (3,)).copy()
    ionic = dict(E.MS_DEFAULT, exc=0.0, tau_out=math.inf)
    inst = E.Instance(name="mom", n=shape, h=h, dt=dt, steps=0, mask=np.ones(shape, np.uint8),
                      fibre=fib, scale=None, sigma_l=sl, sigma_t=st, stims=[], diff=diff,
                      prec="f64", ionic=ionic)
    X = np.stack(np.meshgrid(*[h * (np.arange(k) + 0.5) for k in shape], indexing="ij"), -1)
    c = np.array([k * h / 2 for k in shape]) + np.array([0.1, -0.2, 0.15])
    r2 = ((X - c) ** 2).sum(-1)
    v0 = np.exp(-r2 / (2 * 0.3 ** 2))   # the walls at > 8.7 sigma
    o = orc.Oracle(inst)
    o.set_state(v=v0, w=np.ones(shape))
    o.run(1)
    v1 = o.field("v")

    Y = X - c        # about the blob centre (the first moment does not move)

    def moments(v):
        return np.einsum("xyz,xyzi,xyzj->ij", v, Y, Y) * h**3, v.sum() * h**3

    M0, m0 = moments(v0)
    M1, m1 = moments(v1)
    D = st * np.eye(3) + (sl - st) * np.outer(f, f)
    assert abs(m1 - m0) <= 1e-13 * m0
    assert np.abs((M1 - M0) - 2 * D * dt * m0).max() <= 1e-9 * np.abs(2 * D * dt * m0).max()
