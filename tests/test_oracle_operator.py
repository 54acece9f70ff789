"""Pins for the oracle's 19-point energy-form diffusion operator A."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def random_tensors(rng, n, mask):
    """Random SPD per-voxel tensors (6, N) from random unit fibres."""
    N = int(np.prod(n))
    f = rng.standard_normal((N, 3))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    sl = rng.uniform(0.1, 0.3, N)
    st = rng.uniform(0.02, 0.08, N)
    a = sl - st
    D = np.stack([st + a * f[:, 0] ** 2, st + a * f[:, 1] ** 2, st + a * f[:, 2] ** 2,
                  a * f[:, 0] * f[:, 1], a * f[:, 0] * f[:, 2], a * f[:, 1] * f[:, 2]])
    return D * mask.ravel()[None, :]


def random_mask(rng, n, p=0.8):
    return (rng.uniform(size=n) < p).astype(np.uint8)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dense_symmetric_zero_rowsum_psd(orc, seed):
    rng = np.random.default_rng(seed)
    n = (5, 4, 6)
    mask = random_mask(rng, n)
    D = random_tensors(rng, n, mask)
    A = orc.dense_matrix(n, 0.25, mask, D)
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-15 * scale
    assert np.abs(A.sum(axis=1)).max() <= 1e-14 * scale
    # rows and columns of non-tissue voxels are zero
    off = mask.ravel() == 0
    assert np.all(A[off] == 0) and np.all(A[:, off] == 0)
    ev = np.linalg.eigvalsh(-A)
    assert ev.min() >= -1e-13 * ev.max()
    # at most 19 non-zeros per row
    assert (np.abs(A) > 0).sum(axis=1).max() <= 19
    # the diagonal helper agrees with the assembled matrix
    d = orc.diag(n, 0.25, mask, D).ravel()
    assert np.abs(d - np.diag(A)).max() <= 1e-14 * scale


def seven_point(n, h, mask, Dc):
    """Textbook cell-centred 7-point Neumann Laplacian with face value
    (D_p + D_q)/2 on faces between tissue voxels."""
    N = int(np.prod(n))
    L = np.zeros((N, N))
    idx = np.arange(N).reshape(n)
    for x in range(n[0]):
        for y in range(n[1]):
            for z in range(n[2]):
                p = idx[x, y, z]
                if not mask[x, y, z]:
                    continue
                for d in range(3):
                    for s in (-1, 1):
                        q3 = [x, y, z]
                        q3[d] += s
                        if not (0 <= q3[d] < n[d]):
                            continue
                        if not mask[tuple(q3)]:
                            continue
                        q = idx[tuple(q3)]
                        c = 0.5 * (Dc.ravel()[p] + Dc.ravel()[q]) / h ** 2
                        L[p, q] += c
                        L[p, p] -= c
    return L


def test_isotropic_reduces_to_seven_point(orc):
    rng = np.random.default_rng(7)
    n = (4, 5, 3)
    mask = random_mask(rng, n, 0.85)
    c = rng.uniform(0.05, 0.2, n)
    D = np.zeros((6, int(np.prod(n))))
    D[0] = D[1] = D[2] = (c * mask).ravel()
    A = orc.dense_matrix(n, 0.25, mask, D)
    L = seven_point(n, 0.25, mask, c)
    assert np.abs(A - L).max() <= 1e-13 * np.abs(L).max()


def test_edge_term_matches_reference_gradient_weights(orc):
    """One 2x2 block in the x-y plane with only an xy conductivity c: the energy
    is 2 c g_x g_y with the block gradient of the printed reference-gradient
    weights, so A = -c (Gx Gy^T + Gy Gx^T)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "refgrad2.txt"))
            if l.strip() and not l.startswith("#")]
    W = {r[0]: (float(r[1]), float(r[2])) for r in rows}
    h, c = 0.25, 0.37
    n = (2, 2, 1)
    mask = np.ones(n, np.uint8)
    D = np.zeros((6, 4))
    D[3] = c
    A = orc.dense_matrix(n, h, mask, D)
    # flat index (x*2 + y): u00 -> (0,0), u10 -> (1,0), u01 -> (0,1), u11 -> (1,1)
    order = {"u00": 0, "u10": 2, "u01": 1, "u11": 3}
    Gx = np.zeros(4)
    Gy = np.zeros(4)
    for k, (wx, wy) in W.items():
        Gx[order[k]] = 0.5 * wx / h
        Gy[order[k]] = 0.5 * wy / h
    ref = -c * (np.outer(Gx, Gy) + np.outer(Gy, Gx))
    assert np.abs(A - ref).max() <= 1e-14 * np.abs(ref).max()


def test_exact_on_quadratics_interior(orc):
    rng = np.random.default_rng(11)
    n = (7, 7, 7)
    h = 0.25
    N = int(np.prod(n))
    f = rng.standard_normal(3)
    f /= np.linalg.norm(f)
    Dt = 0.05 * np.eye(3) + 0.15 * np.outer(f, f)
    D = np.zeros((6, N))
    for c, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        D[c] = Dt[i, j]
    M = rng.standard_normal((3, 3))
    M = M + M.T
    ax = [(np.arange(k) + 0.5) * h for k in n]
    X = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)
    u = np.einsum("...i,ij,...j->...", X, M, X)
    Au = orc.apply(n, h, np.ones(n, np.uint8), D, u)
    exact = 2.0 * np.sum(Dt * M)
    inner = Au[1:-1, 1:-1, 1:-1]
    assert np.abs(inner - exact).max() <= 1e-11 * abs(exact) + 1e-12


def _field(X, Y, Z):
    """Smooth SPD tensor field and the manufactured scalar u = sin x cos y e^z
    (first component of the thesis's convergence-study field), with the
    analytic div(D grad u)."""
    u = np.sin(X) * np.cos(Y) * np.exp(Z)
    ux = np.cos(X) * np.cos(Y) * np.exp(Z)
    uy = -np.sin(X) * np.sin(Y) * np.exp(Z)
    uz = u
    uxx, uyy, uzz = -u, -u, u
    uxy = -np.cos(X) * np.sin(Y) * np.exp(Z)
    uxz = ux
    uyz = uy
    Dxx = 1 + 0.5 * np.sin(X)
    Dyy = 1 + 0.5 * np.cos(Y)
    Dzz = 1 + 0.5 * np.sin(Z)
    Dxy = 0.2 * np.sin(X + Y)
    Dxz = 0.2 * np.cos(X - Z)
    Dyz = 0.2 * np.sin(Y * Z)
    dDxx_x = 0.5 * np.cos(X)
    dDyy_y = -0.5 * np.sin(Y)
    dDzz_z = 0.5 * np.cos(Z)
    dDxy_x = dDxy_y = 0.2 * np.cos(X + Y)
    dDxz_x = -0.2 * np.sin(X - Z)
    dDxz_z = 0.2 * np.sin(X - Z)
    dDyz_y = 0.2 * Z * np.cos(Y * Z)
    dDyz_z = 0.2 * Y * np.cos(Y * Z)
    div = ((dDxx_x + dDxy_y + dDxz_z) * ux + (dDxy_x + dDyy_y + dDyz_z) * uy
           + (dDxz_x + dDyz_y + dDzz_z) * uz
           + Dxx * uxx + Dyy * uyy + Dzz * uzz + 2 * (Dxy * uxy + Dxz * uxz + Dyz * uyz))
    D = np.stack([Dxx, Dyy, Dzz, Dxy, Dxz, Dyz]).reshape(6, -1)
    return u, D, div


def test_second_order_convergence_manufactured(orc):
    """L2 error (volume-weighted, eqn:l2norm1) of A u against the analytic
    div(D grad u) on [-1, 1]^3, over voxels whose whole stencil is interior."""
    errs, hs = [], []
    for n1 in (24, 48, 96):
        h = 2.0 / n1
        n = (n1, n1, n1)
        ax = -1.0 + (np.arange(n1) + 0.5) * h
        X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
        u, D, div = _field(X, Y, Z)
        Au = orc.apply(n, h, np.ones(n, np.uint8), D, u)
        e = (Au - div)[1:-1, 1:-1, 1:-1]
        errs.append(math.sqrt(np.sum(e * e) * h ** 3))
        hs.append(h)
    orders = [math.log(errs[k] / errs[k + 1]) / math.log(hs[k] / hs[k + 1]) for k in range(2)]
    for o in orders:
        assert abs(o - 2.0) < 0.1, (errs, orders)


def test_scale_gradient_matches_finite_difference(orc):
    """mu^T (dA/ds_q) v against central differences of mu^T A(s) v."""
    rng = np.random.default_rng(5)
    n = (4, 4, 4)
    mask = random_mask(rng, n, 0.9)
    D0 = random_tensors(rng, n, mask)
    s = rng.uniform(0.5, 1.5, int(np.prod(n)))
    mu = rng.standard_normal(n) * mask
    v = rng.standard_normal(n) * mask
    g = orc.dA_ds(n, 0.25, mask, D0, mu, v).ravel()
    eps = 1e-6
    for q in np.flatnonzero(mask.ravel())[:12]:
        sp, sm = s.copy(), s.copy()
        sp[q] += eps
        sm[q] -= eps
        fp = np.sum(mu * orc.apply(n, 0.25, mask, D0 * sp[None], v))
        fm = np.sum(mu * orc.apply(n, 0.25, mask, D0 * sm[None], v))
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])
