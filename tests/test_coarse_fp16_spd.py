"""The elliptic inner solve's two-level preconditioner keeps CG's
requirement of a symmetric positive definite preconditioner after the
coarse inverse is rounded to FP16.

The preconditioner is M = D^-1 + P C P^T: D the diagonal of
K = -(A_i + A_e), P the piecewise-constant prolongation over aggregates of
8x8x8 bricks, C = (P^T K P + s/n)^-1 with s = trace(K)/n.  The library
stores C scaled so that its largest (diagonal) entry is 2^14, rounded to
FP16 through FP32, and multiplies the GEMV by the FP32 unscale factor.  This
test forms C in FP64 from the oracle's operator on the test grids, rounds it
the same way, and checks that the rounded matrix stays positive definite (so
M does: D^-1 is positive and P C P^T then positive semidefinite), with the
rounding perturbation well inside the smallest eigenvalue.  K is recovered
exactly from 27 operator applications (voxels of one residue class modulo 3
per axis never share a 3x3x3 neighbourhood)."""
import numpy as np
import pytest
import scipy.sparse as sp

import ep_inputs as E


def sparse_operator(orc, shape, h, masks_and_tensors):
    """Sparse sum of the operators (mask, D) as a CSR matrix, probed with
    27 coloured indicator vectors."""
    N = int(np.prod(shape))
    X, Y, Z = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    color = ((X % 3) * 9 + (Y % 3) * 3 + (Z % 3)).ravel()
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [], [], []
    for c in range(27):
        e = (color == c).astype(np.float64)
        y = np.zeros(N)
        for mask, D in masks_and_tensors:
            y += orc.apply(shape, h, mask, D, e.reshape(shape)).ravel()
        nz = np.nonzero(y)[0]
        # the column of row i probed by colour c is the voxel of colour c
        # inside i's 3x3x3 neighbourhood
        px, py, pz = np.unravel_index(nz, shape)
        best = np.full(nz.size, -1)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    qx, qy, qz = px + dx, py + dy, pz + dz
                    ok = ((qx >= 0) & (qy >= 0) & (qz >= 0) & (qx < shape[0]) &
                          (qy < shape[1]) & (qz < shape[2]))
                    q = np.where(ok, idx[np.clip(qx, 0, shape[0] - 1),
                                         np.clip(qy, 0, shape[1] - 1),
                                         np.clip(qz, 0, shape[2] - 1)], -1)
                    hit = ok & (color[np.maximum(q, 0)] == c)
                    best = np.where(hit, q, best)
        assert (best >= 0).all()
        rows.append(nz)
        cols.append(best)
        vals.append(y[nz])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A


def coarse_inverse_check(orc, inst):
    o = orc.Oracle(inst)
    shape, h = inst.n, inst.h
    heart = inst.mask
    if inst.bath is not None:
        dom = ((inst.mask > 0) | (inst.bath > 0)).astype(np.uint8)
        Deo = np.zeros_like(o.De)
        m, bt = heart.ravel() > 0, inst.bath.ravel() > 0
        Deo[:, m] = o.De[:, m]
        Deo[:3, bt] = inst.sigma_bath
    else:
        dom, Deo = heart, o.De
    K = -sparse_operator(orc, shape, h, [(heart, o.Di), (dom, Deo)])
    d = dom.ravel() > 0
    K = K[d][:, d]
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    # aggregates: single 8x8x8 bricks (the library's choice up to 8192)
    X, Y, Z = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    brick = ((X // 8) * 1000000 + (Y // 8) * 1000 + (Z // 8)).ravel()[d]
    _, agg = np.unique(brick, return_inverse=True)
    n = int(agg.max()) + 1
    P = sp.csr_matrix((np.ones(agg.size), (np.arange(agg.size), agg)), shape=(agg.size, n))
    Kc = (P.T @ K @ P).toarray()
    s = K.diagonal().sum() / n
    Kc = Kc + s / n
    C = np.linalg.inv(Kc)
    C = 0.5 * (C + C.T)
    dmax = np.diag(C).max()
    scale = 16384.0 / dmax
    unscale = float(np.float32(dmax / 16384.0))
    C16 = (C * scale).astype(np.float32).astype(np.float16).astype(np.float64) * unscale
    lam = np.linalg.eigvalsh(C)
    lam16 = np.linalg.eigvalsh(C16)
    pert = np.linalg.norm(C16 - C, 2)
    return n, lam[0], lam16[0], pert


@pytest.mark.parametrize("case", ["bidomain_32", "bidomain_48", "bath_32"])
def test_fp16_coarse_inverse_stays_positive_definite(orc, case):
    if case.startswith("bath"):
        inst = E.bidomain_bath(int(case.split("_")[1]), steps=0)
    else:
        inst = E.bidomain(int(case.split("_")[1]), steps=0)
    n, lmin, lmin16, pert = coarse_inverse_check(orc, inst)
    print(f"{case}: {n} aggregates, lambda_min(C) {lmin:.3e}, rounded {lmin16:.3e}, "
          f"||C16 - C|| {pert:.3e}")
    assert n > 1
    assert lmin > 0.0
    assert lmin16 > 0.0
    # the perturbation is a small fraction of the smallest eigenvalue: the
    # rounded matrix is positive definite with a wide margin, not by chance
    assert pert <= 0.25 * lmin
