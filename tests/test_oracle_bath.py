"""Pins for the oracle's bidomain elliptic solve with a conducting bath
(Bidomain Model subsection, Boundary Conditions; eqn:bidomain1) and for its
ECG leads (Cardiac Simulation chapter, Results, ECG):

- the solve equals the minimum-norm least-squares solution of the dense
  system, assembled here from the operator and a tensor field built in numpy
  (heart: D_i + D_e, bath: sig_bath I), in the sum-zero gauge;
- a layered heart/bath slab with a potential linear across the heart has a
  closed-form solution: phi falls with slope sigma_i/(sigma_i + sigma_e)
  through the heart (no net current anywhere in 1-D) and is constant in the
  bath;
- an empty bath gives the heart-only solve (to rounding);
- the leads obey Einthoven's law I + III = II and Goldberger's
  aVR + aVL + aVF = 0, and give the textbook values on a known field.
"""
import numpy as np

import ep_inputs as E


def inst_with(mask, bath, fib, sl, st, sel, set_, sig_bath, h=0.5):
    shape = mask.shape
    return E.Instance(name="bath", n=shape, h=h, dt=0.01, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=sl, sigma_t=st, sigma_el=sel, sigma_et=set_,
                      stims=[], model="bido", prec="f64", bath=bath, sigma_bath=sig_bath,
                      electrodes=((0, 0, 0), (shape[0] - 1, 0, 0), (0, shape[1] - 1, 0)))


def test_bath_solve_matches_dense_lstsq(orc):
    rng = np.random.default_rng(41)
    shape = (7, 6, 5)
    mask = np.zeros(shape, np.uint8)
    mask[2:5, 1:5, 1:4] = 1
    mask[2, 1, 1] = 0
    bath = (mask == 0).astype(np.uint8)
    bath[0, :, 0] = 0           # a few non-conducting voxels too
    fib = rng.normal(size=shape + (3,))
    fib /= np.linalg.norm(fib, axis=-1, keepdims=True)
    sl, st, sel, set_, sb = 0.17, 0.02, 0.62, 0.24, 0.9
    inst = inst_with(mask, bath, fib, sl, st, sel, set_, sb)
    o = orc.Oracle(inst)
    v = rng.random(shape) * mask
    b = orc.apply(shape, inst.h, mask, o.Di, v)
    phi, it = o.solve_elliptic(b, rtol=1e-14, maxit=5000)
    assert it > 0
    # dense reference from a numpy-built tensor field
    N = mask.size
    Dk = np.zeros((6, N))
    m, bt = mask.ravel() > 0, bath.ravel() > 0
    Dk[:, m] = (orc.tensors(shape, mask, fib, None, sl, st)
                + orc.tensors(shape, mask, fib, None, sel, set_))[:, m]
    Dk[:3, bt] = sb
    dom = (m | bt).reshape(shape).astype(np.uint8)
    K = -orc.dense_matrix(shape, inst.h, dom, Dk)
    d = dom.ravel() > 0
    x = np.linalg.lstsq(K[np.ix_(d, d)], b.ravel()[d], rcond=None)[0]
    x -= x.mean()
    ref = np.zeros(N)
    ref[d] = x
    got = phi.ravel()
    assert np.abs(got[~d]).max() == 0.0
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_layered_slab_closed_form(orc):
    """Heart x < 6, bath x >= 6, isotropic conductivities, v = x (mm) in the
    heart.  The net current vanishes everywhere (1-D, no flux at both ends),
    so phi' = -sigma_i/(sigma_i + sigma_e) in the heart and phi' = 0 in the
    bath, continuous at the interface."""
    shape, h = (12, 3, 3), 0.5
    mask = np.zeros(shape, np.uint8)
    mask[:6] = 1
    bath = 1 - mask
    fib = np.zeros(shape + (3,))
    fib[..., 2] = 1.0
    si, se, sb = 0.2, 0.3, 1.3
    inst = inst_with(mask, bath, fib, si, si, se, se, sb, h=h)
    o = orc.Oracle(inst)
    x = (np.arange(shape[0]) + 0.5) * h
    v = np.broadcast_to(x[:, None, None], shape) * mask
    b = orc.apply(shape, h, mask, o.Di, v)
    phi, _ = o.solve_elliptic(b, rtol=1e-14, maxit=5000)
    slope = -si / (si + se)
    want = np.where(x < 6 * h, slope * x, slope * x[5])
    want = want - want.mean()
    assert np.abs(phi - want[:, None, None]).max() <= 1e-10


def test_empty_bath_is_heart_only(orc):
    inst = E.bidomain(16, steps=0)
    inst.prec = "f64"
    o1 = orc.Oracle(inst)
    inst.bath = np.zeros(inst.n, np.uint8)
    inst.sigma_bath = 1.0
    o2 = orc.Oracle(inst)
    v = E.random_state(inst, 5)[0]
    b = orc.apply(inst.n, inst.h, inst.mask, o1.Di, v)
    p1, _ = o1.solve_elliptic(b, rtol=1e-13)
    p2, _ = o2.solve_elliptic(b, rtol=1e-13)
    # the same system; the bath path sums D_i + D_e per voxel before the
    # operator instead of adding the two operators, so rounding differs
    assert np.abs(p1 - p2).max() <= 1e-11 * np.abs(p1).max()


def test_lead_identities_and_values(orc):
    inst = E.bidomain_bath(20, steps=6)
    inst.prec = "f64"
    o = orc.Oracle(inst)
    o.run(6)
    I, II, III, aVR, aVL, aVF = o.ecg()
    scale = max(abs(I), abs(II), abs(III), 1e-300)
    assert abs(I + III - II) <= 1e-14 * scale
    assert abs(aVR + aVL + aVF) <= 1e-14 * scale
    assert scale > 0.0
    # a known field: phi = 1 + 2x + 3y + 5z at the electrode voxels
    n = inst.n
    X, Y, Z = np.meshgrid(*[np.arange(k, dtype=float) for k in n], indexing="ij")
    o.phi = (1 + 2 * X + 3 * Y + 5 * Z).ravel()
    (ra, la, ll) = [1 + 2 * a + 3 * b + 5 * c for a, b, c in inst.electrodes]
    want = [la - ra, ll - ra, ll - la, ra - (la + ll) / 2, la - (ra + ll) / 2,
            ll - (ra + la) / 2]
    assert np.allclose(o.ecg(), want, rtol=0, atol=1e-12)
