"""Pins for the oracle's bidomain elliptic solve with a conducting bath
(Bidomain Model subsection, Boundary Conditions; eqn:bidomain1) and for its
ECG leads (Cardiac Simulation chapter, Results, ECG).

The elliptic equation is the sum of the intracellular and extracellular
current balances.  Its operator is therefore A_i (intracellular tensor, heart
only: no intracellular current crosses the heart's boundary) plus A_e (D_e on
the heart, sig_bath I on the bath, over both: the extracellular normal current
equals the bath current on the heart's boundary).

- A 3-D layered heart/bath problem with isotropic tensors and v a cosine mode
  along the interface separates: phi is the same cosine mode times a profile
  across the layers that solves a tridiagonal 1-D finite-volume system, whose
  face conductances are written here from the boundary conditions alone.
  Current crosses the interface (asserted), and a reading that lets
  intracellular current through the interface fails.
- The solve equals the minimum-norm least-squares solution of the dense
  system assembled from two separate dense operators (the pinned 19-point
  operator on the heart with D_i, and on heart + bath with D_e | sig_bath),
  in the sum-zero gauge, on a masked anisotropic grid with interface current.
- A layered slab with v linear across the heart (1-D, no net current
  anywhere): phi falls with slope sigma_i/(sigma_i + sigma_e) in the heart and
  is constant in the bath.
- An empty bath gives the heart-only solve exactly.
- The leads obey Einthoven's law I + III = II and Goldberger's
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


def layered_profile(nx, a, h, si, se, so, mu, f):
    """Profile g(x) of phi = g(x) c(y) for the layered problem: heart cells
    x < a, bath cells x >= a, isotropic conductivities, v = f(x) c(y) on the
    heart with c a Neumann cosine mode of eigenvalue mu (L_y c = mu c).

    1-D cell-centred finite volumes, one unknown per x cell.  Face
    conductances (times h^2):
      intracellular: si between two heart cells, none elsewhere (isolated);
      extracellular/bath: se between heart cells, so between bath cells and
      the mean (se + so)/2 on the heart-bath face (the face rule of the 3-D
      operator, mean of the two voxel tensors).
    Along y every cell sees its own region's conductivity times mu.
    Equation per cell: intracellular balance of v + phi plus
    extracellular balance of phi = 0."""
    Ki = np.zeros((nx, nx))
    Ke = np.zeros((nx, nx))
    for x in range(nx):
        Ki[x, x] += (si * mu) if x < a else 0.0
        Ke[x, x] += (se if x < a else so) * mu
    for x in range(nx - 1):
        q = x + 1
        if q < a:
            ci = si
            ce = se
        elif x >= a:
            ci = 0.0
            ce = so
        else:
            ci = 0.0
            ce = 0.5 * (se + so)
        for (M, c) in ((Ki, ci), (Ke, ce)):
            M[x, q] += c
            M[q, x] += c
            M[x, x] -= c
            M[q, q] -= c
    Ki /= h * h
    Ke /= h * h
    # Ki (f + g) + Ke g = 0
    g = np.linalg.solve(Ki + Ke, -Ki @ f)
    return g, Ke


def test_layered_cosine_mode_interface_current(orc):
    nx, ny, nz, a, h = 10, 6, 3, 5, 0.5
    si, se, so = 0.17, 0.62, 1.3
    shape = (nx, ny, nz)
    mask = np.zeros(shape, np.uint8)
    mask[:a] = 1
    bath = 1 - mask
    fib = np.zeros(shape + (3,))
    fib[..., 0] = 1.0
    inst = inst_with(mask, bath, fib, si, si, se, se, so, h=h)
    o = orc.Oracle(inst)
    k = 1
    cy = np.cos(np.pi * k * (np.arange(ny) + 0.5) / ny)
    mu = -4.0 * np.sin(np.pi * k / (2 * ny)) ** 2
    f = np.zeros(nx)
    f[:a] = np.random.default_rng(7).random(a) + 0.5
    v = f[:, None, None] * cy[None, :, None] * np.ones((1, 1, nz))
    b = orc.apply(shape, h, mask, o.Di, v)
    phi, it = o.solve_elliptic(b, rtol=1e-14, maxit=5000)
    assert it > 0
    g, _ = layered_profile(nx, a, h, si, se, so, mu, f)
    want = g[:, None, None] * cy[None, :, None] * np.ones((1, 1, nz))
    scale = np.abs(want).max()
    assert np.abs(phi - want).max() <= 1e-10 * scale
    # current crosses the heart-bath face: phi jumps there by a sizeable
    # fraction of its range
    assert abs(g[a] - g[a - 1]) > 0.05 * np.abs(g).max()
    # a reading with intracellular conductivity on the heart-bath face
    # (one summed tensor field, faces taking its mean) gives another profile
    Kw = np.zeros((nx, nx))
    for x in range(nx):
        Kw[x, x] += ((si + se) if x < a else so) * mu
    for x in range(nx - 1):
        q = x + 1
        c = (si + se) if q < a else (so if x >= a else 0.5 * (si + se + so))
        Kw[x, q] += c; Kw[q, x] += c; Kw[x, x] -= c; Kw[q, q] -= c
    Kiw = np.zeros((nx, nx))
    for x in range(nx):
        Kiw[x, x] += si * mu if x < a else 0.0
    for x in range(a - 1):
        Kiw[x, x + 1] += si; Kiw[x + 1, x] += si; Kiw[x, x] -= si; Kiw[x + 1, x + 1] -= si
    gw = np.linalg.solve(Kw, -Kiw @ f)
    assert np.abs(gw - g).max() > 1e-3 * np.abs(g).max()


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
    # dense reference: intracellular operator on the heart, extracellular
    # operator with the bath tensor on heart + bath, each assembled alone
    N = mask.size
    m, bt = mask.ravel() > 0, bath.ravel() > 0
    Di = orc.tensors(shape, mask, fib, None, sl, st)
    Deo = np.zeros((6, N))
    Deo[:, m] = orc.tensors(shape, mask, fib, None, sel, set_)[:, m]
    Deo[:3, bt] = sb
    dom = (m | bt).reshape(shape).astype(np.uint8)
    Ai = orc.dense_matrix(shape, inst.h, mask, Di)
    Ae = orc.dense_matrix(shape, inst.h, dom, Deo)
    K = -(Ai + Ae)
    d = dom.ravel() > 0
    x = np.linalg.lstsq(K[np.ix_(d, d)], b.ravel()[d], rcond=None)[0]
    x -= x.mean()
    ref = np.zeros(N)
    ref[d] = x
    got = phi.ravel()
    assert np.abs(got[~d]).max() == 0.0
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    # current crosses the heart's boundary: the couplings of A_e between a
    # heart and a bath voxel carry a sizeable share of the extracellular
    # current (the net over the boundary is zero, as the bath has no source)
    dphi = ref[None, :] - ref[:, None]
    flow = np.abs(Ae * dphi)
    across = flow[np.ix_(m, bt)].sum()
    inside = flow[np.ix_(m, m)].sum()
    assert across > 0.05 * inside
    # and no intracellular current leaves: the heart rows of A_i (v + phi)
    # sum to zero
    vi = v.ravel() + ref
    assert abs((Ai @ vi)[m].sum()) <= 1e-12 * np.abs(Ai @ vi).max()


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
    # the same two operators on the same domain: identical arithmetic
    assert np.array_equal(p1, p2)


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
