"""GPU parity of the explicit step with the thesis's corner-gradient
operator A27 (EP_DIFF_EXPLICIT27) against the oracle's orc_apply27 path:

- FP64 runs from a random state on shells, with and without a per-voxel
  conductivity scale: every corner, mask and brick-boundary case;
- FP32 runs from rest through activation (a 32^3 box and a 40^3 shell);
- the 256^3 shell in the benchmark's launch configuration: one step from the
  GPU's own mid-run state against the oracle's step, every voxel;
- the stability bound: accepted just below, rejected just above, at a dt
  where the 19-point operator is already rejected;
- combinations that A27 does not serve are refused.
"""
import numpy as np
import pytest

import ep_inputs as E

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2302_12519_amd as P
    return P


def c27_shell(n, prec, scale=False, seed=9, n_stim=3, dt=0.05):
    shape, mask, fib, stims = E.shell(n, seed, n_stim)
    sc = E.smooth_scale(shape, 77) if scale else None
    return E.Instance(name=f"shell{n}_c27", n=shape, h=0.25, dt=dt, steps=0, mask=mask,
                      fibre=fib, scale=sc, sigma_l=0.2, sigma_t=0.05, stims=stims,
                      model="mono", diff="explicit27", prec=prec)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,scale", [(17, False), (26, True), (33, False)])
def test_explicit27_fp64_against_oracle(P, orc, n, scale):
    """30 FP64 steps from a random state: within 1e-12 of max |v| (each step
    is a handful of FP64 sums, the oracle's in another order)."""
    inst = c27_shell(n, "f64", scale=scale)
    say(f"case shell_{n} fp64 A27 scale={scale}")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 13)
    g.write("v", v0)
    g.write("w", w0)
    o.set_state(v=v0, w=w0)
    g.step(30)
    o.run(30)
    err, werr = rel(g.read("v"), o.field("v")), rel(g.read("w"), o.field("w"))
    say(f"shell_{n} fp64 A27: v err {err:.2e}, w err {werr:.2e}")
    g.close()
    assert err <= 1e-12 and werr <= 1e-12


@pytest.mark.parametrize("which", ["plain_box_32", "shell_40"])
def test_explicit27_fp32_activation(P, orc, which):
    """FP32 from rest through activation against the FP64 oracle: 1e-4 of
    max |v| and activation times within one dt (the FP32 bar of the other
    explicit runs)."""
    if which == "plain_box_32":
        inst = E.plain_box(32, steps=1000, prec="f32")
        inst.diff = "explicit27"
        steps = 1000
    else:
        inst = c27_shell(40, "f32", n_stim=4)
        steps = 300
    say(f"case {which} fp32 A27 {steps} steps")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    g.step(steps)
    o.run(steps)
    err = rel(g.read("v"), o.field("v"))
    T, To = g.read("tact"), o.field("tact")
    fin = np.isfinite(T) & np.isfinite(To)
    dT = np.abs(T[fin] - To[fin]).max()
    say(f"{which} fp32 A27: v err {err:.2e}, activated {fin.sum()}, dT {dT:.2e}")
    g.close()
    assert fin.sum() > 100
    assert err <= 1e-4
    assert dT <= inst.dt
    assert (np.isfinite(T) != np.isfinite(To)).sum() <= 0.001 * T.size


def test_explicit27_256_one_step_every_voxel(P, orc):
    """The 256^3 shell (5.0M tissue voxels), FP32, dt 0.05: 40 steps on the
    GPU, then one step against the oracle's from the same state.  One FP32
    step of 64 signed terms: bar 1e-6 of max |v|."""
    inst = E.aniso_be(256, steps=41)
    inst.diff = "explicit27"
    say("case aniso_256 fp32 A27: 40 steps on the GPU")
    g = P.Grid.from_instance(inst)
    g.step(40)
    v, w, T = g.read("v"), g.read("w"), g.read("tact")
    say("case aniso_256 A27: one oracle step from the GPU state")
    o = orc.Oracle(inst)
    o.set_state(v=v, w=w, tact=T, step=40)
    o.run(1)
    g.step(1)
    err = rel(g.read("v"), o.field("v"))
    werr = np.abs(g.read("w") - o.field("w")).max()
    Tg, To = g.read("tact"), o.field("tact")
    both = np.isfinite(Tg) & np.isfinite(To)
    dT = np.abs(Tg[both] - To[both]).max()
    say(f"aniso_256 A27 one step: v err {err:.2e}, w err {werr:.2e}, dT {dT:.2e}")
    g.close()
    assert err <= 1e-6
    assert werr <= 1e-6
    assert dT <= inst.dt
    assert (np.isfinite(Tg) != np.isfinite(To)).sum() <= 2


@pytest.mark.parametrize("shape", [(8, 9, 1), (1, 1, 1), (12, 2, 11)])
def test_explicit27_degenerate_grids(P, orc, shape):
    """A grid one voxel thick has no 2x2x2 block, so A27 has no corner and
    the step is the reaction alone; a two-voxel-thick slab has one layer of
    corners.  FP64 against the oracle, 20 steps from a random state."""
    rng = np.random.default_rng(sum(shape))
    fib = rng.normal(size=shape + (3,))
    fib /= np.linalg.norm(fib, axis=-1, keepdims=True)
    inst = E.Instance(name="c27_thin", n=shape, h=0.25, dt=0.02, steps=0,
                      mask=np.ones(shape, np.uint8), fibre=fib, scale=None, sigma_l=0.2,
                      sigma_t=0.05, stims=[], diff="explicit27", prec="f64")
    say(f"case A27 degenerate grid {shape}")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 3)
    g.write("v", v0)
    g.write("w", w0)
    o.set_state(v=v0, w=w0)
    g.step(20)
    o.run(20)
    err = rel(g.read("v"), o.field("v"))
    g.close()
    assert err <= 1e-13
    if min(shape) == 1:
        bare = orc.Oracle(inst)
        bare.set_state(v=v0, w=w0)
        for _ in range(20):
            vs, ws = bare.ionic(bare.field("v"), bare.field("w"))
            bare.set_state(v=vs, w=ws)
        assert rel(o.field("v"), bare.field("v")) <= 1e-15


def test_explicit27_stability_bound(P):
    """h 0.25, sigma_l 0.2: A27 needs dt * 12.8 / ms < 2, so dt 0.155 is
    accepted (where the 19-point operator, lambda_max ~ 19.5 / ms, is not)
    and dt 0.157 is rejected."""
    ok = c27_shell(26, "f32", dt=0.155)
    say("case shell_26 A27 dt 0.155 / 0.157")
    g = P.Grid.from_instance(ok)
    g.step(100)
    v = g.read("v")
    g.close()
    assert np.isfinite(v).all() and np.abs(v).max() < 2.0
    for diff, dt in (("explicit27", 0.157), ("explicit", 0.155)):
        bad = c27_shell(26, "f32", dt=dt)
        g = P.Grid(bad.n, bad.h, bad.dt, mask=bad.mask, prec="f32", diff=diff,
                   ionic=bad.ionic, stims=bad.stims)
        with pytest.raises(P.ep.EPError) as e:
            g.set_conductivity(bad.fibre, None, bad.sigma_l, bad.sigma_t)
        g.close()
        assert e.value.status == P.ep.EP_ERR_ARG


def test_explicit27_refused_combinations(P):
    inst = c27_shell(17, "f32")
    say("case A27 bidomain / adjoint refused")
    with pytest.raises(P.ep.EPError) as e:
        P.Grid(inst.n, inst.h, inst.dt, mask=inst.mask, model="bido", diff="explicit27",
               ionic=inst.ionic)
    assert e.value.status == P.ep.EP_ERR_UNSUPPORTED
    g = P.Grid.from_instance(inst)
    with pytest.raises(P.ep.EPError):
        g.adjoint_scale(np.zeros(inst.n), 5)
    g.close()
