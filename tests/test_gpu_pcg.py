"""GPU tests of the implicit-Euler Jacobi-PCG (one launch per iteration,
next residual norms expanded in the previous launch's dot products, the
launch that finds the solve done applying the last x update):

- FP64 runs of several steps against the oracle, so that the extrapolated
  initial guess goes through every order it uses;
- a solve that is done before its first iteration (zero right-hand side);
- the iteration limit, reported as EP_ERR_NOCONV;
- bitwise reproducibility of FP32 runs (fixed-order reductions), also when
  the steps are split over several calls;
- the activation check of steps whose guess already solves the system;
- FP32 iteration counts step by step against FP64 on the same problem.
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


def be_shell(n, n_stim=3, prec="f64", seed=9):
    shape, mask, fib, stims = E.shell(n, seed, n_stim)
    return E.Instance(name=f"shell{n}", n=shape, h=0.25, dt=0.05, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=0.2, sigma_t=0.05, sigma_el=0.0, sigma_et=0.0,
                      stims=stims, model="mono", diff="be_pcg", prec=prec)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n", [17, 26])
def test_be_pcg_fp64_run_against_oracle(P, orc, n):
    """20 FP64 steps solved to 1e-13 from a random state: every step's
    guess order (0 to 4) and the iteration / last-update launches take part.
    Bar: 1e-10 of max |v| after 20 steps (each step's solve error is about
    1e-13 times the condition number, about 2)."""
    inst = be_shell(n)
    inst.pcg_rtol = 1e-13
    inst.pcg_maxit = 200
    say(f"case shell_{n} fp64 BE-PCG 20 steps")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 11)
    g.write("v", v0)
    g.write("w", w0)
    o.set_state(v=v0, w=w0)
    info = g.step(20)
    o.run(20)
    err = rel(g.read("v"), o.field("v"))
    werr = rel(g.read("w"), o.field("w"))
    say(f"shell_{n} fp64 BE: iters {info['cg_iters']} (max {info['cg_max']}), v err {err:.2e}, "
        f"w err {werr:.2e}")
    g.close()
    assert info["cg_iters"] >= 20
    assert err <= 1e-10
    assert werr <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_be_pcg_zero_rhs_takes_no_iteration(P, orc, prec):
    """At rest with no stimulus the reaction leaves v = 0, so b = 0: the
    first PCG launch finds the solve done and no x update happens."""
    inst = be_shell(17, n_stim=0, prec=prec)
    say(f"case shell_17 {prec} BE-PCG at rest")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    info = g.step(5)
    o.run(5)
    v = g.read("v")
    g.close()
    assert info["cg_iters"] == 0 and info["cg_max"] == 0
    assert np.array_equal(v, np.zeros_like(v))
    assert np.abs(o.field("v")).max() == 0.0


def test_be_pcg_iteration_limit_reports_noconv(P):
    inst = be_shell(17, prec="f64")
    inst.pcg_rtol = 1e-15
    inst.pcg_maxit = 1
    say("case shell_17 fp64 BE-PCG maxit 1")
    g = P.Grid.from_instance(inst)
    v0, w0 = E.random_state(inst, 3)
    g.write("v", v0)
    g.write("w", w0)
    out = g.step(1, check=False)
    g.close()
    assert out["status"] == P.ep.EP_ERR_NOCONV


def test_be_pcg_fp32_bitwise_reproducible(P):
    """Two grids built from the same inputs give bitwise the same state after
    60 FP32 steps: every reduction runs in a fixed order."""
    inst = E.aniso_be(40, steps=60)
    inst.pcg_rtol = 1e-7
    say("case aniso_be_40 fp32 reproducibility")
    out = []
    for _ in range(2):
        g = P.Grid.from_instance(inst)
        info = g.step(60)
        out.append((g.read("v"), g.read("w"), g.read("tact"), info["cg_iters"]))
        g.close()
    (v1, w1, t1, i1), (v2, w2, t2, i2) = out
    assert i1 == i2
    assert np.array_equal(v1, v2) and np.array_equal(w1, w2)
    assert np.array_equal(t1, t2, equal_nan=True)



@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_be_pcg_activation_when_the_guess_solves(P, orc, prec):
    """A uniform state has no diffusion, so every step's initial guess solves
    the system and no launch makes a last x update.  From v = 0.45, w = 1
    the reaction carries every voxel across theta = 0.5 during step 4; T_act
    must match the oracle's on every voxel."""
    inst = be_shell(17, n_stim=0, prec=prec)
    say(f"case shell_17 {prec} BE-PCG uniform state crossing threshold")
    m = inst.mask.astype(np.float64)
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    g.write("v", 0.45 * m)
    g.write("w", m)
    o.set_state(v=0.45 * m, w=m)
    info = g.step(8)
    o.run(8)
    T, To = g.read("tact"), o.field("tact")
    v = g.read("v")
    g.close()
    tis = inst.mask > 0
    tol = 1e-12 if prec == "f64" else 1e-6
    assert info["cg_iters"] == 0
    assert np.isfinite(To[tis]).all() and np.isfinite(T[tis]).all()
    assert np.abs(T[tis] - To[tis]).max() <= tol
    assert np.abs(v - o.field("v")).max() <= tol


def test_be_pcg_split_calls_bitwise(P):
    """The solver state carried between steps (the extrapolation history, the
    activation check of each step) does not depend on how the steps are
    grouped into calls: 60 FP32 steps in one call and in six calls of ten
    give bitwise the same v, w and T_act."""
    inst = E.aniso_be(40, steps=60)
    inst.pcg_rtol = 1e-7
    say("case aniso_be_40 fp32 one call against six")
    out = []
    for calls in (1, 6):
        g = P.Grid.from_instance(inst)
        it = 0
        for _ in range(calls):
            it += g.step(60 // calls)["cg_iters"]
        out.append((g.read("v"), g.read("w"), g.read("tact"), it))
        g.close()
    (v1, w1, t1, i1), (v2, w2, t2, i2) = out
    assert i1 == i2
    assert np.isfinite(t1).sum() > 0
    assert np.array_equal(v1, v2) and np.array_equal(w1, w2)
    assert np.array_equal(t1, t2, equal_nan=True)


def test_be_pcg_fp32_iterations_match_fp64(P):
    """The FP32 solver is CG in its own right, not just a method that ends
    within tolerance: step by step on the same problem it needs the FP64
    solver's iteration count while the counts are large (the first 30
    steps: 3 to 8 iterations, where a wrong search direction or step length
    shows at once), and at most one more later, where FP32 rounding near
    the 1e-7 tolerance can cost one."""
    say("case aniso_be_40 fp32 against fp64 iteration counts, 60 steps")
    counts = {}
    for prec in ("f64", "f32"):
        inst = E.aniso_be(40, steps=60)
        inst.pcg_rtol = 1e-7
        g = P.Grid.from_instance(inst, prec=prec)
        counts[prec] = np.array([g.step(1)["cg_iters"] for _ in range(60)])
        g.close()
    a, b = counts["f64"], counts["f32"]
    say(f"iterations: fp64 {a.sum()}, fp32 {b.sum()}; first 30 steps equal: "
        f"{int((a[:30] == b[:30]).sum())}")
    assert a[:30].min() >= 3
    assert np.array_equal(a[:30], b[:30])
    assert np.all(b - a <= 1) and np.all(b - a >= -1)
