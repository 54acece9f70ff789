"""GPU parity of the implicit Euler step by the thesis's fixed number of
Jacobi sweeps (eqn:iejac1) against the oracle's same recurrence."""
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


def jacobi_shell(n, sweeps, prec="f64", seed=9, n_stim=3):
    shape, mask, fib, stims = E.shell(n, seed, n_stim)
    return E.Instance(name=f"shell{n}", n=shape, h=0.25, dt=0.05, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=0.2, sigma_t=0.05, sigma_el=0.0, sigma_et=0.0,
                      stims=stims, model="mono", diff="be_jacobi", prec=prec,
                      jacobi_sweeps=sweeps)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("sweeps", [1, 2, 7])
def test_jacobi_fp64_steps_match_oracle(P, orc, sweeps):
    """FP64, 20 steps from a random state: the sweep recurrence is linear and
    its rounding is FP64, so the two sides agree to 1e-12 of max |v|."""
    inst = jacobi_shell(26, sweeps)
    say(f"case shell_26 fp64 Jacobi {sweeps} sweeps, 20 steps")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    v0, w0 = E.random_state(inst, 7)
    g.write("v", v0)
    g.write("w", w0)
    o.set_state(v=v0, w=w0)
    info = g.step(20)
    o.run(20)
    err, werr = rel(g.read("v"), o.field("v")), rel(g.read("w"), o.field("w"))
    g.close()
    say(f"shell_26 Jacobi {sweeps}: v err {err:.2e}, w err {werr:.2e}")
    assert info["cg_iters"] == 20 * sweeps and info["cg_max"] == sweeps
    assert err <= 1e-12 and werr <= 1e-12


def test_jacobi_fp32_run_matches_oracle(P, orc):
    """FP32 state, 10 sweeps per step, 200 steps with ball stimuli against the
    FP64 oracle: the FP32 bar (1e-4 of max |v|, activation within one dt)."""
    inst = E.aniso_be(40, steps=200)
    inst.diff = "be_jacobi"
    inst.jacobi_sweeps = 10
    say("case aniso_be_40 fp32 Jacobi 10 sweeps, 200 steps")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    g.step(200)
    o.run(200)
    err = np.abs(g.read("v") - o.field("v")).max() / np.abs(o.field("v")).max()
    T, To = g.read("tact"), o.field("tact")
    fin = np.isfinite(T) & np.isfinite(To)
    g.close()
    say(f"aniso_be_40 Jacobi fp32: err {err:.2e}, dT {np.abs(T[fin] - To[fin]).max():.2e}")
    assert err <= 1e-4
    assert np.abs(T[fin] - To[fin]).max() <= inst.dt
    assert (np.isfinite(T) != np.isfinite(To)).sum() <= 0.001 * T.size


def test_jacobi_needs_a_sweep(P):
    inst = jacobi_shell(17, 0)
    with pytest.raises(P.EPError) as e:
        P.Grid.from_instance(inst)
    assert e.value.status == P.ep.EP_ERR_ARG
