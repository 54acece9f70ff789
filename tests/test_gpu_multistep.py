"""Several explicit steps per cooperative launch (grids whose bricks all fit
on the device at once) against one launch per step and the FP64 oracle.

The multi-step kernel runs the per-step kernel's reaction and operator code
on the same values, so the two paths must agree bitwise: v, w, T_act, the
injected charge and the potential integral, over stimulus switches, odd and
even launch lengths, ragged masks (ghost neighbours) and both precisions.
A grid too large for one co-resident launch falls back to one launch per
step."""
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


def shell_inst(n, prec, seed=9, n_stim=3, dt=0.02):
    shape, mask, fib, stims = E.shell(n, seed, n_stim)
    # staggered stimulus windows: several switches inside the run
    for k, s in enumerate(stims):
        s.t_on, s.t_off = 0.1 * k, 0.5 + 0.3 * k
    return E.Instance(name=f"shell{n}", n=shape, h=0.25, dt=dt, steps=0, mask=mask, fibre=fib,
                      scale=None, sigma_l=0.2, sigma_t=0.05, sigma_el=0.0, sigma_et=0.0,
                      stims=stims, model="mono", diff="explicit", prec=prec)


def run(P, inst, spl, chunks):
    g = P.Grid.from_instance(inst, steps_per_launch=spl)
    g.kernel_timing(kernels=["multistep"])
    infos = [g.step(k) for k in chunks]
    out = {f: g.read(f) for f in ("v", "w", "tact")}
    out["q"] = [i["q_stim"] for i in infos]
    out["mass"] = [i["mass"] for i in infos]
    out["launches"] = g.kernel_time("multistep")[1]
    out["bricks"] = g.stats()["n_bricks"]
    g.close()
    return out


def differ(x, y):
    """Where x and y differ (infinities equal), with the first few values."""
    d = ~((x == y) | (np.isnan(x) & np.isnan(y)))
    idx = np.argwhere(d)[:4]
    return (f"{int(d.sum())} differ; first at {idx.tolist()}: "
            f"{[float(x[tuple(i)]) for i in idx]} vs {[float(y[tuple(i)]) for i in idx]}")


def same(a, b):
    for f in ("v", "w", "tact"):
        assert np.array_equal(a[f], b[f]), f"{f}: {differ(a[f], b[f])}"
    assert a["q"] == b["q"]
    assert a["mass"] == b["mass"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("spl", [0, 7])
def test_shell_multistep_bitwise_equals_per_step(P, prec, spl):
    """Ragged 29^3 shell (bricks with ghost neighbours), three stimuli that
    switch on and off at different steps, 300 steps in calls of 1, 64, 235
    steps: the multi-step path (unbounded, or at most 7 steps per launch)
    gives bitwise the results of one launch per step."""
    inst = shell_inst(29, prec)
    chunks = [1, 64, 235]
    say(f"case shell_29 {prec} steps_per_launch {spl}")
    ref = run(P, inst, 1, chunks)
    got = run(P, inst, spl, chunks)
    assert ref["launches"] == 0
    assert got["launches"] > 0
    if spl == 7:
        assert got["launches"] >= 299 // 7
    same(got, ref)
    assert np.isfinite(got["tact"]).sum() > 0


def test_plain_box_fp64_multistep_matches_oracle(P, orc):
    """32^3 FP64 box, 1000 steps in one call (a stimulus switch at 1 ms):
    the multi-step path against the oracle to the FP64 bar, and bitwise
    against one launch per step."""
    inst = E.plain_box(32, steps=1000, prec="f64")
    say("case plain_box_32 fp64 multistep 1000 steps")
    got = run(P, inst, 0, [1000])
    ref = run(P, inst, 1, [1000])
    assert got["launches"] == 2          # steps 0..99 under the stimulus, then 100..999
    same(got, ref)
    o = orc.Oracle(inst)
    _, oi = o.run(1000)
    vo = o.field("v")
    assert np.abs(got["v"] - vo).max() <= 1e-10 * np.abs(vo).max()
    To = o.field("tact")
    fin = np.isfinite(To)
    assert np.array_equal(np.isfinite(got["tact"]), fin)
    assert np.abs(got["tact"][fin] - To[fin]).max() <= 1e-9
    assert abs(got["q"][0] - oi.q_stim) <= 1e-12 * oi.q_stim
    assert abs(got["mass"][0] - oi.mass) <= 1e-10 * abs(oi.mass)


def test_large_grid_falls_back_to_one_launch_per_step(P):
    """A box of more bricks than fit on the device at once (128^3: 4096
    bricks) runs one launch per step, with the same results as asking for
    that explicitly."""
    inst = E.plain_box(128, steps=4, prec="f64")
    say("case plain_box_128 fp64 fallback")
    got = run(P, inst, 0, [4])
    ref = run(P, inst, 1, [4])
    assert got["bricks"] == 4096
    assert got["launches"] == 0
    same(got, ref)


def test_negative_steps_per_launch_refused(P):
    inst = E.plain_box(16, steps=1, prec="f64")
    with pytest.raises(P.EPError):
        P.Grid.from_instance(inst, steps_per_launch=-1)
