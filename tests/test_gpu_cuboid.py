"""The thesis's electrophysiology benchmark geometry (20 x 7 x 3 mm cuboid,
corner stimulus; Benchmark Studies section) on the GPU against the oracle at
the coarsest resolution (dx 0.5 mm), through the whole activation."""
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


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cuboid_activation_matches_oracle(P, orc, prec):
    """dx 0.5 mm, dt 0.05 ms, 60 ms explicit: every voxel activates, and the
    activation times agree with the oracle's (FP64: to 1e-9 ms; FP32: within
    one dt, the bar of the other FP32 runs), so does the potential at the end."""
    inst = E.cuboid(0.5, 0.05, t_end=60.0, prec=prec)
    say(f"case cuboid dx 0.5 {prec}: {inst.n}, {inst.steps} steps")
    g = P.Grid.from_instance(inst)
    o = orc.Oracle(inst)
    g.step(inst.steps)
    o.run(inst.steps)
    T, To = g.read("tact"), o.field("tact")
    v, vo = g.read("v"), o.field("v")
    g.close()
    assert np.isfinite(To).all() and np.isfinite(T).all()
    dT = np.abs(T - To).max()
    err = np.abs(v - vo).max() / np.abs(vo).max()
    say(f"cuboid {prec}: far corner T {T[-1, -1, -1]:.3f} ms (oracle {To[-1, -1, -1]:.3f}), "
        f"max dT {dT:.2e}, v err {err:.2e}")
    if prec == "f64":
        assert dT <= 1e-9 and err <= 1e-10
    else:
        assert dT <= inst.dt and err <= 1e-4
    # activation spreads away from the stimulated corner
    diag = [T[int(f * (inst.n[0] - 1)), int(f * (inst.n[1] - 1)), int(f * (inst.n[2] - 1))]
            for f in np.linspace(0.25, 1.0, 4)]
    assert all(b > a for a, b in zip(diag, diag[1:]))
