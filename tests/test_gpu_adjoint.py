"""GPU tests of the activation-time adjoint (ep_adjoint_scale): FP64 against
the oracle's discrete adjoint, FP32 against it at the proposed 1e-3, central
differences of the GPU loss, checkpoint-interval independence, the autograd
wrapper, errors, and properties at the full 128^3 / 500-step workload."""
import numpy as np
import pytest

import ep_inputs as E

pytestmark = pytest.mark.gpu

NSMALL = 32
STEPS = 240


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2302_12519_amd as P
    return P


@pytest.fixture(scope="module")
def small(orc):
    """32^3 shell, scale from seed 5001, target T* from the oracle run with
    the seed-5002 scale."""
    inst = E.adjoint_shell(NSMALL, steps=STEPS)
    tgt = E.adjoint_shell(NSMALL, steps=STEPS, target=True)
    o = orc.Oracle(dict_inst(tgt, "f64"))
    o.run(STEPS)
    tstar = o.field("tact")
    D0 = orc.tensors(inst.n, inst.mask, inst.fibre, None, inst.sigma_l, inst.sigma_t)
    ref = orc.Oracle(dict_inst(inst, "f64")).adjoint(D0, STEPS, tstar)
    return inst, tstar, D0, ref


def dict_inst(inst, prec):
    import dataclasses
    return dataclasses.replace(inst, prec=prec)


def gpu_adjoint(P, inst, tstar, prec, steps=STEPS, K=0, scale=None):
    g = P.Grid.from_instance(dict_inst(inst, prec))
    if scale is not None:
        g.set_conductivity(inst.fibre, scale, inst.sigma_l, inst.sigma_t)
    out = g.adjoint_scale(tstar, steps, K)
    g.close()
    return out


def test_fp64_matches_oracle_adjoint(P, small):
    inst, tstar, _, (L0, g0, used0, _) = small
    say(f"case adjoint FP64 n {NSMALL} steps {STEPS}")
    L, g, used = gpu_adjoint(P, inst, tstar, "f64")
    say(f"loss {L:.12e} oracle {L0:.12e} used {used}/{used0}")
    assert used == used0 and used > 0
    assert abs(L - L0) <= 1e-10 * abs(L0)
    err = np.abs(g - g0).max() / np.abs(g0).max()
    say(f"grad max rel err {err:.2e}")
    assert err <= 1e-9


def test_fp32_matches_oracle_adjoint(P, small):
    inst, tstar, _, (L0, g0, used0, _) = small
    say(f"case adjoint FP32 n {NSMALL} steps {STEPS}")
    L, g, used = gpu_adjoint(P, inst, tstar, "f32")
    err = np.linalg.norm(g - g0) / np.linalg.norm(g0)
    # element by element: max-abs normalised, and relative on the voxels
    # that carry the gradient (|g0| >= 1% of its largest value)
    emax = np.abs(g - g0).max() / np.abs(g0).max()
    big = np.abs(g0) >= 0.01 * np.abs(g0).max()
    erel = (np.abs(g - g0)[big] / np.abs(g0)[big]).max()
    say(f"loss {L:.6e} oracle {L0:.6e} used {used}/{used0} grad rel-norm err {err:.2e}, "
        f"max-abs normalised {emax:.2e}, relative on {int(big.sum())} large voxels {erel:.2e}")
    assert abs(used - used0) <= max(2, used0 // 1000)
    assert abs(L - L0) <= 1e-3 * abs(L0)
    assert err <= 1e-3
    assert emax <= 1e-4
    assert erel <= 1e-3


@pytest.mark.parametrize("K", [1, 7, STEPS])
def test_checkpoint_interval_does_not_change_bits(P, small, K):
    inst, tstar, _, _ = small
    say(f"case adjoint FP32 checkpoint every {K}")
    Lr, gr, ur = gpu_adjoint(P, inst, tstar, "f32", K=50)
    L, g, u = gpu_adjoint(P, inst, tstar, "f32", K=K)
    assert L == Lr and u == ur
    assert np.array_equal(g, gr)


def test_fp64_central_differences(P, small):
    """Central differences of the GPU loss.  The loss is piecewise smooth: a
    voxel that changes gate branch (v crossing v_gate one step earlier or
    later) or enters the loss set makes a jump; on this grid one falls
    within +-1e-5 along these directions, none within +-1e-6."""
    inst, tstar, _, _ = small
    say("case adjoint FP64 central differences")
    _, g, used = gpu_adjoint(P, inst, tstar, "f64")
    eps = 1e-6
    for d in E.fd_directions(inst.n, count=3):
        d = np.where(inst.mask > 0, d, 0.0)
        Lp, _, up = gpu_adjoint(P, inst, tstar, "f64", scale=inst.scale + eps * d)
        Lm, _, um = gpu_adjoint(P, inst, tstar, "f64", scale=inst.scale - eps * d)
        fd = (Lp - Lm) / (2 * eps)
        ad = float(np.sum(g * d))
        say(f"fd {fd:.10e} adjoint {ad:.10e} used {up} {um}")
        assert up == um == used
        assert abs(fd - ad) <= 1e-6 * abs(fd)


def test_autograd_function(P, small):
    import torch
    from paper_2302_12519_amd.adjoint import activation_time_loss
    inst, tstar, _, _ = small
    say("case adjoint through torch.autograd")
    g = P.Grid.from_instance(dict_inst(inst, "f32"))
    s = torch.tensor(inst.scale, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = activation_time_loss(g, s, inst.fibre, inst.sigma_l, inst.sigma_t, tstar, STEPS)
    (3.0 * loss).backward()
    L, gr, _ = gpu_adjoint(P, inst, tstar, "f32")
    assert loss.item() == L
    assert np.array_equal(s.grad.cpu().numpy(), 3.0 * gr)
    g.close()


def test_forward_only_call(P, small):
    """Without a gradient to compute (the scale does not require one, or
    grad=False), the call runs the forward simulation and the loss only: the
    same loss, voxel count and final state as the full call."""
    import torch
    from paper_2302_12519_amd.adjoint import activation_time_loss
    inst, tstar, _, _ = small
    say("case adjoint forward only")
    L, gr, used = gpu_adjoint(P, inst, tstar, "f32")
    g = P.Grid.from_instance(dict_inst(inst, "f32"))
    L2, g2, used2 = g.adjoint_scale(tstar, STEPS, 0, grad=False)
    v_a = g.read("v")
    g.close()
    assert g2 is None and L2 == L and used2 == used
    g = P.Grid.from_instance(dict_inst(inst, "f32"))
    g.step(STEPS)
    assert np.array_equal(g.read("v"), v_a)
    s = torch.tensor(inst.scale, dtype=torch.float64, device="cuda")   # no grad
    loss = activation_time_loss(g, s, inst.fibre, inst.sigma_l, inst.sigma_t, tstar, STEPS)
    g.close()
    assert loss.item() == L and not loss.requires_grad


def test_adjoint_errors(P, small):
    inst, tstar, _, _ = small
    ep = P.ep
    say("case adjoint errors")
    g = P.Grid.from_instance(dict_inst(inst, "f32"))
    with pytest.raises(P.EPError) as e:
        g.adjoint_scale(tstar, 0)
    assert e.value.status == ep.EP_ERR_ARG
    with pytest.raises(P.EPError) as e:
        g.adjoint_scale(tstar, 10, -1)
    assert e.value.status == ep.EP_ERR_ARG
    g.close()
    import dataclasses
    be = dataclasses.replace(dict_inst(inst, "f32"), diff="be_pcg", dt=0.1)
    g = P.Grid.from_instance(be)
    with pytest.raises(P.EPError) as e:
        g.adjoint_scale(tstar, 10)
    assert e.value.status == ep.EP_ERR_UNSUPPORTED
    g.close()
    g = P.Grid(inst.n, inst.h, inst.dt, mask=inst.mask, ionic=inst.ionic, stims=inst.stims)
    with pytest.raises(P.EPError) as e:
        g.adjoint_scale(tstar, 10)
    assert e.value.status == ep.EP_ERR_STATE
    g.close()


@pytest.mark.slow
def test_full_size_properties(P):
    """128^3 shell, 500 FP32 steps, checkpoints every 50: the forward part
    leaves exactly the state of ep_step, and the FP32 gradient agrees with
    the FP64 one (which matches the oracle at 32^3).  No finite differences
    here: with 0.63M voxels and a moving front, branch switches fall within
    any usable step."""
    inst = E.adjoint_shell(128)
    tgt = E.adjoint_shell(128, target=True)
    say("case adjoint full size: target run")
    gt = P.Grid.from_instance(tgt)
    gt.step(500)
    tstar = gt.read("tact")
    gt.close()
    say("case adjoint full size: FP32 K 50")
    g = P.Grid.from_instance(inst)
    L32, g32, used = g.adjoint_scale(tstar, 500, 50)
    v_adj, t_adj = g.read("v"), g.read("tact")
    g.close()
    g = P.Grid.from_instance(inst)
    g.step(500)
    assert np.array_equal(g.read("v"), v_adj)
    assert np.array_equal(g.read("tact"), t_adj, equal_nan=True)
    g.close()
    say("case adjoint full size: FP64 K 50")
    L64, g64, used64 = gpu_adjoint(P, inst, tstar, "f64", steps=500, K=50)
    err = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    say(f"loss {L32:.6e} / {L64:.6e}, used {used}/{used64}, grad rel-norm {err:.2e}")
    assert abs(used - used64) <= max(2, used64 // 1000)
    assert abs(L32 - L64) <= 1e-3 * abs(L64)
    assert err <= 1e-3
