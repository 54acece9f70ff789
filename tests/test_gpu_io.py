"""GPU test of ep_read_state_device: fields written in box layout straight
into device memory (a torch tensor) agree with the host read."""
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


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_read_state_device_matches_host_read(P, prec):
    """ep_read_state_device writes every field in box layout into a torch
    tensor: the same values as ep_read_state (FP64 output bitwise, FP32
    output the rounded values), 0 / +inf outside tissue."""
    import torch
    inst = be_shell(17, prec=prec) if prec == "f64" else E.aniso_be(24, steps=20)
    say(f"case device read {prec}")
    g = P.Grid.from_instance(inst)
    g.step(15)
    for f in ("v", "w", "tact", "phi"):
        host = g.read(f)
        d64 = g.read_tensor(f, torch.float64).cpu().numpy()
        d32 = g.read_tensor(f, torch.float32).cpu().numpy()
        assert d64.shape == tuple(inst.n)
        assert np.array_equal(d64, host, equal_nan=True), f
        assert np.array_equal(d32, host.astype(np.float32), equal_nan=True), f
        outside = inst.mask == 0
        fill = np.inf if f == "tact" else 0.0
        assert np.all(d64[outside] == fill), f
    g.close()


def test_grid_in_caller_arena_matches_own_allocation(P):
    """A grid built inside a caller-owned torch buffer (ep_grid_desc.arena)
    gives bitwise the same run as one that allocates, takes no more than the
    peak ep_grid_stats reported, and a too-small arena is EP_ERR_OOM."""
    import torch
    inst = E.aniso_be(32, steps=60)
    say("case arena grid aniso_be_32 fp32")
    ref = P.Grid.from_instance(inst)
    ref.step(60)
    v_ref, t_ref = ref.read("v"), ref.read("tact")
    need = ref.stats()["device_bytes"]
    ref.close()
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    g = P.Grid.from_instance(inst, arena=arena)
    g.step(60)
    assert np.array_equal(g.read("v"), v_ref)
    assert np.array_equal(g.read("tact"), t_ref, equal_nan=True)
    assert g.stats()["device_bytes"] <= need
    g.close()
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.EPError) as e:
        P.Grid.from_instance(inst, arena=small)
    assert e.value.status == P.ep.EP_ERR_OOM


def test_bidomain_bath_grid_in_caller_arena(P):
    """The bidomain grid with a bath, whose conductivity set-up builds the
    coarse operator in large temporaries (the FP64 matrix and its panels),
    runs bitwise the same inside an arena of the reported peak size."""
    import torch
    inst = E.bidomain_bath(24, steps=20)
    say("case arena grid bidomain_bath_24 fp32")
    ref = P.Grid.from_instance(inst)
    ref.step(20)
    v_ref, p_ref = ref.read("v"), ref.read("phi")
    need = ref.stats()["device_bytes"]
    ref.close()
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    g = P.Grid.from_instance(inst, arena=arena)
    g.step(20)
    assert np.array_equal(g.read("v"), v_ref) and np.array_equal(g.read("phi"), p_ref)
    assert g.stats()["device_bytes"] <= need
    g.close()
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.EPError) as e:
        P.Grid.from_instance(inst, arena=small)
    assert e.value.status == P.ep.EP_ERR_OOM


def test_kernel_timing_on_a_sample_of_steps(P):
    """ep_kernel_timing_period: with a period of 4 only the launches of steps
    whose index is a multiple of 4 are timed, each implicit step's launches
    keep their roles (one init, one set-up and one last-update launch per
    timed step), and the results do not change."""
    inst = be_shell(17, prec="f32")
    say("case kernel timing period")
    runs = {}
    for every in (1, 4):
        g = P.Grid.from_instance(inst)
        g.step(3)                                    # steps 0..2
        g.kernel_timing(True, every=every)
        g.step(12)                                   # steps 3..14: 4, 8, 12 sampled
        counts = {k: g.kernel_time(k)[1] for k in ("be_init", "cg_setup", "cg_update",
                                                   "stencil")}
        runs[every] = (counts, g.read("v"))
        g.close()
    full, sampled = runs[1][0], runs[4][0]
    assert full["be_init"] == full["cg_setup"] == full["cg_update"] == 12
    assert sampled["be_init"] == sampled["cg_setup"] == sampled["cg_update"] == 3
    assert 0 <= sampled["stencil"] < full["stencil"]
    assert np.array_equal(runs[1][1], runs[4][1])
    g = P.Grid.from_instance(inst)
    with pytest.raises(P.EPError):
        g.kernel_timing(True, every=0)
    g.close()
