"""GPU tests of batched serving (ep_batch_*): every request gives the same
bits alone, in a mix admitted under a tight HBM budget, and through the
per-grid FP32 path; results meet the FP32 bar against the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import ep_inputs as E
from parity_util import one_sided_activations

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2302_12519_amd as P
    from paper_2302_12519_amd import serve  # noqa: F401
    return P


@pytest.fixture(scope="module")
def stream6():
    return E.serving_stream(count=6, n_range=(24, 40), steps_range=(30, 120), burst=True)


def run_batch(P, reqs, budget, slots, K, fields=("v", "tact")):
    from paper_2302_12519_amd import serve
    b = P.ep.Batch(budget, max_slots=slots, steps_per_launch=K)
    out = serve.serve(b, [serve.InstanceRequest(r.rid, 0.0, r.inst) for r in reqs], fields=fields)
    st = b.stats()
    b.close()
    return out, st


def test_mix_alone_and_single_grid_are_bitwise_equal(P, stream6):
    say("case serving mix of 6, budget 8 MiB, 3 slots, K 8")
    mix, st = run_batch(P, stream6, 8 << 20, 3, 8)
    assert st["admitted"] == 6 and st["released"] == 6
    assert st["arena_peak"] <= 8 << 20
    assert st["graph_launches"] > 0
    for r in stream6:
        say(f"case serving alone request {r.rid} n {r.inst.n[0]} steps {r.inst.steps}")
        alone, _ = run_batch(P, [r], 64 << 20, 1, 5)
        g = P.Grid.from_instance(r.inst)
        g.step(r.inst.steps)
        single = {"v": g.read("v"), "tact": g.read("tact")}
        g.close()
        for f in ("v", "tact"):
            a, b_, c = mix["results"][r.rid][f], alone["results"][r.rid][f], single[f]
            assert np.array_equal(a, b_, equal_nan=True), (r.rid, f)
            assert np.array_equal(a, c, equal_nan=True), (r.rid, f)


def test_request_matches_oracle(P, orc, stream6):
    r = stream6[0]
    say(f"case serving vs oracle request {r.rid} n {r.inst.n[0]}")
    out, _ = run_batch(P, [r], 64 << 20, 1, 7)
    o = orc.Oracle(r.inst)
    o.run(r.inst.steps)
    v, ref = out["results"][r.rid]["v"], o.field("v")
    err = np.abs(v - ref).max() / np.abs(ref).max()
    T, To = out["results"][r.rid]["tact"], o.field("tact")
    fin = np.isfinite(T) & np.isfinite(To)
    say(f"serving vs oracle: err {err:.2e}, dT {np.abs(T[fin] - To[fin]).max() if fin.any() else 0:.2e}")
    assert err <= 1e-4
    if fin.any():
        assert np.abs(T[fin] - To[fin]).max() <= r.inst.dt


def test_mix_of_full_size_requests_matches_oracle(P, orc):
    """Four requests drawn like the serving workload (n 48..80, conductivity
    scale, excitability, 200-500 steps) served together in one mix; each
    result against its own FP64 oracle run: max-abs normalised potential
    <= 1e-4, activation times within one dt, and the same voxels activated
    (but for voxels the FP32 rounding leaves within 1e-4 of the threshold
    at the very end of the run)."""
    reqs = E.serving_stream(count=4, n_range=(48, 80), steps_range=(200, 500), burst=True)
    say("case serving mix of 4 (n " + ", ".join(str(r.inst.n[0]) for r in reqs) + ") vs oracle")
    out, st = run_batch(P, reqs, 1 << 30, 4, 16)
    assert st["admitted"] == 4
    for r in reqs:
        o = orc.Oracle(r.inst)
        o.run(r.inst.steps)
        v, ref = out["results"][r.rid]["v"], o.field("v")
        err = np.abs(v - ref).max() / np.abs(ref).max()
        T, To = out["results"][r.rid]["tact"], o.field("tact")
        fin = np.isfinite(T) & np.isfinite(To)
        odd, odd_ok = one_sided_activations(T, To, v, ref, r.inst.theta,
                                            r.inst.steps * r.inst.dt, r.inst.dt)
        dT = np.abs(T[fin] - To[fin]).max() if fin.any() else 0.0
        say(f"  request {r.rid}: n {r.inst.n[0]} steps {r.inst.steps} err {err:.2e} "
            f"dT {dT:.2e} activated {int(fin.sum())} one-sided {odd}")
        assert fin.sum() > 0
        assert err <= 1e-4
        assert dT <= r.inst.dt
        assert odd_ok and odd <= 10


def test_read_and_cancel_while_running(P, stream6):
    """A running request read between advances holds the state of a whole
    step: bitwise one of the per-grid path's states, at a multiple of K.
    Cancelling a running request frees its slot for a later one, and neither
    the request that keeps running nor the newcomer changes its bits."""
    ep = P.ep
    a, c, d = stream6[0], stream6[1], stream6[2]
    K = 4
    say(f"case serving read/cancel while running: requests {a.rid}, {c.rid}, {d.rid}, K {K}")
    b = ep.Batch(64 << 20, max_slots=2, steps_per_launch=K)
    ia = b.submit_instance(a.inst, n_steps=40)
    ic = b.submit_instance(c.inst, n_steps=40)
    b.advance()
    b.advance()
    va = b.read(ia, "v")
    g = P.Grid.from_instance(a.inst)
    match = None
    for s in range(1, 41):
        g.step(1)
        if np.array_equal(g.read("v"), va, equal_nan=True):
            match = s
            break
    g.close()
    say(f"  running read matches per-grid step {match}")
    assert match is not None and match % K == 0
    b.release(ic)
    idd = b.submit_instance(d.inst, n_steps=30)
    done = set()
    for _ in range(100):
        if len(done) == 2:
            break
        b.advance()
        done.update(b.finished())
    assert done == {ia, idd}
    res = {rid: {f: b.read(rid, f) for f in ("v", "tact")} for rid in (ia, idd)}
    st = b.stats()
    b.close()
    assert st["admitted"] == 3 and st["released"] == 1
    for rid, inst, steps in ((ia, a.inst, 40), (idd, d.inst, 30)):
        g = P.Grid.from_instance(inst)
        g.step(steps)
        for f in ("v", "tact"):
            assert np.array_equal(res[rid][f], g.read(f), equal_nan=True), (rid, f)
        g.close()


def test_batch_errors(P, stream6):
    ep = P.ep
    b = ep.Batch(4 << 20, max_slots=2, steps_per_launch=4)
    inst = stream6[1].inst
    say("case serving errors")
    # a request bigger than the whole budget
    big = E.serving_stream(count=1, n_range=(160, 160), steps_range=(10, 10), burst=True)[0].inst
    with pytest.raises(P.EPError) as e:
        b.submit_instance(big)
    assert e.value.status == ep.EP_ERR_OOM
    # stimuli with different windows
    st = [dataclasses.replace(s) for s in inst.stims]
    st[0].t_off = 2.0
    with pytest.raises(P.EPError) as e:
        b.submit(inst.n, inst.h, inst.dt, inst.mask, inst.ionic, st, inst.theta, inst.fibre,
                 None, inst.sigma_l, inst.sigma_t, 10)
    assert e.value.status == ep.EP_ERR_UNSUPPORTED
    # unstable explicit step
    with pytest.raises(P.EPError) as e:
        b.submit(inst.n, inst.h, 0.5, inst.mask, inst.ionic, inst.stims, inst.theta, inst.fibre,
                 None, inst.sigma_l, inst.sigma_t, 10)
    assert e.value.status == ep.EP_ERR_ARG
    # queue, then release before admission
    rid = b.submit_instance(inst, n_steps=5)
    b.release(rid)
    assert b.stats()["queued"] == 0
    b.close()
