"""Benchmark: voxel-steps/s of the voxel cardiac-EP time step on one MI355X.

Default workload: anisotropic monodomain on a 256^3 ventricle-like shell
(~30 % tissue, sigma 0.2/0.05 mm^2/ms, transmural +-60 deg fibres, 16 seeded
ball stimuli), FP32 state, implicit-Euler diffusion by Jacobi-PCG, dt 0.05 ms.
One "step" is one full operator-split time step (reaction, PCG diffusion
solve, activation times).  Inputs are seeded and synthetic and already
resident in HBM when timing starts.

Prints ONE JSON line with the metric, the live-measured roofline of the
dominant kernel (HIP events on the library's stream) and the FP64 oracle
timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
# the timed region brackets the dominant kernel with HIP events in this
# fraction of its steps (every TIMING_EVERY-th step index)
TIMING_EVERY = 10

# Algorithmic HBM bytes per tissue voxel for one launch of each kernel
# (FP32 state; each array read or written once):
#   implicit-step init (k_be_init): reads v, w, the previous step's v, b and
#             Q, two older increments d (28 B) and the 6 operator weights
#             (24 B); writes x0, b, d, Q, w, z0 = M^-1 r0 (24 B)          -> 76 B
#   PCG launch 0 (k_pcg_step, first): reads z (4 B) and the weights
#             (24 B), writes p, t = M^-1 q (8 B)                        -> 36 B
#   PCG iteration (k_pcg_step): reads x, z, t, p (16 B) and the weights
#             (24 B), writes x, z, p, t (16 B)                          -> 56 B
#   PCG last x update (k_pcg_step, solve done): reads x, p, writes x    -> 12 B
#   elliptic inner iteration, two-level preconditioner:
#     update (k_cg2_update): reads z, w, p, s, x, r (24 B), writes p, s,
#             x, r (16 B)                                               -> 40 B
#     apply (k_cg2_apply): reads r, D^-1 (8 B) and the weights (24 B),
#             writes z, w (8 B)                                         -> 40 B
#     coarse correction: the scaled FP16 coarse inverse, 2 B per entry (not
#             per voxel)
#   explicit fused step: reads v, w (8 B) + 24 B weights, writes v, w   -> 40 B
#   adjoint step: reads lambda_v, lambda_w, v, w, v_next, crossing step (24 B),
#             weights and unscaled tensors (48 B), mask (1 B), gradient (8 B,
#             FP64); writes lambda_v, lambda_w (8 B) and gradient (8 B)  -> 97 B
ALGO_BYTES = {"be_init": 76, "pcg_first": 36, "pcg_iter": 56, "pcg_final": 12,
              "cg2_update": 40, "cg2_apply": 40, "stencil_explicit": 40, "adjoint_step": 97}
STEP_KERNELS = {"be_init": ("k_be_init<float>", "be_init"),
                "cg_setup": ("k_pcg_step<float> (launch 0: p0 = z0, q0 = K p0)", "pcg_first"),
                "stencil": ("k_pcg_step<float> (iteration)", "pcg_iter"),
                "cg_update": ("k_pcg_step<float> (last x update)", "pcg_final")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid edge of the shell workload")
    ap.add_argument("--rtol", type=float, default=1e-7)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget for the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-err", action="store_true",
                    help="skip the checks against the oracle (headline one-step error, "
                         "serving sample runs)")
    ap.add_argument("--bidomain", type=int, default=192,
                    help="grid edge of the bidomain line (0 = skip)")
    ap.add_argument("--adjoint", type=int, default=128,
                    help="grid edge of the adjoint line (0 = skip)")
    ap.add_argument("--serving", type=int, default=64,
                    help="requests of the serving measurement (0 skips it)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-box FP64 line")
    ap.add_argument("--serving-k", type=int, default=32,
                    help="steps per captured graph launch of the serving line")
    ap.add_argument("--jacobi", type=int, default=256,
                    help="grid edge of the fixed-sweep Jacobi line (0 = skip)")
    ap.add_argument("--explicit27", type=int, default=256,
                    help="shell size of the A27 vs 19-point explicit line (0: skip)")
    ap.add_argument("--bath", type=int, default=128,
                    help="box size of the bidomain-with-bath (ECG) line (0: skip)")
    ap.add_argument("--no-cuboid", action="store_true",
                    help="skip the benchmark-geometry cuboid line")
    ap.add_argument("--only", choices=["serving", "plain", "bidomain", "adjoint", "jacobi",
                                       "cuboid", "explicit27", "bath"],
                    help="run one side workload alone and print its JSON (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--traffic-file", default=None,
                    help="counter summary of the dominant kernel (default: "
                         "profiles/traffic_<kernel>_aniso_be_<n>.txt)")
    return ap.parse_args()


def read_traffic(path, kernel):
    """Per-launch HBM bytes of `kernel` from the committed counter summary
    (lines 'kernel: K', 'traffic_bytes_per_launch: X' and
    'kernel_source_sha: S'); None if absent, taken on another kernel, or on
    another version of the kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        import hashlib
        src = open(os.path.join(ROOT, "paper_2302_12519_amd", "csrc", "ep_kernels.hip"), "rb").read()
        if vals.get("kernel_source_sha") != hashlib.sha256(src).hexdigest()[:16]:
            return None
        if vals.get("kernel") != kernel:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(inst, state, gpu_iters_per_step, budget_s):
    """The FP64 oracle on the host cores, on the GPU's own step window: it
    starts from the GPU's state at the first timed step (v, w, step) and
    solves each implicit step to the same relative residual (pcg_rtol).  One
    warm-up step, then the median of 3 runs of the same k steps (k sized to
    the budget), each from that state; then one step on a single thread."""
    import oracle
    v, w, step = state
    o = oracle.Oracle(inst, cg_rtol=inst.pcg_rtol)

    def run(k):
        o.set_state(v=v, w=w, tact=np.full(inst.nb, np.inf), step=step)
        t = time.perf_counter()
        _, info = o.run(k)
        return time.perf_counter() - t, info.cg_iters

    t1, _ = run(1)
    k = max(1, int(budget_s / 3.0 / max(t1, 1e-9)))
    runs = [run(k) for _ in range(3)]
    times = sorted(r[0] for r in runs)
    med = times[1]
    cores = oracle.threads()
    oracle.set_threads(1)
    t_one, _ = run(1)
    oracle.set_threads(cores)
    return {"value": inst.nt * k / med, "unit": "voxel-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"the GPU's timed window of the same {inst.n[0]}^3 workload: from the "
                      f"GPU state at step {step}, {k} step(s) per run, median of 3 runs after "
                      f"1 warm-up step; FP64, CG to the same rtol {inst.pcg_rtol:g}",
            "runs_s": [r[0] for r in runs], "steps_per_run": k,
            "oracle_cg_iters_per_step": runs[0][1] / k,
            "gpu_cg_iters_per_step": gpu_iters_per_step,
            "value_1_thread": inst.nt / t_one, "seconds_1_thread_step": t_one,
            "cpu_model": oracle.cpu_model()}


def oracle_step_error(inst, g, cg_rtol=1e-10, fields=("v",)):
    """err_vs_oracle of a side line: one oracle step (FP64) from the GPU's
    current state against the GPU's own next step; max |difference| over
    max |oracle| per field."""
    import oracle
    o = oracle.Oracle(inst, cg_rtol=cg_rtol)
    kw = dict(v=g.read("v"), w=g.read("w"), step=g.step_index)
    if "phi" in fields:
        kw["phi"] = g.read("phi")
    o.set_state(**kw)
    o.run(1)
    g.step(1)
    out = {"kind": f"one FP64 oracle step from the GPU state at step {kw['step']}"}
    for f in fields:
        a, b = g.read(f), o.field(f)
        out[f"max_abs_norm_{f}"] = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    return out


def oracle_run_error(inst, results, steps):
    """err_vs_oracle of a whole run from rest: the FP64 oracle runs the same
    steps; v as max-abs normalised difference, T_act as the largest
    difference (ms) where both activated, plus the voxels activated on one
    side only."""
    import oracle
    o = oracle.Oracle(inst)
    o.run(steps)
    out = {"kind": f"whole run of {steps} steps from rest against the FP64 oracle"}
    if "v" in results:
        vo = o.field("v")
        out["max_abs_norm_v"] = float(np.abs(results["v"] - vo).max() / np.abs(vo).max())
    if "tact" in results:
        T, To = results["tact"], o.field("tact")
        both = np.isfinite(T) & np.isfinite(To)
        out["t_act_max_diff_ms"] = float(np.abs(T[both] - To[both]).max()) if both.any() else 0.0
        out["activated_one_side_only"] = int((np.isfinite(T) != np.isfinite(To)).sum())
    return out


def bench_serving(count, K=32, n_err=3):
    """Serving workload: `count` requests (grids 48^3..160^3 shells, sigma x
    U[0.5,1.5], excitability U[0.8,1.2], 200..1000 FP32 explicit steps).  A
    burst run measures capacity; a Poisson stream at 0.9 x capacity gives
    p50/p99 latency.  The same requests one at a time on the plain FP64
    per-grid path give the comparison: its grids are built before its timed
    steps (step-only time), and separately with their creation (end to end).
    err_vs_oracle: the `n_err` cheapest requests of both paths against their
    own FP64 oracle runs."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid, serve
    from paper_2302_12519_amd.ep import Batch

    t = time.perf_counter()
    reqs = E.serving_stream(count=count, burst=True)
    gen_s = time.perf_counter() - t
    work = sum(r.inst.nt * r.inst.steps for r in reqs)
    budget, slots = 16 << 30, count
    sample = {r.rid for r in sorted(reqs, key=lambda r: r.inst.nt * r.inst.steps)[:n_err]}

    def run(rs):
        b = Batch(budget, max_slots=slots, steps_per_launch=K)
        out = serve.serve(b, rs, fields=("tact",),
                          fields_of=lambda rid: ("v", "tact") if rid in sample else ("tact",))
        b.close()
        return out

    burst = run([serve.InstanceRequest(r.rid, 0.0, r.inst) for r in reqs])
    capacity = count / burst["makespan"]
    rate = 0.9 * capacity
    arrivals = E.serving_stream(count=count, rate=rate, burst=False)
    poisson = run([serve.InstanceRequest(r.rid, a.arrival, r.inst)
                   for r, a in zip(reqs, arrivals)])
    # the plain one-request-at-a-time FP64 GPU path on the same requests
    torch.cuda.synchronize()
    t = time.perf_counter()
    grids = [Grid.from_instance(r.inst, prec="f64") for r in reqs]
    torch.cuda.synchronize()
    build64 = time.perf_counter() - t
    t = time.perf_counter()
    for r, g in zip(reqs, grids):
        g.step(r.inst.steps)
    torch.cuda.synchronize()
    step64 = time.perf_counter() - t
    res64 = {}
    for r, g in zip(reqs, grids):
        if r.rid in sample:
            res64[r.rid] = {"v": g.read("v"), "tact": g.read("tact")}
        g.close()
    errs = []
    for r in reqs:
        if r.rid not in sample:
            continue
        e32 = oracle_run_error(r.inst, burst["results"][r.rid], r.inst.steps)
        e64 = oracle_run_error(r.inst, res64[r.rid], r.inst.steps)
        errs.append({"request": r.rid, "n": r.inst.n[0], "steps": r.inst.steps,
                     "fp32_batched": {k: v for k, v in e32.items() if k != "kind"},
                     "fp64_per_grid": {k: v for k, v in e64.items() if k != "kind"}})
    t64 = build64 + step64
    rate32 = work / burst["makespan"]
    return {"requests": count, "voxel_steps": work, "steps_per_graph": K,
            "burst": {"makespan_s": burst["makespan"], "voxel_steps_per_s": rate32,
                      "p50_s": burst["p50"], "p99_s": burst["p99"]},
            "poisson": {"rate_per_s": rate, "makespan_s": poisson["makespan"],
                        "voxel_steps_per_s": work / poisson["makespan"],
                        "p50_s": poisson["p50"], "p99_s": poisson["p99"]},
            "fp64_one_at_a_time": {"build_s": build64, "step_s": step64,
                                   "voxel_steps_per_s_steps_only": work / step64,
                                   "voxel_steps_per_s_end_to_end": work / t64},
            "speedup_vs_fp64_end_to_end": rate32 / (work / t64),
            "speedup_vs_fp64_steps_only": rate32 / (work / step64),
            "speedup_note": "the batched makespan includes admission (uploads, weight "
                            "kernels) of every request; steps_only leaves the FP64 "
                            "path's grid builds out",
            "err_vs_oracle": {"kind": "whole runs of the cheapest requests against the FP64 "
                                      "oracle", "requests": errs},
            "generation_s": gen_s}


def bench_plain_fp64(steps=1000):
    """Plain monodomain 32^3 FP64 box (dt 0.01, 1000 steps from rest, the
    stimulus on for the first 1 ms): microseconds per step with several
    steps per cooperative launch (the library's default at this size) and
    with one launch per step, each the median of 3 timed runs after a
    warm-up run; the multi-step result's error against the oracle."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    inst = E.plain_box(32, steps=steps, prec="f64")
    out = {}
    for name, spl in (("multistep", 0), ("one_launch_per_step", 1)):
        g = Grid.from_instance(inst, steps_per_launch=spl)
        times = []
        for rep in range(4):
            g.write("v", np.zeros(inst.n))
            g.write("w", np.ones(inst.n))
            g.write("tact", np.full(inst.n, np.inf))
            g.step_index = 0
            torch.cuda.synchronize()
            t = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t)
        dt = float(np.median(times))
        res = {"us_per_step": 1e6 * dt / steps, "voxel_steps_per_s": inst.nt * steps / dt}
        if spl == 0:
            g.kernel_timing(kernels=["multistep"])
            g.write("v", np.zeros(inst.n))
            g.write("w", np.ones(inst.n))
            g.write("tact", np.full(inst.n, np.inf))
            g.step_index = 0
            g.step(steps)
            ms, launches = g.kernel_time("multistep")
            res["launches"] = launches
            res["kernel_us_per_step"] = 1e3 * ms / steps
            res["err_vs_oracle"] = oracle_run_error(
                inst, {"v": g.read("v"), "tact": g.read("tact")}, steps)
        g.close()
        out[name] = res
    out["us_per_step"] = out["multistep"]["us_per_step"]
    out["voxel_steps_per_s"] = out["multistep"]["voxel_steps_per_s"]
    out["err_vs_oracle"] = out["multistep"]["err_vs_oracle"]
    return out


def bench_jacobi(n, steps=200, sweeps=(4, 10)):
    """The thesis's own implicit solver on the same shell as the headline:
    a fixed number of Jacobi sweeps per step from the current potential
    (no stopping test).  For each sweep count: voxel-steps/s over `steps`
    steps from rest, and the largest difference of v from the PCG solve
    (rtol 1e-7) after the same steps, relative to max |v|."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    inst = E.aniso_be(n, steps=steps)
    inst.pcg_rtol = 1e-7
    ref = Grid.from_instance(inst)
    ref.step(steps)
    v_ref = ref.read("v")
    ref.close()
    out = {"workload": f"aniso_be_{n}: {inst.nt} tissue voxels, {steps} FP32 steps from rest"}
    for k in sweeps:
        inst.diff, inst.jacobi_sweeps = "be_jacobi", k
        g = Grid.from_instance(inst)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        v = g.read("v")
        err = oracle_step_error(inst, g)
        g.close()
        out[f"sweeps_{k}"] = {"voxel_steps_per_s": inst.nt * steps / dt,
                              "ms_per_step": 1e3 * dt / steps,
                              "max_rel_diff_vs_pcg": float(np.abs(v - v_ref).max()
                                                           / np.abs(v_ref).max()),
                              "err_vs_oracle": err}
    return out


def bench_explicit27(n, steps=200):
    """The thesis's corner-gradient operator A27 beside the 19-point operator
    on the headline shell: FP32 explicit steps (dt 0.05 ms) from rest.  For
    each: voxel-steps/s over `steps` untimed-event steps, then the fused
    kernel's mean duration from a second pass with events on it, its
    algorithmic rate (40 B per tissue voxel), and how far the two operators'
    activation times lie apart after the same steps (v itself differs by
    O(1) wherever the fronts are a voxel apart)."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    inst = E.aniso_be(n, steps=steps)
    out = {"workload": f"aniso_{n}: {inst.nt} tissue voxels, {steps} FP32 explicit steps "
                       f"of dt {inst.dt} from rest"}
    vs, ts = {}, {}
    for diff in ("explicit", "explicit27"):
        inst.diff = diff
        g = Grid.from_instance(inst)
        g.step(5)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        vs[diff] = g.read("v")
        ts[diff] = g.read("tact")
        g.kernel_timing(True, kernels=["stencil"])
        g.step(50)
        ms, cnt = g.kernel_time("stencil")
        g.kernel_timing(False)
        err = oracle_step_error(inst, g)
        g.close()
        k_us = 1e3 * ms / max(cnt, 1)
        out[diff] = {"voxel_steps_per_s": inst.nt * steps / sec, "ms_per_step": 1e3 * sec / steps,
                     "kernel_us": k_us,
                     "kernel_GBps": ALGO_BYTES["stencil_explicit"] * inst.nt / (k_us * 1e-6) / 1e9,
                     "err_vs_oracle": err}
    a, b = vs["explicit27"], vs["explicit"]
    out["max_rel_diff_v_27_vs_19"] = float(np.abs(a - b).max() / np.abs(b).max())
    ta, tb = ts["explicit27"], ts["explicit"]
    both = np.isfinite(ta) & np.isfinite(tb)
    d = ta[both] - tb[both]
    out["activated"] = {"explicit": int(np.isfinite(tb).sum()),
                        "explicit27": int(np.isfinite(ta).sum())}
    out["t_act_27_minus_19_ms"] = {"mean": float(d.mean()), "max_abs": float(np.abs(d).max())}
    return out


def bench_bath(n, steps=40, every=10):
    """Bidomain with a conducting bath (the ECG configuration): an n^3 box,
    a shell heart inside it, every other voxel bath.  FP32 steps of dt 0.05
    ms from rest: ms per step, the elliptic solve's inner iterations per
    step, and the six leads every `every` steps."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    inst = E.bidomain_bath(n, steps=steps)
    g = Grid.from_instance(inst)
    leads, sec, inner = [], 0.0, 0
    for k in range(steps // every):
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = g.step(every)
        torch.cuda.synchronize()
        sec += time.perf_counter() - t
        inner += info["cg_iters"]
        leads.append([float(x) for x in g.ecg(inst.electrodes)])
    err = elliptic_residual(inst, g)
    g.close()
    done = every * (steps // every)
    return {"workload": f"bidomain_bath_{n}: {inst.nt} heart voxels, {int(inst.bath.sum())} "
                        f"bath voxels, {done} FP32 steps of dt {inst.dt} from rest",
            "ms_per_step": 1e3 * sec / done, "inner_iters_per_step": inner / done,
            "heart_voxel_steps_per_s": inst.nt * done / sec,
            "leads_every_ms": every * inst.dt, "leads_I_II_III_aVR_aVL_aVF": leads,
            "err_vs_oracle": err}


def bench_cuboid(dxs=(0.5, 0.2, 0.1), dt=0.005, t_end=60.0):
    """The thesis's benchmark geometry (20 x 7 x 3 mm cuboid, 1.5 mm corner
    stimulus) at each voxel width, FP32 explicit, dt 0.005 ms: activation
    time (ms) at points along the long diagonal and at the far corner, and
    the GPU time of the run."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    out = {"dt_ms": dt, "t_end_ms": t_end, "diagonal_fractions": [0.25, 0.5, 0.75, 1.0]}
    for dx in dxs:
        inst = E.cuboid(dx, dt, t_end=t_end)
        g = Grid.from_instance(inst)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.step(inst.steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        T = g.read("tact")
        if dx >= 0.5:
            err = oracle_run_error(inst, {"v": g.read("v"), "tact": T}, inst.steps)
        else:
            err = oracle_step_error(inst, g)
        g.close()
        n = inst.n
        diag = [float(T[int(f * (n[0] - 1)), int(f * (n[1] - 1)), int(f * (n[2] - 1))])
                for f in out["diagonal_fractions"]]
        out[f"dx_{dx:g}"] = {"grid": list(n), "steps": inst.steps, "seconds": sec,
                             "voxel_steps_per_s": inst.nt * inst.steps / sec,
                             "t_act_diagonal_ms": diag,
                             "t_act_far_corner_ms": float(T[-1, -1, -1]),
                             "err_vs_oracle": err}
    return out


def elliptic_residual(inst, g):
    """err_vs_oracle of a bidomain line: the elliptic solve for the run's
    final v (ep_solve_elliptic), put through the oracle's FP64 operators:
    ||A_i v - K phi|| / ||A_i v|| with K = -(A_i on the heart + A_e over the
    elliptic domain), the relative residual the refinement drives to
    ell_rtol."""
    import oracle
    o = oracle.Oracle(inst)
    g.solve_elliptic(inst.ell_rtol, 12)
    v, phi = g.read("v"), g.read("phi")
    b = oracle.apply(inst.n, inst.h, inst.mask, o.Di, v)
    if inst.bath is not None:
        dom = ((inst.mask > 0) | (inst.bath > 0)).astype(np.uint8)
        De = np.zeros_like(o.De)
        m, bt = inst.mask.ravel() > 0, inst.bath.ravel() > 0
        De[:, m] = o.De[:, m]
        De[:3, bt] = inst.sigma_bath
    else:
        dom, De = inst.mask, o.De
    Kphi = -(oracle.apply(inst.n, inst.h, inst.mask, o.Di, phi)
             + oracle.apply(inst.n, inst.h, dom, De, phi))
    # the solve's right-hand side is projected to zero sum over the domain
    d = dom > 0
    b = np.where(d, b - b[d].mean(), 0.0)
    return {"kind": "relative residual of the last elliptic solve through the FP64 oracle's "
                    "operators", "relres": float(np.linalg.norm(b - Kphi) / np.linalg.norm(b)),
            "ell_rtol": inst.ell_rtol}


def bench_bidomain(n, steps=20, warmup=3):
    """Bidomain n^3 shell (sigma_i 0.17/0.019, sigma_e 0.62/0.24, dt 0.05):
    per-step time of the full step (ionic, elliptic FP32 PCG with the
    two-level preconditioner inside FP64 refinement to 1e-8, parabolic
    update), timed on `steps` steps after `warmup` from rest, with per-kernel
    averages: an inner iteration is an update, a coarse correction and an
    apply launch."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    n_diag = 5
    inst = E.bidomain(n, steps=warmup + steps + n_diag)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = Grid.from_instance(inst)      # includes the coarse operator and its inverse
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    g.step(warmup)
    torch.cuda.synchronize()
    t = time.perf_counter()
    info = g.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # per-kernel averages on further steps with every launch timed (the
    # events between launches would slow the timed steps)
    g.kernel_timing(True)
    g.step(n_diag)
    torch.cuda.synchronize()
    it_ms, it_n = g.kernel_time("stencil")      # apply launches of the inner iterations
    up_ms, up_n = g.kernel_time("cg_update")    # update launches
    co_ms, co_n = g.kernel_time("coarse")       # aggregate sums + coarse GEMV
    rs_ms, rs_n = g.kernel_time("resid")
    pb_ms, pb_n = g.kernel_time("parabolic")
    g.kernel_timing(False)
    err = elliptic_residual(inst, g)
    g.close()
    avg_ap = it_ms / max(it_n, 1)
    avg_up = up_ms / max(up_n, 1)
    avg_co = co_ms / max(co_n, 1)
    avg_it = avg_ap + avg_up + avg_co
    return {"workload": f"bidomain_{n}: {inst.nt} tissue voxels, {steps} steps after {warmup}",
            "voxel_steps_per_s": inst.nt * steps / dt, "ms_per_step": 1e3 * dt / steps,
            "setup_s": setup_s,
            "inner_iters_per_step": info["cg_iters"] / steps,
            "outer_per_step": info["ell_outer"] / steps, "relres_last": info["relres"],
            "inner_iter_avg_us": 1e3 * avg_it,
            "inner_apply_avg_us": 1e3 * avg_ap, "inner_update_avg_us": 1e3 * avg_up,
            "inner_coarse_avg_us": 1e3 * avg_co,
            "inner_iter_achieved_gbs": (ALGO_BYTES["cg2_update"] + ALGO_BYTES["cg2_apply"])
                                       * inst.nt / (avg_it * 1e-3) / 1e9,
            "resid64_avg_us": 1e3 * rs_ms / max(rs_n, 1),
            "parabolic_avg_us": 1e3 * pb_ms / max(pb_n, 1),
            "err_vs_oracle": err}


def bench_adjoint(n, steps=500, K=50):
    """Activation-time adjoint on the n^3 shell (smooth scale in [0.5, 1.5],
    8 stimuli, FP32 explicit, dt 0.04): one ep_adjoint_scale call (forward
    with checkpoints every K, per-segment recompute, adjoint steps); the
    target comes from a GPU forward run with the second scale field."""
    import ep_inputs as E
    import torch
    from paper_2302_12519_amd import Grid
    inst = E.adjoint_shell(n, steps=steps)
    gt = Grid.from_instance(E.adjoint_shell(n, steps=steps, target=True))
    gt.step(steps)
    tstar = gt.read("tact")
    gt.close()
    g = Grid.from_instance(inst)
    g.adjoint_scale(tstar, steps, K)          # warm-up (allocates the work block)
    g.write("v", np.zeros(inst.n))
    g.write("w", np.ones(inst.n))
    g.step_index = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    loss, grad, used = g.adjoint_scale(tstar, steps, K)
    dt = time.perf_counter() - t
    # per-kernel averages from one more call with every launch timed
    g.write("v", np.zeros(inst.n))
    g.write("w", np.ones(inst.n))
    g.step_index = 0
    torch.cuda.synchronize()
    g.kernel_timing(True)
    g.adjoint_scale(tstar, steps, K)
    st_ms, st_n = g.kernel_time("stencil")
    ad_ms, ad_n = g.kernel_time("adjoint")
    g.kernel_timing(False)
    g.close()
    # accuracy: the same call in FP64 (the FP64 path matches the oracle's
    # discrete adjoint to 1e-9 on the test grids)
    g = Grid.from_instance(inst, prec="f64")
    loss64, grad64, used64 = g.adjoint_scale(tstar, steps, K)
    g.close()
    m = inst.mask > 0
    err = {"kind": "FP32 gradient against the FP64 GPU adjoint of the same call",
           "grad_rel_norm": float(np.linalg.norm(grad[m] - grad64[m]) / np.linalg.norm(grad64[m])),
           "grad_max_abs_norm": float(np.abs(grad[m] - grad64[m]).max() / np.abs(grad64[m]).max()),
           "loss_rel": float(abs(loss - loss64) / abs(loss64)), "n_used_fp64": used64}
    avg_ad = ad_ms / max(ad_n, 1)
    return {"workload": f"adjoint_{n}: {inst.nt} tissue voxels, {steps} FP32 steps, "
                        f"checkpoints every {K}",
            "voxel_steps_per_s": inst.nt * steps / dt, "seconds": dt,
            "loss": loss, "n_used": used,
            "forward_recompute_avg_us": 1e3 * st_ms / max(st_n, 1), "forward_launches": st_n,
            "adjoint_avg_us": 1e3 * avg_ad, "adjoint_launches": ad_n,
            "adjoint_achieved_gbs": ALGO_BYTES["adjoint_step"] * inst.nt / (avg_ad * 1e-3) / 1e9,
            "err_vs_oracle": err}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the library runs each grid on one GPU; --gpus {a.gpus} is not "
              "supported (grids are not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    import ep_inputs as E
    from paper_2302_12519_amd import Grid

    if a.copy_calibration:
        # plain copy of known size: 1 GiB read + 1 GiB written
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if a.only:
        side = {"serving": lambda: bench_serving(a.serving or 64, a.serving_k,
                                                 0 if a.no_err else 3),
                "plain": bench_plain_fp64,
                "bidomain": lambda: bench_bidomain(a.bidomain or 192),
                "adjoint": lambda: bench_adjoint(a.adjoint or 128),
                "jacobi": lambda: bench_jacobi(a.jacobi or 256),
                "cuboid": bench_cuboid,
                "explicit27": lambda: bench_explicit27(a.explicit27 or 256),
                "bath": lambda: bench_bath(a.bath or 128)}[a.only]
        print(json.dumps({a.only: side()}), flush=True)
        return

    from paper_2302_12519_amd.ep import stream_bandwidth
    copy_gbs, read_gbs = stream_bandwidth(1 << 30, 5)

    t_gen = time.perf_counter()
    inst = E.aniso_be(a.n, steps=a.warmup + a.steps)
    inst.pcg_rtol = a.rtol
    gen_s = time.perf_counter() - t_gen
    g = Grid.from_instance(inst)
    st = g.stats()
    print(f"# workload {inst.name}: N_t {inst.nt}, bricks {st['n_bricks']}, "
          f"device {st['device_bytes'] / 2**20:.0f} MiB, generated in {gen_s:.1f} s",
          file=sys.stderr, flush=True)

    if a.warmup:
        g.step(a.warmup)
    # per-kernel breakdown, every kernel timed, on the steps after the
    # warm-up; it also names the dominant kernel (the largest share of the
    # step's kernel time)
    n_diag = min(a.steps, 200)
    g.kernel_timing(True)
    g.step(n_diag)
    torch.cuda.synchronize()
    times = {k: g.kernel_time(k) for k in list(STEP_KERNELS) + ["cg_tail"]}
    dom = max(STEP_KERNELS, key=lambda k: times[k][0])
    dom_name, dom_bytes = STEP_KERNELS[dom]
    # timed region: events around the dominant kernel's launches only, in
    # every TIMING_EVERY-th step (an event pair delays the launch that follows
    # by ~9 us; around every launch it would add ~35 us to a 0.4 ms step)
    g.kernel_timing(True, kernels=[dom], every=TIMING_EVERY)
    # the state at the first timed step, for the CPU baseline's window
    state0 = (g.read("v"), g.read("w"), g.step_index)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = g.step(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    dom_ms, dom_n = g.kernel_time(dom)
    g.kernel_timing(False)

    value = inst.nt * a.steps / elapsed
    avg_it = dom_ms / max(dom_n, 1)
    achieved = ALGO_BYTES[dom_bytes] * inst.nt / (avg_it * 1e-3) / 1e9
    tfile = a.traffic_file or os.path.join(
        ROOT, "profiles", f"traffic_{dom_name.split('<')[0]}_aniso_be_{a.n}.txt")
    traffic = read_traffic(tfile, dom_name)
    out = {
        "metric": "voxel-steps/s",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"aniso_be_{a.n}: monodomain FP32, {a.n}^3 ellipsoidal shell "
                               f"({inst.nt} tissue voxels), 19-point anisotropic stencil, "
                               f"implicit Euler by Jacobi-PCG rtol {a.rtol:g}, dt {inst.dt} ms",
                   "n_tissue": inst.nt, "grid": list(inst.n), "dt_ms": inst.dt},
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algo_bytes_per_launch": ALGO_BYTES[dom_bytes] * inst.nt,
                     "avg_launch_us": 1e3 * avg_it, "launches": dom_n,
                     "timed_steps": f"every {TIMING_EVERY}th step of the timed region"},
        "cg": {"iters_total": info["cg_iters"], "iters_per_step": info["cg_iters"] / a.steps,
               "iters_max": info["cg_max"],
               "breakdown_steps": n_diag,
               "kernels": {STEP_KERNELS[k][0]: {
                   "avg_us": 1e3 * times[k][0] / max(times[k][1], 1),
                   "launches": times[k][1], "ms_per_step": times[k][0] / n_diag,
                   "achieved_gbs": ALGO_BYTES[STEP_KERNELS[k][1]] * inst.nt
                   / max(1e-3 * times[k][0] / max(times[k][1], 1), 1e-12) / 1e9}
                   for k in STEP_KERNELS},
               "tail_avg_us": 1e3 * times["cg_tail"][0] / max(times["cg_tail"][1], 1),
               "tail_launches": times["cg_tail"][1],
               "kernel_ms_per_step": sum(t[0] for t in times.values()) / n_diag},
        "stream_ceiling": {"copy_gbs": copy_gbs, "read_gbs": read_gbs,
                           "how": "ep_stream_bandwidth: hand-written HIP copy and read-only "
                                  "kernels over 1 GiB buffers, 16-B accesses, best of 5",
                           "frac_of_copy": achieved / copy_gbs},
    }
    if not a.no_err:
        out["err_vs_oracle"] = oracle_step_error(inst, g)
    g.close()
    if a.serving:
        out["serving"] = bench_serving(a.serving, a.serving_k)
    if not a.no_plain:
        out["plain_box_32_fp64"] = bench_plain_fp64()
    if a.bidomain:
        out["bidomain"] = bench_bidomain(a.bidomain)
    if a.adjoint:
        out["adjoint"] = bench_adjoint(a.adjoint)
    if a.jacobi:
        out["jacobi"] = bench_jacobi(a.jacobi)
    if not a.no_cuboid:
        out["cuboid"] = bench_cuboid()
    if a.explicit27:
        out["explicit27"] = bench_explicit27(a.explicit27)
    if a.bath:
        out["bath"] = bench_bath(a.bath)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, state0, info["cg_iters"] / a.steps,
                                           a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
