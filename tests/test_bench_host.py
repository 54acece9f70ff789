"""Host logic of bench.py that runs without a GPU: the refusal of several
GPUs and the rule that a committed HBM-traffic counter summary is used only
for the kernel and the kernel source it was taken on."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_several_gpus_refused_with_message(n):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and f"--gpus {n}" in p.stderr
    assert p.stdout == ""


def _source_sha():
    src = os.path.join(ROOT, "paper_2302_12519_amd", "csrc", "ep_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _summary(tmp_path, sha, kernel="k_be_init<float>", traffic="557791271"):
    p = tmp_path / "traffic.txt"
    p.write_text("command: (not run)\n"
                 f"kernel: {kernel}\n"
                 f"traffic_bytes_per_launch: {traffic}\n"
                 f"kernel_source_sha: {sha}\n")
    return str(p)


def test_traffic_used_for_matching_kernel_and_source(tmp_path):
    assert bench.read_traffic(_summary(tmp_path, _source_sha()),
                              "k_be_init<float>") == 557791271.0


def test_traffic_dropped_for_other_source(tmp_path):
    other = "0" * 16 if _source_sha() != "0" * 16 else "1" * 16
    assert bench.read_traffic(_summary(tmp_path, other), "k_be_init<float>") is None


def test_traffic_dropped_for_other_kernel(tmp_path):
    assert bench.read_traffic(_summary(tmp_path, _source_sha(), kernel="k_pcg_step<float>"),
                              "k_be_init<float>") is None


def test_traffic_absent_or_malformed(tmp_path):
    assert bench.read_traffic(str(tmp_path / "missing.txt"), "k_be_init<float>") is None
    assert bench.read_traffic(_summary(tmp_path, _source_sha(), traffic="n/a"),
                              "k_be_init<float>") is None


@pytest.mark.parametrize("name,kernel", [
    ("traffic_k_pcg_step_aniso_be_256.txt", "k_pcg_step<float> (iteration)"),
    ("traffic_k_be_init_aniso_be_256.txt", "k_be_init<float>")])
def test_committed_summary_names_its_kernel_and_source(name, kernel):
    """The counter summaries the bench can pick for C2's dominant kernel (the
    file name is the kernel's, the key line the role bench.py names)."""
    path = os.path.join(ROOT, "profiles", name)
    keys = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            keys[k.strip()] = v.strip()
    assert keys["kernel"] == kernel
    assert len(keys["kernel_source_sha"]) == 16
    assert float(keys["traffic_bytes_per_launch"]) > float(keys["algorithmic_bytes_per_launch"]) > 0


def test_cpu_baseline_protocol():
    """The baseline starts from the given state (the GPU's at its first timed
    step), solves to the same rtol, reports the median of 3 runs, a
    one-thread figure, the thread count and the CPU model, and leaves the
    oracle's thread count as it was."""
    import ep_inputs as E
    import oracle
    inst = E.aniso_be(16, steps=2)
    inst.pcg_rtol = 1e-7
    v, w = E.random_state(inst, 3)
    threads = oracle.threads()
    out = bench.cpu_baseline(inst, (v, w, 25), 2.5, 0.0)
    assert oracle.threads() == threads
    assert out["kind"] == "oracle" and out["unit"] == "voxel-steps/s"
    assert out["cores"] == threads >= 1
    assert out["value"] > 0 and out["value_1_thread"] > 0
    assert len(out["runs_s"]) == 3 and out["steps_per_run"] == 1
    assert "step 25" in out["sample"] and "rtol 1e-07" in out["sample"]
    assert out["oracle_cg_iters_per_step"] > 0 and out["gpu_cg_iters_per_step"] == 2.5
    assert isinstance(out["cpu_model"], str)
