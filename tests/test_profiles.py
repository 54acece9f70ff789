"""The committed profiler summaries: short text, each naming the rocprofv3
command that made it (which runs committed files only) and a kernel that
the HIP sources define."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2302_12519_amd", "csrc")

FILES = sorted(f for f in os.listdir(PROF) if not f.startswith("."))


def _kernels():
    names = set()
    for f in os.listdir(CSRC):
        if f.endswith(".hip"):
            names |= set(re.findall(r"void\s+(k_\w+)\s*\(", open(os.path.join(CSRC, f)).read()))
    return names


def test_there_are_summaries():
    assert "k_pcg_step_aniso_be_256.txt" in FILES
    assert "traffic_k_pcg_step_aniso_be_256.txt" in FILES
    assert "traffic_k_be_init_aniso_be_256.txt" in FILES


@pytest.mark.parametrize("name", FILES)
def test_summary_is_short_text_with_its_command(name):
    path = os.path.join(PROF, name)
    assert name.endswith((".txt", ".md"))
    assert os.path.getsize(path) < 16 * 1024
    text = open(path, encoding="utf-8").read()
    assert "rocprofv3" in text
    assert "_work" not in text and "gpurun" not in text


@pytest.mark.parametrize("name", FILES)
def test_summary_names_a_defined_kernel(name):
    m = re.search(r"(k_[a-z0-9]+(?:_[a-z0-9]+)*?)_(?:aniso|bidomain|adjoint|serving|plain|cuboid)",
                  name)
    assert m, name
    assert m.group(1) in _kernels(), (name, m.group(1))
