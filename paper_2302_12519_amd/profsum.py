"""Summaries of rocprofv3 CSV output for the library's kernels (measurement
tooling; no part of the simulation path).

- ``trace``: per-kernel launch counts and mean / min / max durations from a
  ``--kernel-trace`` CSV.
- ``counters``: per-kernel mean of one counter per dispatch from a ``--pmc``
  run's counter-collection CSV, optionally scaled by a calibration factor:
  the factor that makes the counter read `calib_bytes` for the largest
  ``__amd_rocclr_copyBuffer`` dispatch of the same run (a plain copy of known
  size, e.g. bench.py --copy-calibration: 1 GiB read and 1 GiB written).

The launches of the implicit-step CG kernel ``k_pcg_step`` do different
work by position, so they are split into roles by dispatch order: in each
run of consecutive ``k_pcg_step`` dispatches the first is the set-up launch
(p0 = z0, q0 = K p0), the last applies the final x update, and those in
between are full iterations.

Usage:
  python -m paper_2302_12519_amd.profsum trace    KERNEL_TRACE.csv [--skip-steps S]
  python -m paper_2302_12519_amd.profsum counters COUNTER_COLLECTION.csv NAME [--calib-bytes B]
"""
from __future__ import annotations

import argparse
import csv
import sys
from collections import OrderedDict

PCG = "k_pcg_step"
ROLES = ("launch 0", "iteration", "last x update")


def demangled_tail(name: str) -> str:
    """Last identifier of a nested mangled name the profiler left mangled
    ('_ZN2ep12_GLOBAL__N_113k_coarse_gemvEi...' -> 'k_coarse_gemv')."""
    i, last = 3, name
    while i < len(name) and name[i].isdigit():
        j = i
        while name[j].isdigit():
            j += 1
        n = int(name[i:j])
        last = name[j:j + n]
        i = j + n
    return last


def short_name(name: str) -> str:
    """'void ep::(anonymous namespace)::k_x<float, true>(int, ...)' -> 'k_x<float, true>'."""
    if name.startswith("_ZN"):
        return demangled_tail(name)
    s = name.strip().replace("(anonymous namespace)::", "")
    if s.startswith("void "):
        s = s[5:]
    depth, cut = 0, len(s)
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    s = s[:cut]
    # drop namespace qualifiers outside template arguments
    depth, last = 0, 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == ":" and depth == 0 and i + 1 < len(s) and s[i + 1] == ":":
            last = i + 2
    return s[last:]


def with_roles(rows):
    """rows: (dispatch_id, short_name, value) sorted by dispatch id.  Returns
    (label, value) with k_pcg_step dispatches labelled by role."""
    out = []
    i = 0
    while i < len(rows):
        if rows[i][1].startswith(PCG):
            j = i
            while j < len(rows) and rows[j][1] == rows[i][1]:
                j += 1
            n = j - i
            for k in range(i, j):
                pos = k - i
                role = ROLES[0] if pos == 0 else (ROLES[2] if pos == n - 1 else ROLES[1])
                out.append((f"{rows[k][1]} ({role})", rows[k][2]))
            i = j
        else:
            out.append((rows[i][1], rows[i][2]))
            i += 1
    return out


def group(labelled):
    g = OrderedDict()
    for lab, v in labelled:
        g.setdefault(lab, []).append(v)
    return g


def from_step(rows, skip):
    """Drop the dispatches before the (skip + 1)-th k_be_init (the first
    `skip` implicit steps of the run)."""
    if skip <= 0:
        return rows
    seen = 0
    for i, r in enumerate(rows):
        if r[1].startswith("k_be_init"):
            if seen == skip:
                return rows[i:]
            seen += 1
    return []


def trace(path, skip_steps=0):
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
            rows.append((int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]), us))
    rows.sort()
    g = group(with_roles(from_step(rows, skip_steps)))
    print(f"{'kernel':58s} {'calls':>6s} {'avg us':>9s} {'min us':>9s} {'max us':>9s} "
          f"{'total ms':>9s}")
    for lab, v in sorted(g.items(), key=lambda kv: -sum(kv[1])):
        print(f"{lab[:58]:58s} {len(v):6d} {sum(v) / len(v):9.2f} {min(v):9.2f} {max(v):9.2f} "
              f"{sum(v) * 1e-3:9.3f}")


def counters(path, name, calib_bytes=None):
    rows, dur = [], {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != name:
                continue
            rows.append((int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]),
                         float(r["Counter_Value"])))
            if r.get("Start_Timestamp") and r.get("End_Timestamp"):
                dur[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) -
                                              int(r["Start_Timestamp"])) * 1e-3
    rows.sort()
    factor = 1.0
    if calib_bytes:
        cal = [v for _, k, v in rows if k == "__amd_rocclr_copyBuffer"]
        if not cal:
            sys.exit("no __amd_rocclr_copyBuffer dispatch to calibrate with")
        factor = calib_bytes / 1024.0 / max(cal)
        print(f"calibration: largest copy reads {max(cal):.1f} KiB of {name} for "
              f"{calib_bytes / 1024.0:.0f} KiB -> factor {factor:.4f}")
    g = group(with_roles(rows))
    if name in ("FETCH_SIZE", "WRITE_SIZE"):
        # byte counters, in KiB per dispatch; the mean duration of the same
        # dispatches in this (counter-collecting) run gives the rate
        us = group(with_roles([(d, k, dur.get(d, 0.0)) for d, k, _ in rows]))
        print(f"{'kernel':58s} {'calls':>6s} {name + ' KiB':>16s} {'x factor, MB':>13s} "
              f"{'avg us':>9s} {'GB/s':>7s}")
        for lab, v in g.items():
            kib = sum(v) / len(v)
            mb = kib * 1024 * factor / 1e6
            t = sum(us[lab]) / len(us[lab])
            rate = f"{mb / t * 1e3:7.0f}" if t > 0 else "      -"
            print(f"{lab[:58]:58s} {len(v):6d} {kib:16.1f} {mb:13.2f} {t:9.2f} {rate}")
    else:
        print(f"{'kernel':58s} {'calls':>6s} {name + ' per dispatch':>26s}")
        for lab, v in g.items():
            print(f"{lab[:58]:58s} {len(v):6d} {sum(v) / len(v):26.1f}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--skip-steps", type=int, default=0,
                   help="implicit-step runs: leave out the first S steps (k_be_init launches)")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("name")
    c.add_argument("--calib-bytes", type=float, default=None)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        trace(a.csv, a.skip_steps)
    else:
        counters(a.csv, a.name, a.calib_bytes)


if __name__ == "__main__":
    main()
