"""The committed rocprofv3 summaries stay tied to the code they describe.

* A counter summary that the benchmark reads its `traffic` figure from
  carries the hash of the kernel sources it was taken on; the hash must be
  that of the current sources, or the benchmark line would silently report
  no traffic.
* Every profiler command a summary gives runs the committed benchmark with
  options it accepts, so that the figures can be taken again.
"""
import glob
import os
import shlex

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))

# counter summaries the benchmark reads, with the sources their hash covers
TRAFFIC = {
    "stencil_banded_hbm_traffic.txt": bench.BANDED_SOURCES,
    "stencil_hbm_traffic.txt": bench.REAL_SWEEP_SOURCES,
    "complex_stencil_hbm_traffic.txt": bench.COMPLEX_SWEEP_SOURCES,
}


def _fields(path):
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


@pytest.mark.parametrize("name", sorted(TRAFFIC))
def test_traffic_summary_matches_current_sources(name):
    kv = _fields(os.path.join(ROOT, "profiles", name))
    assert kv.get("kernel_source_sha256_16") == bench._kernel_source_sha(TRAFFIC[name]), name
    key = "hbm_bytes_per_sweep" if name.startswith("stencil_banded") else "hbm_bytes_per_launch"
    assert float(kv[key]) > 0


def _bench_commands(path):
    """The bench.py arguments of every rocprofv3 command in a summary (comment
    markers dropped, continuation lines joined)."""
    with open(path) as fh:
        text = fh.read()
    lines = [ln.lstrip("#").strip() for ln in text.replace("\\\n", " ").splitlines()]
    out = []
    for line in lines:
        if line.startswith("rocprofv3 ") and "bench.py" in line:
            out.append(shlex.split(line.split("bench.py", 1)[1]))
    return out


@pytest.mark.parametrize("path", PROFILES, ids=[os.path.basename(p) for p in PROFILES])
def test_profile_commands_parse(path):
    cmds = _bench_commands(path)
    assert cmds, f"{os.path.basename(path)} gives no rocprofv3 command"
    for argv in cmds:
        try:
            bench.arg_parser().parse_args(argv)
        except SystemExit:
            pytest.fail(f"{os.path.basename(path)}: bench.py does not accept {argv}")
