"""The committed rocprofv3 summaries under profiles/: each names its kernel and
workload in its file name, gives the commands that made it, and ends with a
machine-readable block (operating point, sha256 of the kernel's sources,
HBM bytes per launch) that bench.py reads to fill the roofline's `traffic`.
A summary whose sources have changed since it was taken is reported as stale
(skipped), since bench.py then reports no traffic for it."""
import glob
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def _block(text):
    out = {}
    for key in ("operating_point", "kernel_source_sha256", "traffic_bytes_per_launch"):
        m = re.search(rf"^{key}:\s*(.+)$", text, flags=re.M)
        out[key] = m.group(1).strip() if m else None
    return out


def test_there_are_summaries():
    assert SUMMARIES, "no profiles/*.md"


@pytest.mark.parametrize("path", SUMMARIES, ids=[os.path.basename(p) for p in SUMMARIES])
def test_summary_block(path):
    name = os.path.basename(path)
    kernel = next((k for k in bench.KERNEL_SOURCES if name.startswith(k + "_")), None)
    assert kernel, f"{name}: not named <kernel>_<workload>.md for a scan kernel"
    text = open(path).read()
    assert "rocprofv3 --kernel-trace --stats" in text and "rocprofv3 --pmc FETCH_SIZE" in text \
        and "rocprofv3 --pmc WRITE_SIZE" in text, f"{name}: the commands that made it are missing"
    b = _block(text)
    assert all(b.values()), f"{name}: incomplete machine-readable block {b}"
    assert re.fullmatch(r"[0-9a-f]{64}", b["kernel_source_sha256"])
    traffic = float(b["traffic_bytes_per_launch"])
    assert traffic > 0
    if b["kernel_source_sha256"] != bench.source_sha(bench.KERNEL_SOURCES[kernel]):
        pytest.skip(f"{name} is stale: its kernel's sources changed since it was taken")
    # the figure bench.py reports for this operating point is the summary's
    assert bench.pmc_traffic(kernel, b["operating_point"]) == traffic
    assert bench.pmc_traffic(kernel, b["operating_point"] + " other") is None
