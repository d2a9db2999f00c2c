"""Host memory for borrowed raw vectors: ``huge_page_rows`` returns a
2 MiB-aligned private anonymous mapping that the kernel backs with transparent
huge pages where they are enabled for advised regions (the host re-rank's
random row gathers depend on it)."""
import re

import numpy as np
import pytest

from paper_2605_16007_amd import huge_page_rows


def _thp_mode():
    try:
        text = open("/sys/kernel/mm/transparent_hugepage/enabled").read()
    except OSError:
        return None
    m = re.search(r"\[(\w+)\]", text)
    return m.group(1) if m else None


def _anon_huge_kb():
    text = open("/proc/self/smaps_rollup").read()
    return int(re.search(r"AnonHugePages:\s+(\d+)", text).group(1))


def test_rows_are_aligned_writable_and_shaped():
    a = huge_page_rows(1000, 96)
    assert a.shape == (1000, 96) and a.dtype == np.float32
    assert a.ctypes.data % (2 << 20) == 0
    a[:] = 3.0
    assert float(a.sum()) == 3.0 * 96_000


def test_rows_get_transparent_huge_pages():
    if _thp_mode() not in ("always", "madvise"):
        pytest.skip("transparent huge pages are off on this host")
    before = _anon_huge_kb()
    a = huge_page_rows(1 << 18, 256)  # 256 MiB
    a[:] = 1.0
    after = _anon_huge_kb()
    # the mapping is private anonymous memory (a shared one would be shmem,
    # which advised huge pages do not cover)
    assert after - before >= 128 * 1024, (before, after)
    del a
