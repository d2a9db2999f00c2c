"""Host-side check of the fp4 x fp8 list-major scan's operand layouts (no GPU).

The quantiser writes each pair's fp8 bytes of 2 qu at `group_qu8_offset`
(csrc/kernels.hpp); the scan expands code word g of a 128-dimension step into
lane group g's fp4 A operand with bit 4 i + q at nibble i of dword q
(element k = 32 g + 8 q + i). The matrix core's own element order, found on
the device with a probe and documented beside `group_qu8_offset`, reads
B element k of lane group g from byte k - 16 g (k in [16 g, 16 g + 16)) or
byte 16 + k - 64 - 16 g (k in [64 + 16 g, 80 + 16 g)) of that group's 32
bytes. Here the product's offset function is compiled for the host and the
sum over k of A_k B_k is checked against the plain sum over dimensions of
bit_d 2 qu_d on random codes and queries.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

SHIM = r"""
#include <cstdio>
#include "kernels.hpp"
int main() {
  for (int l = 0; l < 16; ++l)
    for (int j = 0; j < 4; ++j) std::printf("%d\n", rbq::group_qu8_offset(l, j));
  return 0;
}
"""


@pytest.fixture(scope="module")
def offsets():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "shim.cpp"), os.path.join(d, "shim")
        open(src, "w").write(SHIM)
        r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I",
                            os.path.join(ROOT, "paper_2605_16007_amd", "csrc"), src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return np.array(out, np.int64).reshape(16, 4)


def test_offsets_cover_the_row_once(offsets):
    pos = np.concatenate([offsets.ravel(), offsets.ravel() + 1])
    assert sorted(pos.tolist()) == list(range(128))
    # the j = 1, 2, 3 offsets are those of j = 0 plus 8, 32, 40 (the quantiser
    # stores through one base address)
    np.testing.assert_array_equal(offsets - offsets[:, :1], np.tile([0, 8, 32, 40], (16, 1)))


def _b_element(g, e):
    """Matrix-core element k read from byte e of lane group g's 32 B bytes."""
    return 16 * g + e if e < 16 else 64 + 16 * g + (e - 16)


@pytest.mark.parametrize("seed", range(4))
def test_operands_give_the_inner_product(offsets, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, 128)
    qu = rng.integers(0, 16, 128)
    # the quantiser's lane l holds dimensions 8 l .. 8 l + 7 of the step
    row = np.full(128, -1)
    for l in range(16):
        for j in range(4):
            o = offsets[l, j]
            row[o], row[o + 1] = 2 * qu[8 * l + j], 2 * qu[8 * l + j + 4]
    assert (row >= 0).all()
    # the scan's A: lane group g expands code word g (dimensions 32 g ..)
    A = np.zeros(128, np.int64)
    for g in range(4):
        w = int(sum(int(bits[32 * g + b]) << b for b in range(32)))
        dw = [(w << 1) & 0x22222222, w & 0x22222222, (w >> 1) & 0x22222222, (w >> 2) & 0x22222222]
        for q in range(4):
            for i in range(8):
                nib = (dw[q] >> (4 * i)) & 0xF
                assert nib in (0, 2)  # fp4 E2M1 0 or 1.0
                A[32 * g + 8 * q + i] = nib // 2
    B = np.zeros(128, np.int64)
    for g in range(4):
        for e in range(32):
            B[_b_element(g, e)] = row[32 * g + e]
    assert int((A * B).sum()) == int((bits * 2 * qu).sum())
