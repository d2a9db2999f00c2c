"""GPU tests of the query rotation P^T q in FP32 and with BF16 inputs.

The kernels are pinned to the exact product of their (possibly rounded)
inputs: with FP32 inputs the rotated query must be within the FP32 summation
bound K u sum|q_k P_kc| of the FP64 product; with BF16 inputs, within the same
bound of the FP64 product of the bfloat16-rounded inputs (rounded by torch,
nearest-even).

The BF16 option changes the estimates, so it is not a parity case: the second
test reports how far the end-to-end d_hat^2 of each rotation lands from the
FP64 oracle's (oracle probes injected, everything after them computed on the
GPU), scaled as in P5, and the recall of both, on a 960-dimensional workload of
the heavy-tailed block-correlated kind.
"""
import json
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import est_scale, lib_index, make_case

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).to(
        torch.float32).numpy()


@pytest.mark.parametrize("d,nq", [(96, 70), (960, 33), (13, 5)])
def test_rotation_kernels_exact_product(d, nq):
    _say(f"[rotation] kernel check d={d} nq={nq}")
    X, Q, idx = make_case(max(1200, 40 * 8), d, 8, nq, seed=61, kind="blocks_abs" if d == 960 else "mixture")
    lib = lib_index(X, idx)
    P = np.asarray(idx.P, np.float32)
    for mode, (qa, pa) in ((0, (Q, P)), (1, (_bf16(Q), _bf16(P)))):
        lib.set_option("rotation", mode)
        try:
            got = lib.search_debug(Q, 2, 1, 1, want={"qrot"})["qrot"].astype(np.float64)
        finally:
            lib.set_option("rotation", 0)
        ref = qa.astype(np.float64) @ pa.astype(np.float64)
        bound = (d + 2) * U32 * (np.abs(qa.astype(np.float64)) @ np.abs(pa.astype(np.float64))) + 1e-30
        assert np.all(np.abs(got - ref) <= bound), (mode, float(np.max(np.abs(got - ref) / bound)))
        if mode == 1:  # the rounding is real: BF16 differs from the FP32 product
            assert np.max(np.abs(ref - Q.astype(np.float64) @ P.astype(np.float64))) > 0


def test_rotation_precision_error_table():
    """P8 report: d_hat^2 error of FP32 and BF16 rotation against the FP64
    oracle, and recall@10 of each (not a pass/fail parity; loose sanity bounds
    only)."""
    n, d, nlist, nq, nprobe, k, R = 12_000, 960, 24, 48, 4, 10, 200
    _say(f"[rotation] error table n={n} d={d} nlist={nlist} nq={nq} nprobe={nprobe} R={R}")
    X, Q, idx = make_case(n, d, nlist, nq, seed=62, kind="blocks_abs")
    lib = lib_index(X, idx)
    _, _, st = O.search(idx, X, Q, nprobe, k, R, stages=True)
    gt, _ = O.brute_force_knn(X, Q, k)
    probes = np.array(st["probes"], np.int32)
    table = {}
    for name, mode in (("fp32", 0), ("bf16", 1)):
        lib.set_option("rotation", mode)
        try:
            out = lib.search_debug(Q, nprobe, k, R, inject_probes=probes, want={"est", "ids"})
        finally:
            lib.set_option("rotation", 0)
        errs = []
        for qi in range(nq):
            for p, pl in enumerate(st["per_list"][qi]):
                m = len(pl["ids"])
                if not m:
                    continue
                S = est_scale(st["rnorm2"][qi][p], st["vl"][qi][p], st["delta"][qi][p],
                              st["sumqu"][qi][p], pl["ip"], pl["pop"], idx.n_x[pl["ids"]],
                              idx.alpha[pl["ids"]], d)
                errs.append(np.abs(out["est"][qi, p, :m].astype(np.float64) - pl["est"]) / S)
        e = np.concatenate(errs)
        rec = float(np.mean([len(set(a.tolist()) & set(b.tolist())) / k for a, b in zip(out["ids"], gt)]))
        table[name] = {"max": float(e.max()), "p99": float(np.percentile(e, 99)),
                       "mean": float(e.mean()), "recall_at_10": rec, "estimates": int(e.size)}
    table["recall_delta_bf16_minus_fp32"] = table["bf16"]["recall_at_10"] - table["fp32"]["recall_at_10"]
    _say("[rotation] P8 " + json.dumps(table))
    assert table["fp32"]["p99"] <= 1e-5
    assert table["bf16"]["mean"] <= 1e-2 and table["bf16"]["max"] < 0.1
    assert table["recall_delta_bf16_minus_fp32"] >= -0.05
