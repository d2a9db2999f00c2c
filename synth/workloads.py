"""The synthetic workloads the search path is measured and checked on.

Each stands in for one of the paper's public datasets (Section 4.1), which are
not available here: the recipes reproduce their shapes, sizes and value
distributions, never their records.

  mixture128   - 100k x 128 Gaussian mixture, a small SIFT1M-like case
  sift10m      - 10M x 128 integer-valued skewed features (SIFT descriptors
                 are integers in 0..255), the SIFT100M/SIFT1B stand-in at the
                 size one GPU holds with raw vectors resident
  embed960     - 1M x 960 non-negative correlated features, the
                 high-dimensional text-embedding stand-in (Cohere 10M, 768-D)
  unit96_400m  - 400M x 96 unit vectors, billion-scale footprint pressure
  serving      - the sift10m index under Poisson arrivals of mixed nprobe / k
"""
from __future__ import annotations

from dataclasses import dataclass, replace


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str              # recipe: mixture | gamma_int | blocks_abs | unit_mixture
    n: int                 # database rows
    d: int                 # dimension
    nlist: int             # IVF lists
    nprobe: tuple          # probe counts run on this workload
    nq: int                # queries per batch
    bq: int = 4            # query quantisation bits
    k: int = 10
    rerank_n: int = 100
    seed: int = 0
    centres: int = 0       # mixture components (mixture kinds)
    sigma: float = 0.0     # mixture noise scale

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS = {
    "mixture128": Workload("mixture128", "mixture", n=100_000, d=128, nlist=256,
                           nprobe=(16,), nq=100, k=10, rerank_n=100,
                           centres=256, sigma=0.3),
    "sift10m": Workload("sift10m", "gamma_int", n=10_000_000, d=128, nlist=4096,
                        nprobe=(32, 64, 128), nq=1024, k=10, rerank_n=100),
    "embed960": Workload("embed960", "blocks_abs", n=1_000_000, d=960, nlist=1024,
                         nprobe=(64,), nq=1000, k=10, rerank_n=200),
    "unit96_400m": Workload("unit96_400m", "unit_mixture", n=400_000_000, d=96,
                            nlist=65_536, nprobe=(128,), nq=10_000, k=10,
                            rerank_n=100, centres=65_536, sigma=0.05),
}
# The serving workload reuses the sift10m index and draws per-request
# nprobe from {8, 16, ..., 256}, k from {10, 100} and rerank_n = 10 k.
WORKLOADS["serving"] = WORKLOADS["sift10m"].with_(name="serving")


def get(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return w.with_(**overrides) if overrides else w
