"""IVF-RaBitQ in plain FP64 NumPy: the reference the GPU library is checked against.

TEST INFRASTRUCTURE ONLY (see the package docstring). Notation follows the
paper: ``c`` an IVF centroid, ``P`` the random orthogonal D x D matrix,
``b`` the sign code in {-1,+1}^D and ``b01 = (b+1)/2`` its 0/1 form,
``n_x = ||x - c||`` the residual norm and ``alpha_x`` the database-side
normalisation constant.

Readings where the paper is silent (each is listed in the design doc):
  * the query residual is scalar-quantised to ``bq`` bits, uniform min-max per
    (query, probed list), deterministic round-half-up (the transformed query
    "can be scalar-quantized", Sec. 2.2.2; the paper's CPU 1-bit+SQ baseline
    uses 4-bit query SQ, Sec. 4.1);
  * the unnormalised residual r = P^T q - P^T c is quantised: the affine
    quantiser is scale invariant, and ||q-c|| * s_hat = E / (sqrt(D) alpha_x);
  * sign(0) = +1; bits are packed LSB-first, dimension d in byte d>>3, bit d&7;
  * n_x = 0 gives alpha_x = 1 and an all-ones code;
  * ties are broken lexicographically by (value, id) everywhere;
  * distances returned are squared L2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "sqdist", "assign", "kmeanspp_init", "lloyd_update", "kmeans", "random_orthogonal",
    "encode", "pack_bits", "unpack_bits", "probe", "rotate", "quantize",
    "ip_dense", "ip_bitplanes", "bitplanes", "est_terms", "estimate",
    "topk_lex", "rerank", "Index", "build", "search", "brute_force_knn",
    "s_hat_unquantized", "est_terms_unquantized", "ivf_flat_search",
]


# --------------------------------------------------------------------------
# IVF construction (Sec. 2.1.2 "Index Construction"; Sec. 3.1.1 Phases 1-2)
# --------------------------------------------------------------------------

def sqdist(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Squared L2 distances ||x_i - c_j||^2 in FP64 (rows of X vs rows of C)."""
    X = np.asarray(X, np.float64)
    C = np.asarray(C, np.float64)
    xx = np.einsum("ij,ij->i", X, X)[:, None]
    cc = np.einsum("ij,ij->i", C, C)[None, :]
    return xx - 2.0 * (X @ C.T) + cc


def assign(X: np.ndarray, C: np.ndarray, chunk: int = 65536):
    """Nearest centroid of every row, ties to the lowest centroid id.

    Returns (assignment int64, squared distance to it, FP64).
    """
    n = len(X)
    a = np.empty(n, np.int64)
    dmin = np.empty(n, np.float64)
    for s in range(0, n, chunk):
        d = sqdist(X[s:s + chunk], C)
        j = np.argmin(d, axis=1)        # first minimum = lowest id on ties
        a[s:s + chunk] = j
        dmin[s:s + chunk] = d[np.arange(len(j)), j]
    return a, dmin


def kmeanspp_init(T: np.ndarray, nlist: int, rng: np.random.Generator) -> np.ndarray:
    """k-means++ seeding: the first centre uniform, then D(x)^2 sampling."""
    T = np.asarray(T, np.float64)
    n = len(T)
    C = np.empty((nlist, T.shape[1]), np.float64)
    C[0] = T[rng.integers(n)]
    d2 = np.sum((T - C[0]) ** 2, axis=1)
    for j in range(1, nlist):
        tot = d2.sum()
        if tot > 0:
            idx = rng.choice(n, p=d2 / tot)
        else:                            # fewer distinct points than centres
            idx = rng.integers(n)
        C[j] = T[idx]
        d2 = np.minimum(d2, np.sum((T - C[j]) ** 2, axis=1))
    return C


def lloyd_update(T, a, C_prev, dmin):
    """Lloyd update: each centroid becomes the mean of its points.

    An empty cluster is re-seeded to the training point farthest from its
    current centroid (distinct points, farthest first).
    """
    nlist, d = C_prev.shape
    sums = np.zeros((nlist, d), np.float64)
    np.add.at(sums, a, T)
    cnt = np.bincount(a, minlength=nlist)
    C = C_prev.copy()
    nz = cnt > 0
    C[nz] = sums[nz] / cnt[nz, None]
    empty = np.flatnonzero(~nz)
    if len(empty):
        far = np.argsort(-dmin, kind="stable")[:len(empty)]
        C[empty] = T[far]
    return C


def kmeans(X: np.ndarray, nlist: int, rng: np.random.Generator, iters: int = 25,
           restarts: int = 3, train_n: int | None = None, trace: list | None = None,
           seed_rows: int | None = None, init: str = "kmeans++"):
    """IVF centroids by k-means on a training subset (Sec. 2.1.2, Sec. 3.1.1).

    The paper fixes neither the initialisation, the subset, the iteration limit
    nor empty-cluster handling; this oracle uses: ``train_n = min(N, 256 nlist)``
    rows sampled without replacement, k-means++ seeding, Lloyd iterations until
    no assignment changes or ``iters`` is reached, ``restarts`` runs keeping the
    lowest objective. Returns FP64 centroids. ``trace`` (if a list) receives the
    objective after every assignment step of every restart.

    ``seed_rows`` (the reading the GPU library takes to keep seeding cheap at
    large nlist): k-means++ draws its centres from the evenly strided subset of
    at most ``seed_rows`` training rows (row t * T // S of the T training rows,
    t < S = min(T, seed_rows)) instead of from all of them; the Lloyd steps
    still use every training row. None: all training rows.

    ``init="random"``: the initial centroids are nlist distinct training rows
    drawn uniformly (the random initial centroids of Sec. 3.1.1 Phase 1)
    instead of k-means++ seeds.
    """
    X = np.asarray(X)
    n = len(X)
    tn = min(n, 256 * nlist if train_n is None else train_n)
    if tn < n:
        T = np.asarray(X[np.sort(rng.choice(n, tn, replace=False))], np.float64)
    else:
        T = np.asarray(X, np.float64)
    S_rows = T
    if seed_rows is not None and seed_rows < len(T):
        S_rows = T[(np.arange(seed_rows, dtype=np.int64) * len(T)) // seed_rows]
    best_obj, best_C = None, None
    for _ in range(restarts):
        if init == "random":
            C = T[rng.choice(len(T), nlist, replace=False)].copy()
        else:
            C = kmeanspp_init(S_rows, nlist, rng)
        prev = None
        run = []
        for _it in range(iters):
            a, dmin = assign(T, C)
            run.append(float(dmin.sum()))
            if prev is not None and np.array_equal(a, prev):
                break
            C = lloyd_update(T, a, C, dmin)
            prev = a
        _, dmin = assign(T, C)
        obj = float(dmin.sum())
        run.append(obj)
        if trace is not None:
            trace.append(run)
        if best_obj is None or obj < best_obj:
            best_obj, best_C = obj, C
    return best_C


def random_orthogonal(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random orthogonal P (Sec. 2.2.1): QR of a Gaussian matrix, with the
    signs of R's diagonal folded into Q. FP64."""
    G = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


# --------------------------------------------------------------------------
# RaBitQ encoding (Sec. 2.2.1: Eqs. normalized-residual, quantize, rabitq-alpha)
# --------------------------------------------------------------------------

def pack_bits(bits01: np.ndarray) -> np.ndarray:
    """Pack 0/1 rows LSB-first: dimension d goes to byte d>>3, bit d&7."""
    return np.packbits(np.asarray(bits01, np.uint8), axis=-1, bitorder="little")


def unpack_bits(codes: np.ndarray, d: int) -> np.ndarray:
    return np.unpackbits(codes, axis=-1, count=d, bitorder="little")


def encode(X: np.ndarray, C: np.ndarray, a: np.ndarray, P: np.ndarray):
    """1-bit codes and stored factors of every row of X in its list a[i].

    z = P^T (x - c) (the sign of z equals the sign of P^T u_x since u_x is a
    positive multiple of x - c); b01_d = [z_d >= 0]; n_x = ||x - c||;
    alpha_x = ||P^T u_x||_1 / sqrt(D) = ||z||_1 / (sqrt(D) ||z||_2).
    Returns (packed codes uint8 [N, ceil(D/8)], n_x float32, alpha_x float32).
    """
    X = np.asarray(X, np.float64)
    C = np.asarray(C, np.float64)
    P = np.asarray(P, np.float64)
    d = X.shape[1]
    r = X - C[a]
    z = r @ P                      # row form of P^T r
    bits = (z >= 0.0).astype(np.uint8)
    n_x = np.sqrt(np.sum(r * r, axis=1))
    z2 = np.sqrt(np.sum(z * z, axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        alpha = np.sum(np.abs(z), axis=1) / (np.sqrt(d) * z2)
    zero = n_x == 0.0
    alpha[zero] = 1.0
    bits[zero] = 1
    return pack_bits(bits), n_x.astype(np.float32), alpha.astype(np.float32)


# --------------------------------------------------------------------------
# Search (Sec. 2.1.2 "Query Processing"; Sec. 2.2.2; Sec. 3.1.2 Phases 1-5)
# --------------------------------------------------------------------------

def probe(q: np.ndarray, C: np.ndarray, nprobe: int):
    """The nprobe nearest centroids of one query, ascending, ties to smaller j.
    Returns (list ids int64, squared distances FP64)."""
    q = np.asarray(q, np.float64)
    C = np.asarray(C, np.float64)
    d = np.sum((C - q[None, :]) ** 2, axis=1)
    order = np.lexsort((np.arange(len(C)), d))[:nprobe]
    return order, d[order]


def rotate(q: np.ndarray, P: np.ndarray) -> np.ndarray:
    """q' = P^T q in FP64 (row form q @ P)."""
    return np.asarray(q, np.float64) @ np.asarray(P, np.float64)


def quantize(r: np.ndarray, bq: int):
    """B_q-bit uniform scalar quantisation of one query residual r (length D).

    v_l = min r, Delta = (max r - v_l) / (2^bq - 1), qu_d = floor((r_d - v_l)
    Delta^-1 + 1/2) clamped to [0, 2^bq - 1]; Delta = 0 gives qu = 0.
    Returns (qu int64, v_l, Delta, sum(qu)).
    """
    r = np.asarray(r, np.float64)
    top = (1 << bq) - 1
    vl = float(r.min())
    delta = (float(r.max()) - vl) / top
    inv = 1.0 / delta if delta > 0.0 else 0.0
    qu = np.floor((r - vl) * inv + 0.5)
    qu = np.clip(qu, 0, top).astype(np.int64)
    return qu, vl, delta, int(qu.sum())


def ip_dense(codes: np.ndarray, qu: np.ndarray, d: int) -> np.ndarray:
    """Integer inner products sum_d b01_d qu_d, as a dense product of small
    integers (exact in FP64 since the sum stays far below 2^53)."""
    b01 = unpack_bits(codes, d).astype(np.float64)
    return np.rint(b01 @ np.asarray(qu, np.float64)).astype(np.int64)


def bitplanes(qu: np.ndarray, bq: int) -> np.ndarray:
    """Bit-planes of qu: plane t holds bit t of every qu_d (0/1, [bq, D])."""
    qu = np.asarray(qu, np.int64)
    return np.stack([(qu >> t) & 1 for t in range(bq)]).astype(np.uint8)


def ip_bitplanes(codes: np.ndarray, qu: np.ndarray, d: int, bq: int) -> np.ndarray:
    """The same inner products by the bitwise route (Sec. 2.2.2 last paragraph):
    sum_t 2^t popcount(code AND plane_t), on packed bytes."""
    planes = pack_bits(bitplanes(qu, bq))          # [bq, ceil(D/8)]
    acc = np.zeros(len(codes), np.int64)
    for t in range(bq):
        anded = np.bitwise_and(codes, planes[t][None, :])
        acc += (1 << t) * np.unpackbits(anded, axis=1).sum(axis=1).astype(np.int64)
    return acc


def est_terms(codes: np.ndarray, qu, vl: float, delta: float, d: int):
    """E = sum_d b_d (v_l + Delta qu_d): the estimator's inner product of the
    sign code with the de-quantised residual (Eq. rabitq-ip-estimator times
    sqrt(D) alpha_x ||q - c||). Returns (E FP64, ip int64, pop int64)."""
    b01 = unpack_bits(codes, d).astype(np.float64)
    b = 2.0 * b01 - 1.0
    rq = vl + delta * np.asarray(qu, np.float64)
    E = b @ rq
    ip = np.rint(b01 @ np.asarray(qu, np.float64)).astype(np.int64)
    pop = b01.sum(axis=1).astype(np.int64)
    return E, ip, pop


def estimate(rnorm2: float, E: np.ndarray, n_x: np.ndarray, alpha: np.ndarray, d: int):
    """Eq. approx-dist with ||q - c|| s_hat = E / (sqrt(D) alpha_x):
    d_hat^2 = ||q - c||^2 + n_x^2 - 2 n_x E / (sqrt(D) alpha_x)."""
    n_x = np.asarray(n_x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    return rnorm2 + n_x * n_x - 2.0 * n_x * np.asarray(E, np.float64) / (np.sqrt(d) * alpha)


def s_hat_unquantized(P, codes, u_q, alpha, d):
    """Eq. rabitq-ip-estimator with an unquantised query: z_q = P^T u_q,
    s_hat = <b, z_q> / (sqrt(D) alpha_x)."""
    z_q = np.asarray(u_q, np.float64) @ np.asarray(P, np.float64)
    b = 2.0 * unpack_bits(codes, d).astype(np.float64) - 1.0
    return (b @ z_q) / (np.sqrt(d) * np.asarray(alpha, np.float64))


def est_terms_unquantized(codes: np.ndarray, r: np.ndarray, d: int):
    """E = sum_d b_d r_d with the query residual r = P^T q - P^T c kept in full
    precision: Eq. rabitq-ip-estimator without query quantisation (the form the
    paper's accelerator path evaluates, Sec. 4.3), times sqrt(D) alpha_x
    ||q - c||. Returns (E FP64, ip = sum_d b01_d r_d FP64, pop int64); since
    b = 2 b01 - 1, E = 2 ip - sum_d r_d."""
    b01 = unpack_bits(codes, d).astype(np.float64)
    b = 2.0 * b01 - 1.0
    r = np.asarray(r, np.float64)
    return b @ r, b01 @ r, b01.sum(axis=1).astype(np.int64)


def topk_lex(values: np.ndarray, ids: np.ndarray, k: int):
    """The k smallest (value, id) pairs in lexicographic order; if fewer than k
    exist, all of them followed by (+inf, -1) padding."""
    values = np.asarray(values, np.float64)
    ids = np.asarray(ids, np.int64)
    o = np.lexsort((ids, values))[:k]
    v = np.full(k, np.inf)
    i = np.full(k, -1, np.int64)
    v[:len(o)] = values[o]
    i[:len(o)] = ids[o]
    return v, i


def rerank(q: np.ndarray, X: np.ndarray, cand_ids: np.ndarray, k: int):
    """Exact re-rank of the coarse candidates (Sec. 3.1.2 Phase 5, Sec. 3.3.4):
    ||q - x||^2 in FP64, top-k by (distance, id), padded with (-1, +inf)."""
    cand_ids = np.asarray(cand_ids, np.int64)
    cand_ids = cand_ids[cand_ids >= 0]
    diff = np.asarray(X[cand_ids], np.float64) - np.asarray(q, np.float64)[None, :]
    d2 = np.sum(diff * diff, axis=1)
    return topk_lex(d2, cand_ids, k)


def brute_force_knn(X: np.ndarray, Q: np.ndarray, k: int, chunk: int = 1 << 16):
    """Exact kNN under squared L2 (Sec. 2.1.1), FP64, ties by id."""
    Q = np.asarray(Q, np.float64)
    best_d = np.full((len(Q), 0), np.inf)
    best_i = np.zeros((len(Q), 0), np.int64)
    for s in range(0, len(X), chunk):
        Xc = np.asarray(X[s:s + chunk], np.float64)
        d = np.maximum(sqdist(Q, Xc), 0.0)
        ids = np.broadcast_to(np.arange(s, s + len(Xc)), d.shape)
        allv = np.concatenate([best_d, d], axis=1)
        alli = np.concatenate([best_i, ids], axis=1)
        o = np.lexsort((alli, allv), axis=1)[:, :k]
        best_d = np.take_along_axis(allv, o, 1)
        best_i = np.take_along_axis(alli, o, 1)
    # final values as exact direct differences
    for qi in range(len(Q)):
        diff = np.asarray(X[best_i[qi]], np.float64) - Q[qi]
        best_d[qi] = np.sum(diff * diff, axis=1)
        o = np.lexsort((best_i[qi], best_d[qi]))
        best_d[qi], best_i[qi] = best_d[qi][o], best_i[qi][o]
    return best_i, best_d


@dataclass
class Index:
    """An IVF-RaBitQ index as the oracle holds it (all arrays in id order)."""
    d: int
    bq: int
    centroids: np.ndarray        # [nlist, D] float32
    P: np.ndarray                # [D, D] float32
    assign: np.ndarray           # [N] int64
    codes: np.ndarray            # [N, ceil(D/8)] uint8
    n_x: np.ndarray              # [N] float32
    alpha: np.ndarray            # [N] float32
    lists: list = field(default_factory=list)   # ids per list, ascending

    @property
    def nlist(self):
        return len(self.centroids)


def build(X, nlist=None, *, bq=4, centroids=None, P=None, assignment=None, rng=None,
          kmeans_iters=25, kmeans_restarts=3) -> Index:
    """Index construction (Sec. 3.1.1): centroids (given or k-means), the
    assignment of every vector to its nearest centroid (given or computed),
    random orthogonal P (given or drawn) and the RaBitQ encoding of every
    vector against its centroid. Centroids and P are stored as FP32, as the
    GPU index stores them; all arithmetic is FP64 from those FP32 values."""
    X = np.asarray(X, np.float32)
    n, d = X.shape
    if rng is None:
        rng = np.random.default_rng(0)
    if centroids is None:
        centroids = kmeans(X, nlist, rng, iters=kmeans_iters, restarts=kmeans_restarts)
    C = np.asarray(centroids, np.float32)
    if P is None:
        P = random_orthogonal(d, rng)
    P = np.asarray(P, np.float32)
    if assignment is None:
        assignment, _ = assign(X, C)
    a = np.asarray(assignment, np.int64)
    codes, n_x, alpha = encode(X, C, a, P)
    order = np.argsort(a, kind="stable")
    bounds = np.searchsorted(a[order], np.arange(len(C) + 1))
    lists = [order[bounds[j]:bounds[j + 1]] for j in range(len(C))]
    return Index(d=d, bq=bq, centroids=C, P=P, assign=a, codes=codes, n_x=n_x,
                 alpha=alpha, lists=lists)


def search(index: Index, X: np.ndarray, Q: np.ndarray, nprobe: int, k: int, rerank_n: int,
           stages: bool = False, probes=None, unquantized: bool = False):
    """IVF-RaBitQ search of a batch (Sec. 3.1.2 Phases 1, 3, 4, 5).

    For each query: probe the nprobe nearest lists; for each probed list j,
    r = P^T q - P^T c_j, quantise r to bq bits, estimate d_hat^2 for every
    vector of the list; keep the rerank_n smallest (d_hat^2, id); re-rank them
    by exact distance and return the k best (ids int64 [nq,k], sqdist FP64).
    With ``unquantized`` the residual r enters the estimator as it is (no
    query quantisation: E = sum_d b_d r_d, ``est_terms_unquantized``).
    With ``stages`` also returns a dict of every intermediate result.
    ``probes`` optionally fixes the probed lists ([nq, nprobe] list ids).
    """
    Q = np.asarray(Q, np.float32)
    nq = len(Q)
    d = index.d
    P = index.P
    Cr = np.asarray(index.centroids, np.float64) @ np.asarray(P, np.float64)   # P^T c_j
    out_ids = np.full((nq, k), -1, np.int64)
    out_d = np.full((nq, k), np.inf)
    st = {"probes": [], "probe_dist": [], "qrot": [], "qu": [], "vl": [], "delta": [],
          "rnorm2": [], "sumqu": [], "cand_ids": [], "cand_est": [], "per_list": []}
    for qi in range(nq):
        if probes is None:
            pr, pd = probe(Q[qi], index.centroids, nprobe)
        else:
            pr = np.asarray(probes[qi], np.int64)
            pd = np.sum((np.asarray(index.centroids[pr], np.float64) - Q[qi].astype(np.float64)) ** 2, axis=1)
        qrot = rotate(Q[qi], P)
        all_e, all_i = [], []
        qus, vls, dls, rns, sqs, pls = [], [], [], [], [], []
        for j in pr:
            r = qrot - Cr[j]
            rnorm2 = float(r @ r)
            ids = index.lists[j]
            if unquantized:
                qu, vl, delta, squ = None, 0.0, 0.0, 0
                E, ip, pop = est_terms_unquantized(index.codes[ids], r, d)
            else:
                qu, vl, delta, squ = quantize(r, index.bq)
                E, ip, pop = est_terms(index.codes[ids], qu, vl, delta, d)
            est = estimate(rnorm2, E, index.n_x[ids], index.alpha[ids], d)
            all_e.append(est)
            all_i.append(ids)
            if stages:
                qus.append(qu); vls.append(vl); dls.append(delta)
                rns.append(rnorm2); sqs.append(squ)
                pls.append({"ids": ids, "ip": ip, "pop": pop, "E": E, "est": est, "r": r})
        e = np.concatenate(all_e) if all_e else np.zeros(0)
        ii = np.concatenate(all_i) if all_i else np.zeros(0, np.int64)
        ce, ci = topk_lex(e, ii, rerank_n)
        fd, fi = rerank(Q[qi], X, ci, k)
        out_ids[qi], out_d[qi] = fi, fd
        if stages:
            st["probes"].append(pr); st["probe_dist"].append(pd); st["qrot"].append(qrot)
            st["qu"].append(np.array(qus)); st["vl"].append(np.array(vls))
            st["delta"].append(np.array(dls)); st["rnorm2"].append(np.array(rns))
            st["sumqu"].append(np.array(sqs)); st["cand_ids"].append(ci)
            st["cand_est"].append(ce); st["per_list"].append(pls)
    if stages:
        return out_ids, out_d, st
    return out_ids, out_d


def ivf_flat_search(index: Index, X: np.ndarray, Q: np.ndarray, nprobe: int, k: int):
    """IVF-Flat search (Sec. 2.1.2 query processing with full-precision
    vectors, the comparison system of Sec. 4.2): probe the nprobe nearest
    lists, compute the exact squared distance ||q - x||^2 (FP64) to every
    vector in them and return the k best by (distance, id), padded with
    (-1, +inf). Returns (ids int64 [nq, k], sqdist FP64 [nq, k])."""
    Q = np.asarray(Q, np.float32)
    nq = len(Q)
    out_ids = np.full((nq, k), -1, np.int64)
    out_d = np.full((nq, k), np.inf)
    for qi in range(nq):
        pr, _ = probe(Q[qi], index.centroids, nprobe)
        ids = np.concatenate([index.lists[j] for j in pr]) if len(pr) else np.zeros(0, np.int64)
        diff = np.asarray(X[ids], np.float64) - np.asarray(Q[qi], np.float64)[None, :]
        out_d[qi], out_ids[qi] = topk_lex(np.sum(diff * diff, axis=1), ids, k)
    return out_ids, out_d
