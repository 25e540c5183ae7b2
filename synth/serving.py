"""Seeded request streams for the serving workload.

Half of the requests solve anisotropic diffusion on 2D or 3D grids, half a
general nonsymmetric sparse matrix with power-law row lengths; 70 % of them
bring a new right-hand side for a matrix id seen among the last 32 ids, the
rest a new matrix.  Arrivals are a Poisson process.  Everything is drawn
from SplitMix64 streams (see generators.py) with base seed 5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .generators import CSR, _GOLDEN, _M1, _M2, aniso5, aniso7, block_partition, splitmix64, uniform01

ROW_CAP = 448  # longest off-diagonal row drawn (the device factorization keeps 512 entries per working row)
PART_ROWS = 65536  # rows per subdomain: p = ceil(n / 65536) contiguous blocks


def _mix(z: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function applied to each state."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def general_sparse(n: int, mean_len: float, seed: int, rho: float | None = None, alpha: float = 2.5,
                   cap: int = ROW_CAP) -> CSR:
    """Nonsymmetric banded matrix with power-law row lengths (vectorised).

    Off-diagonal row length k_i = floor(x_min / (1 - u)^(1/alpha)) (Pareto with
    x_min = mean_len / 3), clipped to [1, min(n - 1, cap)]; up to k_i distinct
    columns drawn uniformly from |j - i| <= max(2 mean_len, k_i), j != i
    (oversampled draws, then the k_i of smallest seeded priority); values
    U(-1, 1); a_ii = rho * sum_j |a_ij| with rho ~ U(1.05, 2) unless given.
    """
    u = uniform01(seed, n + 1)
    if rho is None:
        rho = 1.05 + 0.95 * u[0]
    if n == 1:
        return CSR(1, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.ones(1))
    xmin = mean_len / 3.0
    k = np.floor(xmin / np.power(1.0 - u[1:], 1.0 / alpha)).astype(np.int64)
    k = np.clip(k, 1, min(n - 1, cap))
    i = np.arange(n, dtype=np.int64)
    w = np.maximum(int(2 * mean_len), k)
    lo = np.maximum(0, i - w)
    hi = np.minimum(n - 1, i + w)
    span = hi - lo  # candidates: [lo, hi] without i
    k = np.minimum(k, span)
    draws = (3 * k) // 2 + 8
    rows = np.repeat(i, draws)
    r = uniform01(seed * 7919 + 1, int(draws.sum()))
    c = lo[rows] + np.floor(r * span[rows]).astype(np.int64)
    c += c >= rows  # skip the diagonal
    key = np.unique(rows * n + c)
    rows = key // n
    prio = _mix(key.astype(np.uint64) * _GOLDEN + np.uint64(seed * 104729 + 3))
    bits = max(1, int(n - 1).bit_length())  # (row, priority) in one 64-bit sort key
    order = np.argsort((rows.astype(np.uint64) << np.uint64(64 - bits)) | (prio >> np.uint64(bits)))
    rows, key = rows[order], key[order]
    start = np.searchsorted(rows, i)
    rank = np.arange(rows.size, dtype=np.int64) - start[rows]
    keep = rank < k[rows]
    key = np.sort(key[keep])
    rows = key // n
    cols = key % n
    vals = 2.0 * uniform01(seed * 7919 + 2, key.size) - 1.0
    diag = rho * np.bincount(rows, weights=np.abs(vals), minlength=n)
    diag[diag == 0.0] = 1.0
    allk = np.concatenate([key, i * n + i])
    allv = np.concatenate([vals, diag])
    o = np.argsort(allk, kind="stable")
    allk, allv = allk[o], allv[o]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(allk // n, minlength=n), out=rp[1:])
    return CSR(n, rp, (allk % n).astype(np.int32), allv)


@dataclass
class Request:
    """One request of the stream: which matrix (id and how to build it) and its right-hand side seed."""

    index: int
    matrix_id: int
    new: bool  # first request of this id
    kind: str  # "grid2d", "grid3d" or "general"
    n_target: int
    param: float  # 2D: eps; general: mean row length m
    rhs_seed: int


def request_stream(count: int, seed: int = 5, reuse: float = 0.7, window: int = 32, n_min: float = 1e3,
                   n_max: float = 1e6) -> list[Request]:
    """The request mix: with probability `reuse` (once any id exists) a new right-hand side for an id drawn
    uniformly from the last `window` ids, else a new matrix: half anisotropic grids (2D with eps log-U[1e-3, 1]
    or 3D with coefficients (1, 0.1, 0.01), equally likely), half general matrices with m ~ U(10, 50);
    n log-uniform in [n_min, n_max]."""
    u = uniform01(seed, 8 * count)
    out, recent, info = [], [], {}
    for q in range(count):
        d = u[8 * q: 8 * q + 8]
        if recent and d[0] < reuse:
            mid = recent[int(d[1] * len(recent))]
            kind, n, p = info[mid]
            out.append(Request(q, mid, False, kind, n, p, (seed << 32) + q))
            continue
        mid = len(info)
        n = int(round(math.exp(math.log(n_min) + d[2] * (math.log(n_max) - math.log(n_min)))))
        if d[3] < 0.5:
            kind = "grid2d" if d[4] < 0.5 else "grid3d"
            p = math.exp(math.log(1e-3) + d[5] * (0.0 - math.log(1e-3))) if kind == "grid2d" else 0.0
        else:
            kind = "general"
            p = 10.0 + 40.0 * d[5]
        info[mid] = (kind, n, p)
        recent.append(mid)
        if len(recent) > window:
            recent.pop(0)
        out.append(Request(q, mid, True, kind, n, p, (seed << 32) + q))
    return out


def build_matrix(req: Request, seed: int = 5, part_rows: int = PART_ROWS):
    """(A, part, nparts) of a request's matrix: grids of side round(n^(1/d)), general matrices of n rows;
    p = ceil(n / part_rows) contiguous row blocks (65536 rows each by default)."""
    if req.kind == "grid2d":
        N = max(2, int(round(math.sqrt(req.n_target))))
        A = aniso5(N, req.param)
    elif req.kind == "grid3d":
        N = max(2, int(round(req.n_target ** (1.0 / 3.0))))
        A = aniso7(N)
    else:
        A = general_sparse(req.n_target, req.param, (seed << 40) + req.matrix_id)
    p = max(1, -(-A.n // part_rows))
    return A, block_partition(A.n, p), p


def arrival_times(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Poisson arrivals at `rate` per second: cumulative exponential gaps (first arrival at 0)."""
    u = uniform01((seed << 32) + 0xA11, count)
    gaps = -np.log1p(-u) / rate
    t = np.cumsum(gaps)
    return t - t[0]
