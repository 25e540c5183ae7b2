"""Seeded CSR generators for the model problems of the two-level ILU paper.

The paper's experiments use finite-difference Laplacians on the unit square and
cube (Section 4.1, equation (31) for the 3-D convection-diffusion operator);
the generators below are anisotropic / rotated / upwinded variants of those
operators.  Conventions shared by every generator:

* natural ordering, x fastest: ``idx = ix + Nx*iy (+ Nx*Ny*iz)``;
* homogeneous Dirichlet boundary unknowns are eliminated, so stencil points
  that fall outside the grid are simply dropped;
* every stencil is scaled by ``h**2`` (this leaves Krylov iteration counts
  unchanged);
* columns inside a row are sorted ascending, the diagonal is always present.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), mapped to doubles in [0, 1) as
``(x >> 11) * 2**-53``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


@dataclass
class CSR:
    """Host CSR matrix: int64 row pointers, int32 sorted columns, float64 values."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d

    def matvec(self, x: np.ndarray) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        y = np.zeros(self.n)
        np.add.at(y, rows, self.val * x[self.col])
        return y

    @staticmethod
    def from_dense(d: np.ndarray) -> "CSR":
        d = np.asarray(d, dtype=np.float64)
        n = d.shape[0]
        mask = d != 0
        np.fill_diagonal(mask, True)
        counts = mask.sum(axis=1)
        rp = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=rp[1:])
        r, c = np.nonzero(mask)
        return CSR(n, rp, c.astype(np.int32), d[r, c].astype(np.float64))


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------

def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream seeded with ``seed``."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    return (splitmix64(seed, count, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_rhs(n: int, seed: int) -> np.ndarray:
    """b_i = 2u - 1 with u from SplitMix64(seed): a seeded U(-1, 1) right-hand side."""
    return 2.0 * uniform01(seed, n) - 1.0


# --------------------------------------------------------------------------
# structured stencils
# --------------------------------------------------------------------------

def _stencil(dims, offsets):
    """CSR of a constant-coefficient stencil on a tensor grid.

    ``offsets`` is a list of ((dx, dy, dz), coef) sorted by linear offset, so
    entries of a row come out column-sorted.
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    ix = idx % nx
    iy = (idx // nx) % ny
    iz = idx // (nx * ny)
    offsets = sorted(offsets, key=lambda o: o[0][2] * nx * ny + o[0][1] * nx + o[0][0])
    noff = len(offsets)
    cols = np.empty((n, noff), dtype=np.int64)
    vals = np.empty((n, noff), dtype=np.float64)
    mask = np.empty((n, noff), dtype=bool)
    for k, ((dx, dy, dz), coef) in enumerate(offsets):
        m = (ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < ny) & (iz + dz >= 0) & (iz + dz < nz)
        mask[:, k] = m
        cols[:, k] = idx + dz * nx * ny + dy * nx + dx
        vals[:, k] = coef
    counts = mask.sum(axis=1)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return CSR(n, rp, cols[mask].astype(np.int32), vals[mask])


def aniso5(N: int, cy: float = 0.01, Ny: int | None = None) -> CSR:
    """-(u_xx + cy u_yy) on an N x Ny grid, 5-point stencil scaled by h^2."""
    Ny = N if Ny is None else Ny
    offs = [((0, -1, 0), -cy), ((-1, 0, 0), -1.0), ((0, 0, 0), 2.0 + 2.0 * cy),
            ((1, 0, 0), -1.0), ((0, 1, 0), -cy)]
    return _stencil((N, Ny, 1), offs)


def aniso7(N: int, c=(1.0, 0.1, 0.01), Ny: int | None = None, Nz: int | None = None) -> CSR:
    """-(cx u_xx + cy u_yy + cz u_zz) on an N^3 grid, 7-point stencil scaled by h^2."""
    cx, cy, cz = c
    Ny = N if Ny is None else Ny
    Nz = N if Nz is None else Nz
    offs = [((0, 0, -1), -cz), ((0, -1, 0), -cy), ((-1, 0, 0), -cx),
            ((0, 0, 0), 2.0 * (cx + cy + cz)),
            ((1, 0, 0), -cx), ((0, 1, 0), -cy), ((0, 0, 1), -cz)]
    return _stencil((N, Ny, Nz), offs)


def rotated9(N: int, eps: float = 1e-3, theta: float = math.pi / 6) -> CSR:
    """-div(K grad u), K = R(theta) diag(1, eps) R(theta)^T, 9-point stencil scaled by h^2."""
    cs, sn = math.cos(theta), math.sin(theta)
    a = cs * cs + eps * sn * sn
    c = sn * sn + eps * cs * cs
    b = (1.0 - eps) * cs * sn
    offs = [((-1, -1, 0), -b / 2), ((0, -1, 0), -c), ((1, -1, 0), b / 2),
            ((-1, 0, 0), -a), ((0, 0, 0), 2 * a + 2 * c), ((1, 0, 0), -a),
            ((-1, 1, 0), b / 2), ((0, 1, 0), -c), ((1, 1, 0), -b / 2)]
    return _stencil((N, N, 1), offs)


def convdiff5(s: int, eps: float, theta: float, pe: float) -> CSR:
    """-(u_xx + eps u_yy) + v . grad u, v = pe (cos theta, sin theta), first-order upwind."""
    h = 1.0 / (s + 1)
    vx, vy = pe * math.cos(theta), pe * math.sin(theta)
    offs = [((0, -1, 0), -eps - h * max(vy, 0.0)), ((-1, 0, 0), -1.0 - h * max(vx, 0.0)),
            ((0, 0, 0), 2.0 + 2.0 * eps + h * (abs(vx) + abs(vy))),
            ((1, 0, 0), -1.0 - h * max(-vx, 0.0)), ((0, 1, 0), -eps - h * max(-vy, 0.0))]
    return _stencil((s, s, 1), offs)


def convdiff_batch_params(count: int, seed: int = 4):
    """Per-system (side, eps, theta, Pe): side log-uniform in [32, 256], eps log-uniform
    in [1e-3, 1], theta uniform in [0, pi), Pe uniform in [0, 50]; system k draws from
    its own SplitMix64 stream seeded with ``seed * 2**32 + k``."""
    out = []
    for k in range(count):
        u = uniform01(seed * (1 << 32) + k, 4)
        side = int(round(math.exp(math.log(32) + u[0] * (math.log(256) - math.log(32)))))
        eps = math.exp(math.log(1e-3) + u[1] * (0.0 - math.log(1e-3)))
        out.append((side, eps, math.pi * u[2], 50.0 * u[3]))
    return out


def block_diagonal(mats):
    """One block-diagonal CSR of the given systems (global column numbering) and the first row of each system
    ([len(mats) + 1] int64)."""
    sys_row = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum([m.n for m in mats], out=sys_row[1:])
    nnz = np.zeros(len(mats) + 1, dtype=np.int64)
    np.cumsum([m.nnz for m in mats], out=nnz[1:])
    rp = np.concatenate([m.row_ptr[:-1] + nnz[k] for k, m in enumerate(mats)] + [nnz[-1:]])
    col = np.concatenate([m.col.astype(np.int64) + sys_row[k] for k, m in enumerate(mats)]).astype(np.int32)
    val = np.concatenate([m.val for m in mats])
    return CSR(int(sys_row[-1]), rp.astype(np.int64), col, val), sys_row


def convdiff_batch(count: int, seed: int = 4):
    """The batched workload: `count` convection-diffusion systems with the parameters of
    convdiff_batch_params, as a list of CSR matrices, and their right-hand sides b_k = A_k 1."""
    mats = [convdiff5(*p) for p in convdiff_batch_params(count, seed)]
    return mats, [m.matvec(np.ones(m.n)) for m in mats]


# --------------------------------------------------------------------------
# partitions
# --------------------------------------------------------------------------

def slab_partition(N: int, nslabs: int, Ny: int | None = None, Nz: int | None = None) -> np.ndarray:
    """part[i] = iz // (Nz / nslabs) on an N x Ny x Nz grid (x fastest)."""
    Ny = N if Ny is None else Ny
    Nz = N if Nz is None else Nz
    if Nz % nslabs:
        raise ValueError("Nz must be divisible by nslabs")
    iz = np.arange(N * Ny * Nz, dtype=np.int64) // (N * Ny)
    return (iz // (Nz // nslabs)).astype(np.int32)


def block_partition(n: int, nparts: int) -> np.ndarray:
    """Contiguous row blocks of near-equal size."""
    return ((np.arange(n, dtype=np.int64) * nparts) // max(n, 1)).astype(np.int32)


# --------------------------------------------------------------------------
# general nonsymmetric matrices
# --------------------------------------------------------------------------

def random_sparse(n: int, mean_len: float, seed: int, rho: float | None = None,
                  band: int | None = None, alpha: float = 2.5) -> CSR:
    """Banded random nonsymmetric matrix with power-law row lengths.

    Off-diagonal row lengths follow a Pareto(alpha, x_min = mean_len/3) law,
    floored and clipped to [1, n-1]; columns are distinct and uniform within
    ``|j - i| <= max(band, k_i)``; values are U(-1, 1); the diagonal is
    ``rho * sum_j |a_ij|`` with rho ~ U(1.05, 2) unless given.
    """
    rng_u = uniform01(seed, 4 * n + 2)
    if rho is None:
        rho = 1.05 + 0.95 * rng_u[0]
    band = max(1, int(band if band is not None else 2 * mean_len))
    xmin = mean_len / 3.0
    lens = np.floor(xmin / np.power(1.0 - rng_u[2:2 + n], 1.0 / alpha)).astype(np.int64)
    lens = np.clip(lens, 1, max(n - 1, 1)) if n > 1 else np.zeros(n, dtype=np.int64)
    rows_c, rows_v = [], []
    stream = seed * 7919 + 17
    for i in range(n):
        k = int(lens[i])
        w = max(band, k)
        lo, hi = max(0, i - w), min(n - 1, i + w)
        cand = np.concatenate([np.arange(lo, i), np.arange(i + 1, hi + 1)])
        k = min(k, cand.size)
        # choose k distinct candidates by sorting seeded keys
        keys = splitmix64(stream, cand.size, start=0)
        stream += 1
        pick = np.sort(cand[np.argsort(keys, kind="stable")[:k]])
        v = 2.0 * uniform01(stream, k) - 1.0
        stream += 1
        d = rho * float(np.abs(v).sum()) if k else 1.0
        c = np.concatenate([pick, [i]])
        vals = np.concatenate([v, [d]])
        o = np.argsort(c, kind="stable")
        rows_c.append(c[o])
        rows_v.append(vals[o])
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(c) for c in rows_c], out=rp[1:])
    col = np.concatenate(rows_c).astype(np.int32) if n else np.zeros(0, np.int32)
    val = np.concatenate(rows_v) if n else np.zeros(0)
    return CSR(n, rp, col, val)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def workload(name: str):
    """Return (A, b, part, nparts) for a named workload.

    * ``aniso2d_64``: -(u_xx + 0.01 u_yy), 64 x 64, one block, b = A 1.
    * ``aniso3d_128_slab16``: -(u_xx + 0.1 u_yy + 0.01 u_zz), 128^3, 16 z-slabs,
      b = U(-1, 1) from SplitMix64 seed 2.
    * ``aniso3d_<N>_slab<p>``: the same operator at other sizes (tests).
    * ``rot9_2048``: rotated anisotropic 9-point, eps 1e-3, theta pi/6, b seed 3.
    """
    if name == "aniso2d_64":
        A = aniso5(64, 0.01)
        return A, A.matvec(np.ones(A.n)), np.zeros(A.n, np.int32), 1
    if name.startswith("aniso3d_"):
        rest = name[len("aniso3d_"):]
        n_str, p_str = rest.split("_slab")
        N, p = int(n_str), int(p_str)
        A = aniso7(N)
        return A, uniform_rhs(A.n, 2), slab_partition(N, p), p
    if name.startswith("aniso2d_"):
        N = int(name[len("aniso2d_"):])
        A = aniso5(N, 0.01)
        return A, A.matvec(np.ones(A.n)), np.zeros(A.n, np.int32), 1
    if name.startswith("rot9_"):
        N = int(name[len("rot9_"):])
        A = rotated9(N)
        return A, uniform_rhs(A.n, 3), np.zeros(A.n, np.int32), 1
    raise KeyError(name)
