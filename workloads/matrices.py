"""Synthetic sparse systems shaped like the paper's workloads.

The paper's test matrices (SuiteSparse, HPCG, HPGMP; Sec. 5, Table 2) are not
available here; these seeded generators stand in for them.  All matrices are
CSR with 0-based int32 row pointers and sorted, unique int32 column indices,
lexicographic ordering with x fastest and Dirichlet boundaries eliminated.

Nothing here is part of the solver: it only produces A, x* and b = A x*.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from . import rng


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray      # float64, nnz
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x in fp64, summed row by row in CSR order (input generation)."""
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        return np.bincount(rows, weights=self.val * x[self.col_idx], minlength=self.n)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


# ---------------------------------------------------------------------------
# structured stencils on a box grid
# ---------------------------------------------------------------------------

def _stencil_csr(shape, offsets, coeffs, name=""):
    """CSR of a stencil operator on a grid of `shape` = (nz, ny, nx).

    offsets: list of (dz, dy, dx); coeffs: list of arrays broadcastable to
    `shape` giving the entry of each row for that offset.  Entries whose
    column falls outside the grid are dropped (Dirichlet elimination).
    Columns come out sorted because offsets are visited in increasing
    linear-offset order.
    """
    nz, ny, nx = shape
    n = nz * ny * nx
    lin = [dz * ny * nx + dy * nx + dx for dz, dy, dx in offsets]
    order = np.argsort(lin, kind="stable")
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    z, y, x = z.reshape(-1), y.reshape(-1), x.reshape(-1)
    rows_idx = np.arange(n, dtype=np.int64)
    K = len(offsets)
    # built offset-major (contiguous per offset), then transposed once
    valid = np.zeros((K, n), dtype=bool)
    cols = np.zeros((K, n), dtype=np.int64)
    vals = np.zeros((K, n), dtype=np.float64)
    for kk, o in enumerate(order):
        dz, dy, dx = offsets[o]
        valid[kk] = (z + dz >= 0) & (z + dz < nz) & (y + dy >= 0) & (y + dy < ny) & (x + dx >= 0) & (x + dx < nx)
        cols[kk] = rows_idx + lin[o]
        vals[kk] = np.broadcast_to(np.asarray(coeffs[o], dtype=np.float64), shape).reshape(-1)
    valid = np.ascontiguousarray(valid.T)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = np.ascontiguousarray(cols.T)[valid].astype(np.int32)
    val = np.ascontiguousarray(vals.T)[valid]
    return CSR(n, row_ptr.astype(np.int32), col_idx, val, name)


def poisson2d(N: int) -> CSR:
    """5-point Laplacian on an N x N interior grid: 4 on the diagonal, -1 off.
    nnz = 5N^2 - 4N."""
    offs = [(0, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    coef = [4.0, -1.0, -1.0, -1.0, -1.0]
    return _stencil_csr((1, N, N), offs, coef, f"poisson2d_{N}")


def poisson3d(N: int) -> CSR:
    """7-point Laplacian on an N^3 interior grid: 6 on the diagonal, -1 off.
    nnz = 7N^3 - 6N^2."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    coef = [6.0] + [-1.0] * 6
    return _stencil_csr((N, N, N), offs, coef, f"poisson3d_{N}")


def hpcg(nx: int, ny: int, nz: int) -> CSR:
    """HPCG-like 27-point operator (Sec. 5): 26 on the diagonal, -1 for the
    26 neighbours.  nnz = (3nx-2)(3ny-2)(3nz-2)."""
    offs = list(itertools.product((-1, 0, 1), repeat=3))
    coef = [26.0 if o == (0, 0, 0) else -1.0 for o in offs]
    return _stencil_csr((nz, ny, nx), offs, coef, f"hpcg_{nx}_{ny}_{nz}")


def hpgmp(nx: int, ny: int, nz: int, beta: float = 0.5) -> CSR:
    """HPGMP-like operator (Sec. 5): the HPCG 27-point operator with the
    couplings to the forward and backward neighbours along z replaced by
    -1 + beta and -1 - beta (nonsymmetric; beta = 0.5 as in the paper's
    runs).  nnz = (3nx-2)(3ny-2)(3nz-2)."""
    offs = list(itertools.product((-1, 0, 1), repeat=3))

    def coef(o):
        if o == (0, 0, 0):
            return 26.0
        if o == (1, 0, 0):
            return -1.0 + beta
        if o == (-1, 0, 0):
            return -1.0 - beta
        return -1.0

    return _stencil_csr((nz, ny, nx), offs, [coef(o) for o in offs], f"hpgmp_{nx}_{ny}_{nz}")


def paper_rhs(A: CSR, tag: str) -> np.ndarray:
    """Right-hand side of the paper's runs (Sec. 5): uniform on [0, 1)."""
    return rng.uniform01(rng.substream(f"rhs-paper/{tag}"), A.n)


# ---------------------------------------------------------------------------
# cfg3: Q1 convection-diffusion, lognormal diffusion, Peclet 50
# ---------------------------------------------------------------------------

def convdiff_q1(N: int = 100, sigma: float = 1.5, peclet: float = 50.0,
                tag: str = "convdiff") -> CSR:
    """Galerkin trilinear (Q1) finite elements for -div(k grad u) + w.grad u
    on the unit cube with (N+1)^3 elements and N^3 interior nodes.
    k_e = exp(sigma xi_e), xi_e ~ N(0,1) per element; w = peclet * d with d
    uniform on the unit sphere.  Element integrals are exact tensor products
    of the 1-D integrals (equal to 2-point Gauss).  27-point, nonsymmetric.
    """
    E = N + 1
    h = 1.0 / E
    seed_k = rng.substream(f"{tag}/kappa/{N}")
    seed_w = rng.substream(f"{tag}/wind/{N}")
    kappa = np.exp(sigma * rng.normal(seed_k, E ** 3)).reshape(E, E, E)  # [ez, ey, ex]
    dvec = rng.normal(seed_w, 3)
    dvec = dvec / np.linalg.norm(dvec)
    w = peclet * dvec  # (wx, wy, wz)
    m1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])   # int psi_i psi_j on [0,1]
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])          # int psi_i' psi_j'
    c1 = np.array([[-0.5, 0.5], [-0.5, 0.5]])          # int psi_i psi_j'
    offs = list(itertools.product((-1, 0, 1), repeat=3))  # (dz, dy, dx)
    coef = {o: np.zeros((N, N, N)) for o in offs}
    corners = list(itertools.product((0, 1), repeat=3))  # (az, ay, ax)
    for a in corners:
        for b in corners:
            az, ay, ax = a
            bz, by, bx = b
            kdiff = h * (k1[ax, bx] * m1[ay, by] * m1[az, bz]
                         + m1[ax, bx] * k1[ay, by] * m1[az, bz]
                         + m1[ax, bx] * m1[ay, by] * k1[az, bz])
            conv = h * h * (w[0] * c1[ax, bx] * m1[ay, by] * m1[az, bz]
                            + w[1] * m1[ax, bx] * c1[ay, by] * m1[az, bz]
                            + w[2] * m1[ax, bx] * m1[ay, by] * c1[az, bz])
            off = (bz - az, by - ay, bx - ax)
            # element e = row_node - a; interior row nodes 1..N in the (N+2)-grid
            sl = tuple(slice(1 - ai, N + 1 - ai) for ai in (az, ay, ax))
            coef[off] += kdiff * kappa[sl] + conv
    return _stencil_csr((N, N, N), offs, [coef[o] for o in offs], f"convdiff_q1_{N}")


# ---------------------------------------------------------------------------
# cfg4: elasticity-like bond model with 3x3 blocks
# ---------------------------------------------------------------------------

def elasticity_bonds(N: int = 64, nu: float = 0.3, sigma: float = 1.0,
                     jitter: float = 0.2, tag: str = "elastic") -> CSR:
    """3 dof per point of a jittered N^3 lattice; each point is bonded to its
    26 lattice neighbours.  Bond stiffness (E_e / l) [d d^T + beta (I - d d^T)]
    with beta = (1 - 2 nu) / (2 (1 - nu)) and E_e = exp(sigma xi_e).
    Assembled as a block Laplacian; a penalty (mean diagonal) * I on the
    points of the x = 0 face makes it SPD.  nnz = 9 (3N - 2)^3.
    """
    h = 1.0 / N
    nn = N ** 3
    seed_p = rng.substream(f"{tag}/points/{N}")
    seed_e = rng.substream(f"{tag}/modulus/{N}")
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    pts = np.stack([x, y, z], axis=-1).reshape(-1, 3).astype(np.float64) * h
    pts += h * rng.uniform(seed_p, 3 * nn, -jitter, jitter).reshape(nn, 3)
    beta = (1 - 2 * nu) / (2 * (1 - nu))
    offs = list(itertools.product((-1, 0, 1), repeat=3))  # (dz, dy, dx)
    fwd = [o for o in offs if o > (0, 0, 0)]  # 13 directions
    blocks = {o: np.zeros((nn, 3, 3)) for o in offs}
    zi, yi, xi = z.reshape(-1), y.reshape(-1), x.reshape(-1)
    eye = np.eye(3)
    for di, o in enumerate(fwd):
        dz, dy, dx = o
        ok = ((zi + dz >= 0) & (zi + dz < N) & (yi + dy >= 0) & (yi + dy < N)
              & (xi + dx >= 0) & (xi + dx < N))
        p = np.nonzero(ok)[0]
        q = p + dz * N * N + dy * N + dx
        vec = pts[q] - pts[p]
        ell = np.linalg.norm(vec, axis=1)
        d = vec / ell[:, None]
        Ee = np.exp(sigma * rng.normal(seed_e, p.size, start=di * nn))
        dd = d[:, :, None] * d[:, None, :]
        k = (Ee / ell)[:, None, None] * (dd + beta * (eye - dd))
        neg = (-dz, -dy, -dx)
        blocks[(0, 0, 0)][p] += k
        blocks[(0, 0, 0)][q] += k
        blocks[o][p] -= k
        blocks[neg][q] -= k
    diag = np.einsum("nii->ni", blocks[(0, 0, 0)])
    mean_diag = diag.mean()
    anchor = xi == 0
    blocks[(0, 0, 0)][anchor] += mean_diag * eye
    # expand node blocks to dof rows: row 3p+c, columns 3q+c' for sorted q
    lin = [dz * N * N + dy * N + dx for dz, dy, dx in offs]
    order = np.argsort(lin, kind="stable")
    nd = 3 * nn
    K = len(offs) * 3
    # built offset-major (contiguous per offset), then transposed once
    valid = np.zeros((K, nn, 3), dtype=bool)
    cols = np.zeros((K, nn, 3), dtype=np.int32)
    vals = np.zeros((K, nn, 3))
    node = np.arange(nn, dtype=np.int64)
    for kk, o in enumerate(order):
        dz, dy, dx = offs[o]
        ok = ((zi + dz >= 0) & (zi + dz < N) & (yi + dy >= 0) & (yi + dy < N)
              & (xi + dx >= 0) & (xi + dx < N))
        qn = node + lin[o]
        for cp in range(3):
            valid[3 * kk + cp] = ok[:, None]
            cols[3 * kk + cp] = (3 * qn + cp)[:, None]
            vals[3 * kk + cp] = blocks[offs[o]][:, :, cp]
    valid = np.ascontiguousarray(valid.transpose(1, 2, 0)).reshape(nd, K)
    cols = np.ascontiguousarray(cols.transpose(1, 2, 0)).reshape(nd, K)
    vals = np.ascontiguousarray(vals.transpose(1, 2, 0)).reshape(nd, K)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(nd + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(nd, row_ptr.astype(np.int32), cols[valid].astype(np.int32), vals[valid],
               f"elasticity_bonds_{N}")


# ---------------------------------------------------------------------------
# cfg5: variable-coefficient 2-D systems for the batched solve
# ---------------------------------------------------------------------------

def varcoef2d(s: int, sigma: float = 1.0, tag: str = "varcoef2d/0") -> CSR:
    """Cell-centred 5-point operator on an s x s grid, k_cell = exp(sigma xi);
    interior faces use the harmonic mean 2 k1 k2 / (k1 + k2), a Dirichlet
    boundary face contributes 2 k_cell to the diagonal.  nnz = 5s^2 - 4s."""
    seed = rng.substream(f"{tag}/kappa/{s}")
    k = np.exp(sigma * rng.normal(seed, s * s)).reshape(s, s)  # [y, x]

    def harm(a, b):
        return 2.0 * a * b / (a + b)

    tw = np.zeros((s, s)); te = np.zeros((s, s)); ts = np.zeros((s, s)); tn = np.zeros((s, s))
    tw[:, 1:] = harm(k[:, 1:], k[:, :-1]); tw[:, 0] = 2.0 * k[:, 0]
    te[:, :-1] = harm(k[:, :-1], k[:, 1:]); te[:, -1] = 2.0 * k[:, -1]
    ts[1:, :] = harm(k[1:, :], k[:-1, :]); ts[0, :] = 2.0 * k[0, :]
    tn[:-1, :] = harm(k[:-1, :], k[1:, :]); tn[-1, :] = 2.0 * k[-1, :]
    diag = tw + te + ts + tn
    offs = [(0, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    coef = [diag, -ts, -tn, -tw, -te]
    # interior-face couplings only: boundary entries are dropped by the builder
    return _stencil_csr((1, s, s), offs, [c.reshape(1, s, s) for c in coef], f"varcoef2d_{s}")


def batch_sizes(count: int = 256, lo: int = 32, hi: int = 256, tag: str = "batch") -> np.ndarray:
    return rng.integers(rng.substream(f"{tag}/sizes/{count}"), count, lo, hi)


# ---------------------------------------------------------------------------
# right-hand sides and named workloads
# ---------------------------------------------------------------------------

def rhs(A: CSR, tag: str):
    """x* uniform on [-1, 1] from the named sub-stream, b = A x* (fp64)."""
    xs = rng.uniform(rng.substream(f"{tag}/xstar/{A.n}"), A.n, -1.0, 1.0)
    return xs, A.matvec(xs)


WORKLOADS = {
    "poisson2d_64": dict(cfg=0, desc="2D 5-point Poisson, 64x64 grid (n=4096)"),
    "poisson3d_128": dict(cfg=1, desc="3D 7-point Poisson, 128^3 grid (n=2,097,152)"),
    "convdiff_q1_100": dict(cfg=2, desc="3D Q1 convection-diffusion, 100^3 interior nodes, 27-point, Pe=50"),
    "elasticity_bonds_64": dict(cfg=3, desc="3x3-block bond elasticity, 64^3 jittered points, 26 neighbours"),
    "batch_varcoef2d_256": dict(cfg=4, desc="256 variable-coefficient 2D 5-point systems, sides 32..256"),
}


def build(name: str, scale: int | None = None) -> CSR:
    """Named workload; `scale` overrides the grid size for small test cases."""
    if name.startswith("poisson2d"):
        return poisson2d(scale or 64)
    if name.startswith("poisson3d"):
        return poisson3d(scale or 128)
    if name.startswith("convdiff"):
        return convdiff_q1(scale or 100)
    if name.startswith("elasticity"):
        return elasticity_bonds(scale or 64)
    if name.startswith("hpcg") or name.startswith("hpgmp"):
        gen = hpcg if name.startswith("hpcg") else hpgmp
        if scale:
            return gen(scale, scale, scale)
        x, y, z = (1 << int(t) for t in name.split("_")[1:4])
        return gen(x, y, z)
    raise KeyError(name)
