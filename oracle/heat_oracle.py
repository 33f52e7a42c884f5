"""FP64 CPU oracle of the heat-kernel Gibbs operator on a masked grid.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP library or its binding.

Section 4.1 (eq. heat-kernel) replaces the Gibbs kernel xi = exp(-c/gamma)
on a general domain M by L steps of implicit Euler for the heat equation up
to time gamma:

    xi~ = (Id - (gamma / L) Delta_M)^{-L},

applied by solving L sparse linear systems.  Here M is the set of cells of a
uniform cell-centred grid of [0,1]^2 (n0 x n1 cells) left free by a boolean
mask (obstacles excluded), and Delta_M is the five-point Laplacian of the
cells of M with spacing 1/n_k along axis k and no flux across the grid's
boundary or into an obstacle (a neighbour outside M contributes nothing).
Hence

    Id - (gamma/L) Delta_M = Id + nu_0 G_0 + nu_1 G_1,  nu_k = gamma n_k^2 / L,

with G_k the graph Laplacian of the axis-k neighbour pairs inside M.  The
matrix is symmetric, positive definite, and has unit row sums, so xi~ is
symmetric, entrywise non-negative and conserves mass.  Cells outside M carry
no mass: xi~ is zero on their rows and columns.

Each application runs L solves with one sparse LU factorisation computed
once (the paper pre-factors by a sparse Cholesky; any exact sparse solve is
the same operator).  A one-dimensional grid is n0 = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def heat_nu(shape, gamma: float, L: int):
    """nu_k = gamma n_k^2 / L: the weight of one axis-k neighbour pair in
    Id - (gamma/L) Delta_M with spacing 1/n_k."""
    return [gamma * float(n) ** 2 / L for n in shape]


def heat_system(mask: np.ndarray, gamma: float, L: int):
    """(A, idx): A = Id + sum_k nu_k G_k (sparse CSC, over the cells of M in
    row-major order) and idx, the flat grid index of each of those cells."""
    mask = np.asarray(mask, bool)
    n0, n1 = mask.shape
    nu0, nu1 = heat_nu(mask.shape, gamma, L)
    idx = np.flatnonzero(mask.ravel())
    pos = -np.ones(mask.size, dtype=np.int64)
    pos[idx] = np.arange(len(idx))
    flat = np.arange(mask.size).reshape(mask.shape)
    rows, cols, vals = [], [], []
    for a, b, nu in ((flat[:-1, :], flat[1:, :], nu0), (flat[:, :-1], flat[:, 1:], nu1)):
        a, b = a.ravel(), b.ravel()
        both = mask.ravel()[a] & mask.ravel()[b]
        pa, pb = pos[a[both]], pos[b[both]]
        # each pair adds nu (e_a - e_b)(e_a - e_b)^T
        rows += [pa, pb, pa, pb]
        cols += [pa, pb, pb, pa]
        vals += [np.full(len(pa), nu), np.full(len(pa), nu), np.full(len(pa), -nu), np.full(len(pa), -nu)]
    m = len(idx)
    G = sp.coo_matrix((np.concatenate(vals) if vals else np.zeros(0),
                       (np.concatenate(rows) if rows else np.zeros(0, int),
                        np.concatenate(cols) if cols else np.zeros(0, int))), shape=(m, m))
    A = (sp.identity(m, format="csc") + G.tocsc()).tocsc()
    return A, idx


class HeatKernel:
    """xi~ x for fields x of the mask's shape (Section 4.1, eq. heat-kernel).

    Values of x outside M are ignored; the result is zero there.  xi~ is
    symmetric, so the same call serves xi~^T."""

    def __init__(self, mask: np.ndarray, gamma: float, L: int = 10):
        self.mask = np.asarray(mask, bool)
        self.shape = self.mask.shape
        self.gamma = float(gamma)
        self.L = int(L)
        A, self.idx = heat_system(self.mask, gamma, L)
        self.lu = spla.splu(A) if len(self.idx) else None

    def __call__(self, x: np.ndarray, transpose: bool = False) -> np.ndarray:
        y = np.zeros(self.mask.size)
        if self.lu is None:
            return y.reshape(self.shape)
        v = np.asarray(x, np.float64).reshape(-1)[self.idx]
        for _ in range(self.L):
            v = self.lu.solve(v)
        y[self.idx] = v
        return y.reshape(self.shape)

    def dense(self) -> np.ndarray:
        """The N x N matrix of xi~ over all grid cells (small grids only)."""
        N = self.mask.size
        out = np.zeros((N, N))
        for j in self.idx:
            e = np.zeros(N)
            e[j] = 1.0
            out[:, j] = self(e.reshape(self.shape)).ravel()
        return out
