"""Exact pressure solves for the oracle (TEST INFRASTRUCTURE).

The paper defers the pressure-velocity coupling to its references, so the
operator is the plain reading of a second-order staggered projection:

    (A p)[j, i] = sum over the cell's faces not on a wall of
                  (p_neighbour - p[j, i]) / (rho_face * h^2),

x periodic, wall faces omitted (homogeneous Neumann), rho_face the arithmetic
mean of the two adjacent cell densities.  A has the constants as null space;
the right-hand side is made mean-free and the solution is taken mean-free.

Two independent exact solvers:
  * uniform density: FFT in x and DCT-II in y diagonalise A;
  * variable density: sparse LU (SciPy splu) with one cell pinned, then the
    mean removed.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def apply_A(p: np.ndarray, rfx: np.ndarray, rfy: np.ndarray, h: float) -> np.ndarray:
    """A p with face densities rfx (ny, nx) at x-face i (between cells i-1, i)
    and rfy (ny+1, nx) at y-face j (between cells j-1, j; rows 0, ny unused)."""
    ny, nx = p.shape
    out = np.zeros_like(p)
    # x faces, periodic: face i couples cells i-1 and i
    flux = (p - np.roll(p, 1, axis=1)) / rfx          # at face i: p[i] - p[i-1]
    out += (np.roll(flux, -1, axis=1) - flux)
    # y faces: interior faces j = 1..ny-1 couple rows j-1 and j
    fy = np.zeros((ny + 1, nx))
    fy[1:ny] = (p[1:] - p[:-1]) / rfy[1:ny]
    out += fy[1:] - fy[:-1]
    return out / (h * h)


def solve_uniform(b: np.ndarray, rho: float, h: float) -> np.ndarray:
    """Exact solve of A p = b for uniform density by FFT(x) / DCT-II(y)."""
    ny, nx = b.shape
    bh = sfft.dct(np.fft.fft(b, axis=1), type=2, axis=0, norm="ortho")
    k = np.arange(nx)
    l = np.arange(ny)
    lam = (2.0 * np.cos(2.0 * np.pi * k / nx)[None, :] - 2.0
           + 2.0 * np.cos(np.pi * l / ny)[:, None] - 2.0) / (rho * h * h)
    lam[0, 0] = 1.0
    ph = bh / lam
    ph[0, 0] = 0.0
    p = np.real(np.fft.ifft(sfft.idct(ph, type=2, axis=0, norm="ortho"), axis=1))
    return p - p.mean()


def assemble_A(rfx: np.ndarray, rfy: np.ndarray, h: float) -> sp.csr_matrix:
    """Sparse matrix of A (row-major cell index j*nx + i): every interior face
    contributes +1/(rho_f h^2) off the diagonal and -1/(rho_f h^2) to the
    diagonal of both cells it couples; wall faces contribute nothing."""
    ny, nx = rfx.shape
    n = nx * ny
    cell = np.arange(n).reshape(ny, nx)
    # x faces: face i couples (j, i-1) and (j, i), periodic
    a_c = cell.reshape(-1)
    a_w = np.roll(cell, 1, axis=1).reshape(-1)
    cx = (1.0 / rfx).reshape(-1)
    # y faces j = 1..ny-1 couple (j-1, i) and (j, i)
    b_s = cell[:-1].reshape(-1)
    b_n = cell[1:].reshape(-1)
    cy = (1.0 / rfy[1:ny]).reshape(-1)
    rows = np.concatenate([a_c, a_w, a_c, a_w, b_s, b_n, b_s, b_n])
    cols = np.concatenate([a_w, a_c, a_c, a_w, b_n, b_s, b_s, b_n])
    vals = np.concatenate([cx, cx, -cx, -cx, cy, cy, -cy, -cy])
    return sp.coo_matrix((vals / (h * h), (rows, cols)), shape=(n, n)).tocsr()


def solve_sparse(b: np.ndarray, rfx: np.ndarray, rfy: np.ndarray, h: float) -> np.ndarray:
    """Exact solve of A p = b (b mean-free) by sparse LU with p[0, 0] pinned
    to zero, then the mean removed."""
    ny, nx = b.shape
    A = assemble_A(rfx, rfy, h).tolil()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    rhs = b.reshape(-1).copy()
    rhs[0] = 0.0
    p = spla.splu(A.tocsc()).solve(rhs).reshape(ny, nx)
    return p - p.mean()


def solve(b: np.ndarray, rho_cells: np.ndarray, rfx: np.ndarray, rfy: np.ndarray,
          h: float) -> np.ndarray:
    """Exact solve; FFT/DCT when the density field is uniform, sparse LU otherwise."""
    r0 = rho_cells.flat[0]
    if np.all(rho_cells == r0):
        return solve_uniform(b, float(r0), h)
    return solve_sparse(b, rfx, rfy, h)
