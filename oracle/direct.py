"""Sparse-matrix view of the discrete problem (test infrastructure only).

The discrete result the multigrid solver approaches is the unique solution
phi_h of  (A phi)_c = f_c  at free nodes c,  phi_d = g_d  at Dirichlet nodes
(Section 3, eq. 19).  On grids small enough this module assembles A from a
9-point stencil (the layout of ``tomg_oracle.h``) as a SciPy sparse matrix
and solves it directly; that direct solution is the reference answer the
iterative solvers are compared with.  The transfer operators are assembled
here as matrices too, so that the oracle's stencil-form Galerkin product can
be checked against P^T A P computed by SciPy."""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_OFFS = [(di, dj) for dj in (-1, 0, 1) for di in (-1, 0, 1)]  # plane k = (dj+1)*3+(di+1)


def assemble_full(st):
    """All nx*ny rows of the stencil as an (n x n) CSR matrix (row c couples
    node c to its 9 neighbours; neighbours outside the grid are dropped)."""
    _, ny, nx = st.shape
    n = nx * ny
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols, vals = [], [], []
    for k, (di, dj) in enumerate(_OFFS):
        ii, jj = I + di, J + dj
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        rows.append((J * nx + I)[ok])
        cols.append((jj * nx + ii)[ok])
        vals.append(st[k][ok])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A


def split(st, dirs):
    """(A_ff, A_fd, free_idx, dir_idx): the rows of the free nodes, split
    into the columns of free and of Dirichlet nodes."""
    A = assemble_full(st)
    d = dirs.ravel().astype(bool)
    free = np.flatnonzero(~d)
    dd = np.flatnonzero(d)
    Af = A[free]
    return Af[:, free].tocsc(), Af[:, dd].tocsc(), free, dd


def direct_solve(st, dirs, f, phi_dir):
    """phi_h with phi = phi_dir on Dirichlet nodes, by a sparse LU solve."""
    Aff, Afd, free, dd = split(st, dirs)
    g = phi_dir.ravel()[dd]
    rhs = f.ravel()[free] - Afd @ g
    x = spla.spsolve(Aff, rhs)
    out = phi_dir.ravel().copy()
    out[free] = x
    return out.reshape(phi_dir.shape)


def dense_solve(st, dirs, f, phi_dir):
    """Same as ``direct_solve`` with a dense numpy solve (tiny grids)."""
    Aff, Afd, free, dd = split(st, dirs)
    g = phi_dir.ravel()[dd]
    rhs = f.ravel()[free] - Afd @ g
    x = np.linalg.solve(Aff.toarray(), rhs)
    out = phi_dir.ravel().copy()
    out[free] = x
    return out.reshape(phi_dir.shape)


def bilinear_P(nxc, nyc, nxf, nyf):
    """Bilinear prolongation as an (nf x nc) matrix over all nodes."""
    rows, cols, vals = [], [], []
    for J in range(nyc):
        for I in range(nxc):
            for b in (-1, 0, 1):
                for a in (-1, 0, 1):
                    i, j = 2 * I + a, 2 * J + b
                    if 0 <= i < nxf and 0 <= j < nyf:
                        rows.append(j * nxf + i)
                        cols.append(J * nxc + I)
                        vals.append((1.0 if a == 0 else 0.5) * (1.0 if b == 0 else 0.5))
    return sp.csr_matrix((vals, (rows, cols)), shape=(nxf * nyf, nxc * nyc))


def linear_P_1d(nf, halved):
    """One axis of a prolongation: linear interpolation from the (nf-1)/2+1
    coarse nodes of a halved axis (coarse node K at fine node 2K), or the
    identity for an axis that keeps every node."""
    if not halved:
        return sp.identity(nf, format="csr")
    nc = (nf - 1) // 2 + 1
    M = sp.lil_matrix((nf, nc))
    for K in range(nc):
        M[2 * K, K] = 1.0
        if 2 * K - 1 >= 0:
            M[2 * K - 1, K] = 0.5
        if 2 * K + 1 < nf:
            M[2 * K + 1, K] = 0.5
    return M.tocsr()


def tensor_P(nxf, nyf, sx, sy):
    """Prolongation with per-axis strides (2 halved, 1 kept) as the
    Kronecker product of the axis matrices (x fastest in the node order)."""
    return sp.kron(linear_P_1d(nyf, sy == 2), linear_P_1d(nxf, sx == 2), format="csr")


def five_point_laplacian(n, h):
    """Textbook 5-point Laplacian on the (n-2)^2 interior nodes of an n x n
    grid (x fastest), built as kron(I, T) + kron(T, I) with
    T = tridiag(1, -2, 1)/h^2."""
    m = n - 2
    T = sp.diags([np.ones(m - 1), -2.0 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) / (h * h)
    I = sp.identity(m)
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()
