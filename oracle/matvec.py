"""Operator (I - M N) by explicit summation (oracle; test infrastructure only).

Sec. 2, eq. discrete_form / sys_mat: unknowns w = [w^x; w^y; w^z], each block
ordered over voxels with x fastest, then y, then z; M is diagonal with the
contrast at voxel centres (isotropic, so M^x = M^y = M^z), and
N^{ab}_{ij} = delta_ab delta_ij + K^{ab}(i - j) with K from ``generator``.

    y_i^a = x_i^a - M_i * sum_b sum_j N^{ab}(i - j) x_j^b

No FFT is used anywhere here: ``operator_matrix`` forms the dense 3N x 3N
matrix (small grids), ``matvec_rows`` sums selected rows one by one (any grid).
"""
import numpy as np

from .generator import generator_signed


def _coords(grid):
    nx, ny, nz = grid
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing='ij')
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def n_matrix(Koct, grid):
    """Dense N = I + K (3N x 3N) from the octant generator."""
    nx, ny, nz = grid
    n = nx * ny * nz
    x, y, z = _coords(grid)
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dz = z[:, None] - z[None, :]
    N = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            N[a * n:(a + 1) * n, b * n:(b + 1) * n] = generator_signed(Koct, a, b, dx, dy, dz)
    N += np.eye(3 * n)
    return N


def operator_matrix(Koct, M, grid):
    """Dense A = I - M N (3N x 3N).  ``M`` is [nz, ny, nx] complex."""
    n = int(np.prod(grid))
    m = np.tile(np.asarray(M, dtype=np.complex128).reshape(-1), 3)
    return np.eye(3 * n, dtype=np.complex128) - m[:, None] * n_matrix(Koct, grid)


def matvec(Koct, M, grid, x):
    """y = (I - M N) x for x of length 3N (or [R, 3N]) via the dense matrix."""
    A = operator_matrix(Koct, M, grid)
    x = np.asarray(x, dtype=np.complex128)
    return (A @ x.T).T


def matvec_rows(Koct, M, grid, x, rows):
    """Selected entries y[rows] of y = (I - M N) x, each by explicit summation."""
    nx, ny, nz = grid
    n = nx * ny * nz
    xs, ys, zs = _coords(grid)
    x = np.asarray(x, dtype=np.complex128).reshape(3, n)
    Mf = np.asarray(M, dtype=np.complex128).reshape(-1)
    out = np.zeros(len(rows), dtype=np.complex128)
    for r, row in enumerate(rows):
        a, i = divmod(int(row), n)
        dx, dy, dz = xs[i] - xs, ys[i] - ys, zs[i] - zs
        acc = x[a, i]  # identity part of N
        for b in range(3):
            acc = acc + np.sum(generator_signed(Koct, a, b, dx, dy, dz) * x[b])
        out[r] = x[a, i] - Mf[i] * acc
    return out
