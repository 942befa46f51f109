"""Operator (I - M N) by FFTs of the circulant embedding, for full-size grids
(oracle; test infrastructure only).

Sec. 1 states that products with the three-level Toeplitz matrix cost
O(n log n) "via the FFT"; the embedding is not spelled out there.  This module
writes out the plain definition: each of the nine Toeplitz blocks K^{ab} (six
unique, Sec. 2 after eq. sys_mat) is a sequence over signed offsets
d in (-n, n) per axis; placed on a periodic grid of period 2n per axis (offset
d at d mod 2n, the entry at n left zero) it defines a circulant whose product
with the zero-padded vector, cropped back to the grid, is exactly the Toeplitz
product (a linear convolution computed as a cyclic one of at least twice the
length).  The cyclic convolution is evaluated by a library FFT (scipy.fft):

    (K x)^a = crop( IFFT( sum_b FFT(E^{ab}) . FFT(pad(x^b)) ) ),
    y = x - M (x + K x)                                 (eq. discrete_form, N = I + K)

This is the CPU reference for grids where the dense matrix or the explicit
row sums of ``matvec`` are too slow (hundreds of thousands of voxels).  It is
pinned to ``matvec`` (explicit sums) on small grids and on sampled rows of
the 64x8x4 grid.  Nothing here is shared with the device path: the period
(2n, not the device's smallest smooth length), the layout and the FFT are the
oracle's own.
"""
import os

import numpy as np
import scipy.fft

from .generator import COMPONENTS, component_index, generator_signed


def _workers():
    return max(1, len(os.sched_getaffinity(0)))


def _signed_offsets(n):
    """Signed offset held at each index of a period-2n axis: 0..n-1, (n: none), -(n-1)..-1."""
    return np.r_[np.arange(n), 0, -np.arange(n - 1, 0, -1)]


def embedded_transforms(Koct, grid):
    """FFTs of the six embedded generator blocks: array [6, 2nz, 2ny, 2nx] complex128,
    components ordered as in ``generator.COMPONENTS``."""
    nx, ny, nz = grid
    lz, ly, lx = (_signed_offsets(n) for n in (nz, ny, nx))
    valid = [np.ones(2 * n, dtype=bool) for n in (nz, ny, nx)]
    for v, n in zip(valid, (nz, ny, nx)):
        v[n] = False                                    # the wrap entry at index n stays zero
    mask = valid[0][:, None, None] & valid[1][None, :, None] & valid[2][None, None, :]
    DZ, DY, DX = np.meshgrid(lz, ly, lx, indexing='ij')
    out = np.empty((6, 2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
    for c, (a, b) in enumerate(COMPONENTS):
        emb = np.where(mask, generator_signed(Koct, a, b, DX, DY, DZ), 0.0)
        out[c] = scipy.fft.fftn(emb, workers=_workers())
    return out


class FftOperator:
    """y = (I - M N) x on a full-size grid, from the octant generator and the contrast."""

    def __init__(self, Koct, M, grid):
        self.grid = tuple(int(v) for v in grid)
        nx, ny, nz = self.grid
        self.M = np.asarray(M, dtype=np.complex128).reshape(nz, ny, nx)
        self.Eh = embedded_transforms(Koct, self.grid)

    @property
    def n(self):
        nx, ny, nz = self.grid
        return 3 * nx * ny * nz

    def apply_K(self, x):
        """K x for one vector x of length 3N ([3][nz][ny][nx], x fastest)."""
        nx, ny, nz = self.grid
        w = _workers()
        xs = np.asarray(x, dtype=np.complex128).reshape(3, nz, ny, nx)
        xh = [scipy.fft.fftn(xs[b], s=(2 * nz, 2 * ny, 2 * nx), workers=w) for b in range(3)]
        out = np.empty((3, nz, ny, nx), dtype=np.complex128)
        for a in range(3):
            acc = self.Eh[component_index(a, 0)] * xh[0]
            acc += self.Eh[component_index(a, 1)] * xh[1]
            acc += self.Eh[component_index(a, 2)] * xh[2]
            out[a] = scipy.fft.ifftn(acc, workers=w)[:nz, :ny, :nx]
        return out.reshape(-1)

    def matvec(self, x):
        """(I - M N) x = x - M (x + K x) for x of length 3N or [R, 3N]."""
        x = np.asarray(x, dtype=np.complex128)
        if x.ndim == 2:
            return np.stack([self.matvec(v) for v in x])
        m = np.tile(self.M.reshape(-1), 3)
        return x - m * (x + self.apply_K(x))

    def residual(self, x, b):
        """b - (I - M N) x (same shapes as ``matvec``)."""
        return np.asarray(b, dtype=np.complex128) - self.matvec(x)

    def relres(self, x, b):
        """||b - A x|| / ||b|| per right-hand side (x, b of length 3N or [R, 3N])."""
        x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
        b = np.atleast_2d(np.asarray(b, dtype=np.complex128))
        return np.array([np.linalg.norm(self.residual(x[i], b[i])) / np.linalg.norm(b[i])
                         for i in range(x.shape[0])])
