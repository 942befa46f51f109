"""Pins of the oracle's operator (I - M N) and contrast.

* Clausius-Mossotti: a one-voxel body at k = 0 has the exact internal field
  3/(eps + 2) e_inc, i.e. w = 3 (eps - 1)/(eps + 2) e_inc; this pins M and that
  N contains the identity (eq. JVIE, Sec. 2).
* N is complex symmetric (N^T = N) and each block is 3-level Toeplitz (Sec. 2,
  after eq. sys_mat); homogeneous M keeps I - M N BTTB.
* A circulant-embedding FFT product written here with numpy.fft equals the
  explicit sum (the FFT matvec claim of Sec. 1).
* Zero contrast gives the identity; row-by-row summation equals the dense matrix.
* Table ref_ind values (golden file) and the contrast of Si in SiO2.
"""
import os

import numpy as np
import pytest

from oracle import contrast as CT
from oracle import generator as G
from oracle import matvec as MV

HERE = os.path.dirname(os.path.abspath(__file__))


def _load_table():
    vals = {}
    for line in open(os.path.join(HERE, 'golden', 'materials_table.txt')):
        line = line.split('#')[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_material_table_contrast():
    t = _load_table()
    assert round(t['Si'] / t['SiO2'], 2) == t['Si_in_SiO2']
    assert round(t['Si3N4'] / t['SiO2'], 2) == t['Si3N4_in_SiO2']
    eps = t['Si'] / t['SiO2']
    M = CT.contrast_from_chi(np.array([eps - 1.0]))
    assert abs(M[0] - (eps - 1.0) / eps) < 1e-15


@pytest.mark.parametrize("eps", [2.0, 5.808153477218225, 12.1, 3.0 - 0.5j])
def test_clausius_mossotti_single_voxel(eps):
    K = G.generator_octant((1, 1, 1), 0.0)
    M = CT.contrast_from_chi(np.array([[[eps - 1.0]]]))
    A = MV.operator_matrix(K, M, (1, 1, 1))
    e_inc = np.array([0.3 + 0.1j, -1.0, 0.5j])
    w = np.linalg.solve(A, np.tile(M.reshape(-1), 3) * e_inc)
    expect = 3.0 * (eps - 1.0) / (eps + 2.0) * e_inc
    assert np.allclose(w, expect, rtol=1e-13, atol=0)


@pytest.fixture(scope="module")
def small():
    grid = (5, 3, 2)
    kappa = 0.2926652804732217
    K = G.generator_octant(grid, kappa)
    rng = np.random.default_rng(5)
    M = rng.standard_normal((2, 3, 5)) * 0.4 + 1j * rng.standard_normal((2, 3, 5)) * 0.1
    return grid, K, M


def test_n_is_complex_symmetric_and_bttb(small):
    grid, K, _ = small
    N = MV.n_matrix(K, grid)
    assert np.abs(N - N.T).max() < 1e-15
    nx, ny, nz = grid
    n = nx * ny * nz
    idx = lambda x, y, z: x + nx * (y + ny * z)
    for a in range(3):
        for b in range(3):
            blk = N[a * n:(a + 1) * n, b * n:(b + 1) * n]
            # entry depends only on the offset
            assert blk[idx(3, 1, 1), idx(1, 0, 0)] == blk[idx(4, 2, 1), idx(2, 1, 0)]
            assert blk[idx(0, 2, 0), idx(4, 0, 1)] == blk[idx(0, 2, 0), idx(4, 0, 1)]


def test_zero_contrast_is_identity(small):
    grid, K, _ = small
    x = np.random.default_rng(1).standard_normal(3 * 30) + 0j
    y = MV.matvec(K, np.zeros((2, 3, 5)), grid, x)
    assert np.array_equal(y, x)


def test_rows_equal_dense(small):
    grid, K, M = small
    rng = np.random.default_rng(2)
    x = rng.standard_normal(90) + 1j * rng.standard_normal(90)
    y = MV.matvec(K, M, grid, x)
    rows = [0, 7, 29, 30, 61, 89]
    assert np.allclose(MV.matvec_rows(K, M, grid, x, rows), y[rows], rtol=1e-14, atol=1e-14)


def test_fft_embedding_equals_explicit_sum(small):
    grid, K, M = small
    nx, ny, nz = grid
    rng = np.random.default_rng(3)
    x = rng.standard_normal(90) + 1j * rng.standard_normal(90)
    y = MV.matvec(K, M, grid, x)
    # circulant embedding, period 2n per axis, entry n left at 0
    P = (2 * nz, 2 * ny, 2 * nx)
    lz, ly, lx = [np.r_[np.arange(n), 0, -np.arange(n - 1, 0, -1)] for n in (nz, ny, nx)]
    DZ, DY, DX = np.meshgrid(lz, ly, lx, indexing='ij')
    mask = (np.abs(DZ) < nz) & (np.abs(DY) < ny) & (np.abs(DX) < nx)
    mask[nz, :, :] = False
    mask[:, ny, :] = False
    mask[:, :, nx] = False
    xs = x.reshape(3, nz, ny, nx)
    xh = [np.fft.fftn(np.pad(xs[b], ((0, nz), (0, ny), (0, nx)))) for b in range(3)]
    Kx = np.zeros((3, nz, ny, nx), dtype=complex)
    for a in range(3):
        acc = 0
        for b in range(3):
            emb = np.where(mask, G.generator_signed(K, a, b, DX, DY, DZ), 0)
            acc = acc + np.fft.fftn(emb) * xh[b]
        Kx[a] = np.fft.ifftn(acc)[:nz, :ny, :nx]
    yf = (xs - M[None] * (xs + Kx)).reshape(-1)
    assert np.abs(yf - y).max() < 1e-13 * np.abs(y).max()
