"""Pins of the oracle's FFT reference operator (oracle.fftref) against the explicit sums.

The FFT form is a second, independent evaluation of the same definition
(Sec. 2, eq. discrete_form with N = I + K): it must reproduce the dense matrix
of ``matvec`` on small grids (odd, even and unit extents), sampled explicit row
sums of the 64x8x4 grid, zero contrast = identity, and it must not depend on
the value placed at the unused wrap index of the embedding.
"""
import numpy as np
import pytest

from oracle import contrast as OCT
from oracle import fftref as FR
from oracle import generator as OG
from oracle import matvec as OM
from paper_1903_07884_amd import workloads as W


def _rand_contrast(grid, seed):
    nx, ny, nz = grid
    rng = np.random.default_rng(seed)
    return OCT.contrast_from_chi(2.0 + rng.standard_normal((nz, ny, nx)) + 0.3j * rng.standard_normal((nz, ny, nx)))


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 2), (3, 2, 2), (5, 3, 2), (4, 1, 3), (8, 8, 8)])
def test_fft_operator_equals_dense(grid):
    kappa = W.k_background() * 50e-9
    K = OG.generator_octant(grid, kappa)
    M = _rand_contrast(grid, 1)
    n = 3 * int(np.prod(grid))
    x = W.random_field((2, n), 5)
    ref = OM.matvec(K, M, grid, x)
    y = FR.FftOperator(K, M, grid).matvec(x)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


def test_fft_operator_sampled_rows_of_the_64x8x4_guide():
    """A synthetic decaying generator on the 64x8x4 grid (every offset, so the circulant's
    long-range entries are exercised): sampled rows by explicit summation."""
    grid = (64, 8, 4)
    K = W.synthetic_generator(grid, 3)
    M = OCT.contrast_from_chi(W.waveguide(grid))
    n = 3 * int(np.prod(grid))
    x = W.random_field((n,), 6)
    y = FR.FftOperator(K, M, grid).matvec(x)
    rows = np.random.default_rng(2).choice(n, 40, replace=False)
    ref = OM.matvec_rows(K, M, grid, x, rows)
    assert np.abs(y[rows] - ref).max() < 1e-13 * np.abs(ref).max()


def test_zero_contrast_is_identity_and_residual():
    grid = (6, 3, 2)
    K = W.synthetic_generator(grid, 4)
    M = np.zeros((2, 3, 6), dtype=complex)
    op = FR.FftOperator(K, M, grid)
    x = W.random_field((op.n,), 7)
    assert np.array_equal(op.matvec(x), x)
    assert op.relres(x, x)[0] == 0.0


def test_synthetic_generator_has_the_operator_parities():
    """Off-diagonal components vanish at zero offset along both of their odd axes (Sec. 2):
    the octant table of the synthetic generator must respect that, as the oracle's does."""
    grid = (9, 4, 3)
    K = W.synthetic_generator(grid, 8)
    ref = OG.generator_octant((3, 2, 2), W.k_background() * 25e-9)
    for c, (a, b) in enumerate(OG.COMPONENTS):
        if a == b:
            continue
        for axis in (a, b):
            sl = [slice(None)] * 3
            sl[2 - axis] = 0                      # table axes are [z, y, x]
            assert np.all(K[c][tuple(sl)] == 0)
            assert np.all(ref[c][tuple(sl)] == 0)
