"""Operator products on the cross-sections the register-FFT plane pass is built for.

Cross-sections of the serving catalogue and the workloads (y periods 15, 32, 48, 64 and 96 with
8 layers; 15 and 32 with 4 layers), several right-hand sides, FP64 and complex64, checked entry
by entry against the oracle: the explicit sums on small grids, the oracle's FFT reference
operator (pinned to the explicit sums) on the 1024x48x8 coupler grid, where 13 right-hand sides
are grouped several to a workgroup with a ragged last group.  Bars: FP64 1e-10 and complex64
1e-5 of the largest entry, per entry.
"""
import numpy as np
import pytest

from oracle import contrast as OCT
from oracle import fftref as FR
from oracle import generator as OG
from oracle import matvec as OM
from paper_1903_07884_amd import workloads as W

pytestmark = pytest.mark.gpu

KB = W.k_background()


def _entrywise(y, ref):
    """Largest entry error relative to the largest reference entry, per right-hand side."""
    y, ref = np.atleast_2d(y), np.atleast_2d(ref)
    return max(np.abs(y[i] - ref[i]).max() / np.abs(ref[i]).max() for i in range(ref.shape[0]))


def _products(gpu_lib, op, x, nrhs):
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.empty_like(xd)
    op.matvec(xd, yd, nrhs=nrhs)
    x32 = xd.to(torch.complex64)
    y32 = torch.empty_like(x32)
    op.matvec(x32, y32, nrhs=nrhs)
    return yd.cpu().numpy(), y32.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("grid", [(6, 48, 8), (5, 32, 8), (7, 24, 8), (9, 16, 8), (10, 8, 8), (12, 16, 4),
                                  (11, 8, 4)])
def test_register_plane_pass_matches_explicit_sum(gpu_lib, grid):
    delta = 25e-9
    K = OG.generator_octant(grid, KB * delta)
    rng = np.random.default_rng(sum(grid))
    nx, ny, nz = grid
    chi = 3.0 + rng.standard_normal((nz, ny, nx)) + 0.2j * rng.standard_normal((nz, ny, nx))
    M = OCT.contrast_from_chi(chi)
    n = 3 * nx * ny * nz
    x = W.random_field((3, n), 31)
    ref = OM.matvec(K, M, grid, x)
    op = gpu_lib.Operator(grid, delta, KB, chi, generator=K, build_c64=True)
    y64, y32 = _products(gpu_lib, op, x, 3)
    op.close()
    e64, e32 = _entrywise(y64, ref), _entrywise(y32, ref)
    print('plane pass', grid, 'fp64 %.2e c64 %.2e (entry-wise)' % (e64, e32))
    assert e64 < 1e-10 and e32 < 1e-5


@pytest.mark.parametrize("grid", [(6, 48, 8), (5, 32, 8), (7, 24, 8), (12, 16, 4)])
def test_register_plane_pass_in_pairs_matches_explicit_sum(gpu_lib, grid):
    """Three right-hand sides forced two to a workgroup (the plane pass then runs two planes side
    by side where the pair fits the register file): a full pair and a lone last plane."""
    delta = 25e-9
    K = OG.generator_octant(grid, KB * delta)
    rng = np.random.default_rng(sum(grid) + 1)
    nx, ny, nz = grid
    chi = 3.0 + rng.standard_normal((nz, ny, nx)) + 0.2j * rng.standard_normal((nz, ny, nx))
    M = OCT.contrast_from_chi(chi)
    x = W.random_field((3, 3 * nx * ny * nz), 35)
    ref = OM.matvec(K, M, grid, x)
    keys = []
    try:
        gpu_lib.autotune(True)
        op = gpu_lib.Operator(grid, delta, KB, chi, generator=K, build_c64=True)
        _products(gpu_lib, op, x, 3)  # tunes both precisions
        keys = [k for k in gpu_lib.autotune_entries() if k.startswith('matvec ') and 'grid=%dx%dx%d nrhs=3 ' % grid in k]
        assert len(keys) == 2, gpu_lib.autotune_entries()
        for key in keys:
            gpu_lib.autotune_set(key, [2, 0])
        y64, y32 = _products(gpu_lib, op, x, 3)
        op.close()
    finally:
        for key in keys:
            gpu_lib.autotune_set(key, [])
        gpu_lib.autotune(False)
    e64, e32 = _entrywise(y64, ref), _entrywise(y32, ref)
    print('plane pass in pairs', grid, 'fp64 %.2e c64 %.2e (entry-wise)' % (e64, e32))
    assert e64 < 1e-10 and e32 < 1e-5


def test_register_plane_pass_grouped_rhs_against_fft_reference(gpu_lib):
    """1024x48x8 (the coupler grid) with 13 right-hand sides: several per plane-pass workgroup
    and a ragged last group; a seeded synthetic generator is injected so the oracle holds the
    operator exactly."""
    grid = (1024, 48, 8)
    nx, ny, nz = grid
    K = W.synthetic_generator(grid, 33, scale=0.2)
    chi = W.coupler(grid)
    M = OCT.contrast_from_chi(chi)
    R = 13
    x = W.random_field((R, 3 * nx * ny * nz), 34)
    op = gpu_lib.Operator(grid, 25e-9, KB, chi, generator=K, build_c64=True)
    y64, y32 = _products(gpu_lib, op, x, R)
    op.close()
    ref = FR.FftOperator(K, M, grid).matvec(x)
    e64, e32 = _entrywise(y64, ref), _entrywise(y32, ref)
    print('1024x48x8, 13 RHS: fp64 %.2e c64 %.2e (entry-wise)' % (e64, e32))
    assert e64 < 1e-10 and e32 < 1e-5


@pytest.mark.parametrize("grid", [(8192, 4, 2), (8192, 16, 8), (6000, 8, 4)])
def test_long_x_lines_four_step_against_fft_reference(gpu_lib, grid):
    """x periods beyond one workgroup's LDS in FP64 (16384 and 12000 = 2^5 3 5^3): the four-step
    line transform (columns, twiddle, rows; frequencies left in the transposed order the plane
    pass reads) in the kernel transform and in both x passes of the product, FP64 and complex64,
    entry by entry against the oracle's FFT reference operator with a seeded synthetic generator."""
    nx, ny, nz = grid
    K = W.synthetic_generator(grid, 35, scale=0.2)
    rng = np.random.default_rng(36)
    chi = 2.0 + rng.standard_normal((nz, ny, nx)) + 0.2j * rng.standard_normal((nz, ny, nx))
    M = OCT.contrast_from_chi(chi)
    R = 2
    x = W.random_field((R, 3 * nx * ny * nz), 37)
    op = gpu_lib.Operator(grid, 25e-9, KB, chi, generator=K, build_c64=True)
    y64, y32 = _products(gpu_lib, op, x, R)
    op.close()
    ref = FR.FftOperator(K, M, grid).matvec(x)
    e64, e32 = _entrywise(y64, ref), _entrywise(y32, ref)
    print('long lines', grid, 'fp64 %.2e c64 %.2e (entry-wise)' % (e64, e32))
    assert e64 < 1e-10 and e32 < 1e-5


def test_long_x_lines_solve_against_fft_reference(gpu_lib):
    """A preconditioned FP64 solve on an 8192x8x4 guide (x period 16384: the four-step product;
    the 8192-point box transform of the preconditioner fits one workgroup), its residual
    evaluated by the oracle's FFT reference operator."""
    import torch
    grid = (8192, 8, 4)
    nx, ny, nz = grid
    K = W.synthetic_generator(grid, 38, scale=0.2)
    chi = W.waveguide(grid)
    M = OCT.contrast_from_chi(chi)
    e = W.random_field((1, 3 * nx * ny * nz), 39)
    b = np.tile(M.reshape(-1), 3)[None] * e
    op = gpu_lib.Operator(grid, 25e-9, KB, chi, generator=K)
    pc = gpu_lib.Preconditioner(op)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    st = gpu_lib.solve(op, pc, bd, xd, nrhs=1, tol=1e-10)
    res = FR.FftOperator(K, M, grid).relres(xd.cpu().numpy(), b)
    print('8192x8x4 solve: iters %d, gpu relres %.2e, oracle-evaluated %.2e' % (st[0]['iters'], st[0]['relres'], res[0]))
    assert st[0]['status'] == 0 and res[0] <= 1e-10 * 1.01
