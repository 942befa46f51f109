"""Solves on grids with x-lines of zero contrast, against the oracle's dense solution.

Where the contrast vanishes along a whole x-line the operator I - M N is the identity on that
line (Sec. 2, eq. discrete_form: every row there reads x_i), so the solution there is b itself.
The solver restricts its basis passes to the other lines; these tests cover the ways the skipped
lines can carry data: a right-hand side M e (zero there), a right-hand side with entries there
(the product with x then enters the first residual), a given initial guess, a preconditioner
that homogenises across lines (2-level, projected), mixed precision and no preconditioner (right-
hand sides joining a running batch: the coupler device of the serving tests).  Bars: the oracle-evaluated residual at the solve tolerance
(x 2), x equal to b on the skipped lines, and the error against the dense solution.
"""
import numpy as np
import pytest

from oracle import contrast as OCT
from oracle import generator as OG
from oracle import matvec as OM
from paper_1903_07884_amd import workloads as W

pytestmark = pytest.mark.gpu

KB = W.k_background()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _problem(grid=(40, 12, 4), delta=50e-9, cores=((2, 5), (7, 10))):
    nx, ny, nz = grid
    K = OG.generator_octant(grid, KB * delta)
    chi = W.coupler(grid, cores=cores)
    M = OCT.contrast_from_chi(chi)
    A = OM.operator_matrix(K, M, grid)
    # lines (c, z, y) of the [c][z][y][x] vectors with zero contrast along all x
    zero_yz = ~np.any(M != 0, axis=2)                                    # [nz][ny]
    skipped = np.broadcast_to(zero_yz[None, :, :, None], (3, nz, ny, nx)).reshape(-1)
    return grid, delta, K, chi, M, A, skipped


def _rhs(grid, M, skipped):
    n = 3 * int(np.prod(grid))
    e = W.random_field((3, n), 71)
    b_me = np.tile(M.reshape(-1), 3) * e[0]          # zero on the skipped lines
    b_any = e[1]                                     # entries everywhere
    b_mix = b_me + 0.3 * e[2] * skipped              # M e inside, entries on the skipped lines only
    return np.stack([b_me, b_any, b_mix])


@pytest.mark.parametrize("mode,levels,precond", [('fp64', 1, True), ('fp64', 2, True), ('fp64', 1, False),
                                                 ('mixed', 1, True)])
def test_solve_with_skipped_lines_matches_dense_solution(gpu_lib, mode, levels, precond):
    """levels = 2: the cores cover 9 of the 12 y positions, so the modal contrast of the 2-level
    circulant is silicon and its blocks couple the skipped lines to the others (projected)."""
    import torch
    grid, delta, K, chi, M, A, skipped = _problem(cores=((1, 6), (7, 11)) if levels == 2 else ((2, 5), (7, 10)))
    assert skipped.any() and not skipped.all()
    B = _rhs(grid, M, skipped)
    X_ref = np.linalg.solve(A, B.T).T
    tol = 1e-10 if mode == 'fp64' else 1e-6
    op = gpu_lib.Operator(grid, delta, KB, chi, generator=K, build_c64=(mode == 'mixed'))
    fp = gpu_lib.VIE_C128 if mode == 'fp64' else gpu_lib.VIE_C64
    pc = (gpu_lib.Preconditioner(op, levels=levels, factor_prec=fp, homog='mode' if levels == 2 else 'none')
          if precond else None)
    Bd = _dev(B)
    Xd = torch.zeros_like(Bd)
    st = gpu_lib.solve(op, pc, Bd, Xd, nrhs=3, tol=tol, mode=mode)
    X = Xd.cpu().numpy()
    for q in range(3):
        res = np.linalg.norm(B[q] - A @ X[q]) / np.linalg.norm(B[q])
        err = np.linalg.norm(X[q] - X_ref[q]) / np.linalg.norm(X_ref[q])
        print('%s levels=%d pc=%s rhs %d: iters %d, oracle residual %.2e, error %.2e'
              % (mode, levels, precond, q, st[q]['iters'], res, err))
        assert st[q]['status'] == 0 and res <= 2 * tol
        assert np.array_equal(X[q][skipped], B[q][skipped])
        assert err < (1e-7 if mode == 'fp64' else 1e-4)
    if pc is not None:
        pc.close()
    op.close()


def test_initial_guess_and_skipped_lines(gpu_lib):
    """x0 given (nonzero everywhere, also on the skipped lines): the solve replaces it by b there
    and converges to the dense solution."""
    import torch
    grid, delta, K, chi, M, A, skipped = _problem()
    B = _rhs(grid, M, skipped)[1:2]
    x_ref = np.linalg.solve(A, B[0])
    op = gpu_lib.Operator(grid, delta, KB, chi, generator=K)
    pc = gpu_lib.Preconditioner(op)
    x0 = x_ref + 0.05 * W.random_field((1, B.shape[1]), 72)
    Xd = _dev(x0)
    st = gpu_lib.solve(op, pc, _dev(B), Xd, nrhs=1, tol=1e-10, x0_given=True)[0]
    x = Xd.cpu().numpy()[0]
    res = np.linalg.norm(B[0] - A @ x) / np.linalg.norm(B[0])
    print('x0 given: iters %d, oracle residual %.2e' % (st['iters'], res))
    assert st['status'] == 0 and res <= 2e-10
    assert np.array_equal(x[skipped], B[0][skipped])
    pc.close()
    op.close()


def test_skipped_lines_equal_full_lines_solve(gpu_lib):
    """The same coupler with a contrast of 1e-30 instead of 0 on the cladding (so no line is
    skipped) gives the same iterations and solution to rounding for a right-hand side M e."""
    import torch
    grid, delta, K, chi, M, A, skipped = _problem()
    B = _rhs(grid, M, skipped)[0:1]
    chi_full = np.where(chi == 0, 1e-30, chi)
    out = []
    for c in (chi, chi_full):
        op = gpu_lib.Operator(grid, delta, KB, c, generator=K)
        pc = gpu_lib.Preconditioner(op)
        Xd = torch.zeros_like(_dev(B))
        st = gpu_lib.solve(op, pc, _dev(B), Xd, nrhs=1, tol=1e-10)[0]
        out.append((st['iters'], Xd.cpu().numpy()[0]))
        pc.close()
        op.close()
    diff = np.linalg.norm(out[0][1] - out[1][1]) / np.linalg.norm(out[1][1])
    print('skipped lines: iters %d / %d, difference %.2e' % (out[0][0], out[1][0], diff))
    assert out[0][0] == out[1][0] and diff < 1e-9


def _register_grid_problem():
    """512x16x8 (x period 1024, y period 32: the register x-line and plane passes) with two
    cores in y; a seeded synthetic generator injected so the oracle's FFT operator is exact."""
    grid = (512, 16, 8)
    K = W.synthetic_generator(grid, 81, scale=0.2)
    chi = W.coupler(grid, cores=((2, 6), (9, 13)))
    M = OCT.contrast_from_chi(chi)
    nx, ny, nz = grid
    zero_yz = ~np.any(M != 0, axis=2)
    skipped = np.broadcast_to(zero_yz[None, :, :, None], (3, nz, ny, nx)).reshape(-1)
    return grid, K, chi, M, skipped


def test_products_with_skipped_lines_match_oracle(gpu_lib):
    """Products of inputs with entries everywhere (y = x on the lines without contrast, the other
    lines by the transforms): entry by entry against the oracle's FFT operator, FP64 and complex64."""
    import torch
    grid, K, chi, M, skipped = _register_grid_problem()
    from oracle import fftref as FR
    R = 5
    x = W.random_field((R, 3 * int(np.prod(grid))), 82)
    ref = FR.FftOperator(K, M, grid).matvec(x)
    op = gpu_lib.Operator(grid, 25e-9, KB, chi, generator=K, build_c64=True)
    xd = _dev(x)
    y64 = torch.empty_like(xd)
    op.matvec(xd, y64, nrhs=R)
    x32 = xd.to(torch.complex64)
    y32 = torch.empty_like(x32)
    op.matvec(x32, y32, nrhs=R)
    op.close()
    y64, y32 = y64.cpu().numpy(), y32.cpu().numpy().astype(np.complex128)
    for q in range(R):
        e64 = np.abs(y64[q] - ref[q]).max() / np.abs(ref[q]).max()
        e32 = np.abs(y32[q] - ref[q]).max() / np.abs(ref[q]).max()
        print('rhs %d: fp64 %.2e c64 %.2e (entry-wise)' % (q, e64, e32))
        assert e64 < 1e-10 and e32 < 1e-5
        assert np.array_equal(y64[q][skipped], x[q][skipped])


@pytest.mark.parametrize("mode", ['fp64', 'mixed'])
def test_register_grid_solve_with_skipped_lines(gpu_lib, mode):
    """The step products skip the lines without contrast (input zero there): the solution's
    oracle-evaluated residual, x = b on those lines, and the same iterations and solution as the
    solve where those lines carry a contrast of 1e-30 (nothing skipped)."""
    import torch
    grid, K, chi, M, skipped = _register_grid_problem()
    from oracle import fftref as FR
    n = 3 * int(np.prod(grid))
    e = W.random_field((2, n), 83)
    B = np.stack([np.tile(M.reshape(-1), 3) * e[0], e[1]])
    tol = 1e-8 if mode == 'fp64' else 1e-6
    out = []
    for c in (chi, np.where(chi == 0, 1e-30, chi)):
        op = gpu_lib.Operator(grid, 25e-9, KB, c, generator=K, build_c64=(mode == 'mixed'))
        pc = gpu_lib.Preconditioner(op, factor_prec=gpu_lib.VIE_C128 if mode == 'fp64' else gpu_lib.VIE_C64)
        Xd = torch.zeros_like(_dev(B))
        st = gpu_lib.solve(op, pc, _dev(B), Xd, nrhs=2, tol=tol, mode=mode)
        out.append((st, Xd.cpu().numpy()))
        pc.close()
        op.close()
    (st, X), (st_full, X_full) = out
    A = FR.FftOperator(K, M, grid)
    for q in range(2):
        res = np.linalg.norm(B[q] - A.matvec(X[q])) / np.linalg.norm(B[q])
        diff = np.linalg.norm(X[q] - X_full[q]) / np.linalg.norm(X_full[q])
        print('%s rhs %d: iters %d (nothing skipped: %d), oracle residual %.2e, difference %.2e'
              % (mode, q, st[q]['iters'], st_full[q]['iters'], res, diff))
        assert st[q]['status'] == 0 and res <= 2 * tol
        assert np.array_equal(X[q][skipped], B[q][skipped])
        if q == 0 and mode == 'fp64':  # M e: the same Krylov space in both solves
            assert st[q]['iters'] == st_full[q]['iters'] and diff < 1e-9
        elif q == 0:  # complex64 products: rounding differs between the two, within its bar
            assert abs(st[q]['iters'] - st_full[q]['iters']) <= 2 and diff < 1e-4
