"""Pins of the oracle GMRES (minimal-residual Krylov solver, Sec. 1).

* Without restart and with k = dim steps it returns the direct solution.
* After k steps the iterate is the least-squares minimiser of ||b - A x|| over
  the Krylov space K_k(A M, b) (explicit power basis, small k).
* The residual estimate is non-increasing within a cycle; right
  preconditioning with the exact inverse converges in one step.
* MGS and CGS2 orthogonalisation give the same iterates.
"""
import numpy as np

from oracle import gmres as GM


def _problem(n=30, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3 + 1j * rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_full_dimension_equals_direct_solve():
    A, b = _problem()
    x, info = GM.gmres(lambda v: A @ v, b, tol=1e-15, restart=30, maxit=30)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12 * np.linalg.cond(A)


def test_minimal_residual_property():
    A, b = _problem(seed=1)
    Mi = np.diag(1.0 / (1.0 + np.arange(30) * 0.01))
    for k in (1, 3, 6):
        x, info = GM.gmres(lambda v: A @ v, b, M=lambda v: Mi @ v, tol=0.0, restart=k, maxit=k)
        AM = A @ Mi
        Kr = np.stack([np.linalg.matrix_power(AM, i) @ b for i in range(k)], axis=1)
        u = np.linalg.lstsq(AM @ Kr, b, rcond=None)[0]
        xs = Mi @ (Kr @ u)
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10


def test_residual_monotone_and_exact_preconditioner():
    A, b = _problem(seed=2)
    _, info = GM.gmres(lambda v: A @ v, b, tol=1e-10, restart=50)
    h = info['history']
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
    Ai = np.linalg.inv(A)
    x, info = GM.gmres(lambda v: A @ v, b, M=lambda v: Ai @ v, tol=1e-12)
    assert info['iters'] == 1 and info['converged']


def test_mgs_equals_cgs2_and_restart_converges():
    A, b = _problem(seed=3)
    x1, i1 = GM.gmres(lambda v: A @ v, b, tol=1e-10, restart=5, ortho='mgs')
    x2, i2 = GM.gmres(lambda v: A @ v, b, tol=1e-10, restart=5, ortho='cgs2')
    assert i1['iters'] == i2['iters'] and i1['converged']
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-12
    assert np.linalg.norm(b - A @ x1) / np.linalg.norm(b) <= 1e-10
