"""Restarted right-preconditioned GMRES (oracle; test infrastructure only).

The paper solves the discrete JVIE with GMRES (Sec. 1; tolerance 1e-4 in
Sec. 3) and does not state the restart length, the preconditioning side, the
starting guess or the orthogonalisation.  Readings: restart 50, right
preconditioning (so the residual that is monitored is the true residual of
A x = b), x0 = 0, 2-norm relative to ||b||, modified Gram-Schmidt Arnoldi,
complex Givens rotations (c real, s complex).  A cycle ends when the residual
estimate reaches the tolerance, on happy breakdown (h_{j+1,j} <= 1e-14 ||w||)
or after ``restart`` steps; the true residual is then recomputed and decides
whether to stop.  The iteration count is the number of Arnoldi steps summed
over all cycles.
"""
import numpy as np


def _givens(a, b):
    """(c, s, r) with [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    rho = np.hypot(abs(a), abs(b))
    phase = a / abs(a)
    return abs(a) / rho, phase * np.conj(b) / rho, phase * rho


def gmres(A, b, M=None, tol=1e-6, restart=50, maxit=5000, x0=None, ortho='mgs',
          history=False):
    """Solve A x = b.  ``A`` and ``M`` are callables (vector -> vector).

    M is applied on the right: A M u = b, x = M u.  Returns
    (x, info) with info = dict(iters, restarts, relres (true), converged, history).
    """
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    prec = (lambda v: v) if M is None else M
    if nb == 0:
        return np.zeros_like(b), dict(iters=0, restarts=0, relres=0.0, converged=True, history=[])
    iters, cycles, hist = 0, 0, []
    r = b - A(x)
    beta = np.linalg.norm(r)
    while True:
        if beta / nb <= tol:
            return x, dict(iters=iters, restarts=cycles, relres=beta / nb, converged=True,
                           history=hist)
        if iters >= maxit:
            return x, dict(iters=iters, restarts=cycles, relres=beta / nb, converged=False,
                           history=hist)
        V = np.zeros((restart + 1, b.size), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        j = 0
        while j < restart and iters < maxit:
            w = A(prec(V[j]))
            nw = np.linalg.norm(w)
            if ortho == 'mgs':
                for i in range(j + 1):
                    H[i, j] = np.vdot(V[i], w)
                    w = w - H[i, j] * V[i]
            else:  # classical Gram-Schmidt applied twice
                h = V[:j + 1].conj() @ w
                w = w - V[:j + 1].T @ h
                h2 = V[:j + 1].conj() @ w
                w = w - V[:j + 1].T @ h2
                H[:j + 1, j] = h + h2
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j].real <= 1e-14 * nw
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            cs[j], sn[j], H[j, j] = _givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j += 1
            hist.append(abs(g[j]) / nb)
            if abs(g[j]) / nb <= tol or breakdown:
                break
        # least squares: upper-triangular back substitution
        y = np.zeros(j, dtype=np.complex128)
        for i in range(j - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j] @ y[i + 1:j]) / H[i, i]
        x = x + prec(V[:j].T @ y)
        cycles += 1
        r = b - A(x)
        beta = np.linalg.norm(r)
