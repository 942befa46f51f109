"""Field inside a homogeneous dielectric sphere in a plane wave: the Mie series.

Test infrastructure, written from the textbook series (vector spherical harmonics and the
internal coefficients c_n, d_n of Bohren & Huffman, ch. 4) in the physics time convention
exp(-i w t), incident field x^ exp(+i k z).  For a real relative permittivity the complex
conjugate is the solution in the engineering convention exp(+j w t) with incident field
x^ exp(-j k z), the convention of the volume integral equation (g = exp(-j k R) / (4 pi R)).

Checks of its own (tests/test_oracle_mie.py): with relative index m = 1 the series must
reproduce the incident plane wave (c_n = d_n = 1), and for a small sphere (k a -> 0) the
uniform electrostatic interior field 3 / (eps + 2).
"""
import numpy as np
from scipy.special import spherical_jn, spherical_yn


def internal_coefficients(m, x, nmax):
    """c_n, d_n, n = 1..nmax, for relative index m and size parameter x = k a (mu = mu_1)."""
    n = np.arange(1, nmax + 1)
    mx = m * x
    jx, djx = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    yx, dyx = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    hx, dhx = jx + 1j * yx, djx + 1j * dyx
    jm, djm = spherical_jn(n, mx), spherical_jn(n, mx, derivative=True)
    xj_d = jx + x * djx          # [x j_n(x)]'
    xh_d = hx + x * dhx          # [x h_n(x)]'
    mj_d = jm + mx * djm         # [m x j_n(m x)]'
    c = (jx * xh_d - hx * xj_d) / (jm * xh_d - hx * mj_d)
    d = (m * jx * xh_d - m * hx * xj_d) / (m * m * jm * xh_d - hx * mj_d)
    return c, d


def _angular(mu, nmax):
    """pi_n(mu), tau_n(mu) for n = 1..nmax (upward recurrences)."""
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def internal_field(points, eps, ka, radius=1.0, nmax=None):
    """E inside the sphere at Cartesian points [P, 3] (sphere at the origin, |r| < radius > 0),
    unit incident amplitude, engineering convention (incident x^ exp(-j k z), k = ka / radius).
    Returns [P, 3] complex Cartesian components."""
    m = np.sqrt(complex(eps))
    k = ka / radius
    if nmax is None:
        nmax = int(abs(m) * ka + 4 * (abs(m) * ka) ** (1 / 3) + 8)
    c, d = internal_coefficients(m, ka, nmax)
    p = np.asarray(points, dtype=float)
    r = np.linalg.norm(p, axis=1)
    th = np.arccos(np.clip(p[:, 2] / r, -1.0, 1.0))
    ph = np.arctan2(p[:, 1], p[:, 0])
    rho = m * k * r
    pi, tau = _angular(np.cos(th), nmax)
    E_r = np.zeros(len(r), complex)
    E_t = np.zeros(len(r), complex)
    E_p = np.zeros(len(r), complex)
    cp, sp, st = np.cos(ph), np.sin(ph), np.sin(th)
    for i in range(nmax):
        n = i + 1
        En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
        z = spherical_jn(n, rho)
        dz = z + rho * spherical_jn(n, rho, derivative=True)   # [rho z_n(rho)]'
        # M_o1n and N_e1n with z_n = j_n (regular inside)
        M_t, M_p = cp * pi[i] * z, -sp * tau[i] * z
        N_r = cp * n * (n + 1) * st * pi[i] * z / rho
        N_t, N_p = cp * tau[i] * dz / rho, -sp * pi[i] * dz / rho
        E_r += En * (-1j * d[i] * N_r)
        E_t += En * (c[i] * M_t - 1j * d[i] * N_t)
        E_p += En * (c[i] * M_p - 1j * d[i] * N_p)
    ct = np.cos(th)
    Ex = E_r * st * cp + E_t * ct * cp - E_p * sp
    Ey = E_r * st * sp + E_t * ct * sp + E_p * cp
    Ez = E_r * ct - E_t * st
    return np.conj(np.stack([Ex, Ey, Ez], axis=1))
