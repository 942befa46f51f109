"""Pins of the oracle's Galerkin generator against results it does not compute itself.

* Static self term: the voxel-averaged depolarisation of a cube is 1/3 per
  axis (trace 1, equal by symmetry), so K^{aa}(0) = -1/3 and K^{ab}(0) = 0 at k = 0.
* Trace identity, every offset, any k: from (Laplacian + k^2) g = -delta,
  sum_a K^{aa}(d) = 2 kappa^2 I3(d) - delta_{d0}.  This ties the face
  integrals (2-D) to the volume integral (3-D).
* Newell, Williams & Dunlop's closed-form demagnetising tensor between two
  cubic cells (static, all components, near offsets); its two auxiliary
  functions are first checked against their defining derivatives here.
* Far field (offsets at least two voxels apart): the face form equals the
  volume form int (kappa^2 delta_ab + d_a d_b) g * tent^3, computed here with
  the analytic second derivatives of g.
* Parity/symmetry of Sec. 2 (after eq. sys_mat), checked by evaluating the
  face formula directly at negative offsets and with the roles of a, b swapped.
"""
import itertools

import numpy as np
import pytest

from oracle import generator as G

KAPPAS = [0.2926652804732217, 0.14633264023661085]


def test_static_self_term_is_one_third():
    for c, (a, b) in enumerate(G.COMPONENTS):
        v = G.generator_entry(a, b, (0, 0, 0), 0.0)
        expect = -1.0 / 3.0 if a == b else 0.0
        assert abs(v - expect) < 1e-14


@pytest.mark.parametrize("kappa", KAPPAS + [0.0, 0.3 - 0.2j])
@pytest.mark.parametrize("d", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1), (2, 0, 0), (2, 1, 1),
                               (3, 2, 0), (7, 1, 2), (16, 3, 3)])
def test_trace_identity(d, kappa):
    tr = sum(G.generator_entry(a, a, d, kappa) for a in range(3))
    expect = 2.0 * kappa * kappa * G.volume_term(d, kappa) - (1.0 if d == (0, 0, 0) else 0.0)
    assert abs(tr - expect) < 1e-13 * max(1.0, abs(expect)) + 1e-15


# --- Newell's closed-form static interaction tensor between two unit cubes ---------
def _safe_asinh(num, den):
    return np.arcsinh(num / den) if den > 0 else 0.0


def _safe_atan(num, den):
    return np.arctan(num / den) if den != 0 else 0.0


def newell_f(x, y, z):
    """Four-fold antiderivative with d^2/dy^2 d^2/dz^2 f = 1/R (up to terms killed below)."""
    R = np.sqrt(x * x + y * y + z * z)
    t = 0.0
    if x * x + z * z > 0:
        t += 0.5 * y * (z * z - x * x) * _safe_asinh(y, np.sqrt(x * x + z * z))
    if x * x + y * y > 0:
        t += 0.5 * z * (y * y - x * x) * _safe_asinh(z, np.sqrt(x * x + y * y))
    if x != 0 and R > 0:
        t -= x * y * z * _safe_atan(y * z, x * R)
    t += (2 * x * x - y * y - z * z) * R / 6.0
    return t


def newell_g(x, y, z):
    """Antiderivative with d/dx d/dy d^2/dz^2 g = 1/R (up to terms killed below)."""
    R = np.sqrt(x * x + y * y + z * z)
    t = 0.0
    if x * x + y * y > 0:
        t += x * y * z * np.arcsinh(z / np.sqrt(x * x + y * y))
    if y * y + z * z > 0:
        t += y / 6.0 * (3 * z * z - y * y) * np.arcsinh(x / np.sqrt(y * y + z * z))
    if x * x + z * z > 0:
        t += x / 6.0 * (3 * z * z - x * x) * np.arcsinh(y / np.sqrt(x * x + z * z))
    if z != 0 and R > 0:
        t -= z ** 3 / 6.0 * np.arctan(x * y / (z * R))
    if y != 0 and R > 0:
        t -= z * y * y / 2.0 * np.arctan(x * z / (y * R))
    if x != 0 and R > 0:
        t -= z * x * x / 2.0 * np.arctan(y * z / (x * R))
    t -= x * y * R / 3.0
    return t


def newell_tensor(fun, X):
    """(1/4pi) prod_axes (2 - S+ - S-) fun at X: the demagnetising tensor entry."""
    s = 0.0
    for e in itertools.product((-1, 0, 1), repeat=3):
        w = 1.0
        for ea in e:
            w *= 2.0 if ea == 0 else -1.0
        s += w * fun(X[0] + e[0], X[1] + e[1], X[2] + e[2])
    return s / (4.0 * np.pi)


def test_newell_auxiliary_functions_satisfy_their_definitions():
    h = 1e-2
    for (x, y, z) in [(0.7, 1.3, 0.9), (1.9, 0.4, 1.1), (0.5, 2.2, 1.7)]:
        r = 1.0 / np.sqrt(x * x + y * y + z * z)
        c2 = ((-1, 1.0), (0, -2.0), (1, 1.0))
        d4 = sum(ci * cj * newell_f(x, y + i * h, z + j * h) for i, ci in c2 for j, cj in c2) / h ** 4
        assert abs(d4 - r) < 1e-5
        c1 = ((-1, -1.0), (1, 1.0))
        dg = sum(ci * cj * ck * newell_g(x + i * h, y + j * h, z + k * h)
                 for i, ci in c1 for j, cj in c1 for k, ck in c2) / (4 * h * h * h * h)
        assert abs(dg - r) < 1e-5


def _newell_component(a, b, d):
    """Static K^{ab}(d) = -N_demag^{ab}(d) by relabelling axes of Newell's xx / xy forms."""
    if a == b:
        others = [c for c in range(3) if c != a]
        X = (d[a], d[others[0]], d[others[1]])
        return -newell_tensor(newell_f, X)
    c = 3 - a - b
    X = (d[a], d[b], d[c])
    return -newell_tensor(newell_g, X)


@pytest.mark.parametrize("d", [d for d in itertools.product(range(3), repeat=3)])
def test_static_near_field_matches_newell(d):
    for a, b in G.COMPONENTS:
        v = G.generator_entry(a, b, d, 0.0)
        ref = _newell_component(a, b, d)
        assert abs(v.imag) < 1e-15
        assert abs(v.real - ref) < 2e-13, (a, b, d, v, ref)


# --- far field: dyadic volume form -------------------------------------------------
def _dyadic_volume(a, b, d, kappa, p=16):
    """int (kappa^2 delta_ab + d_a d_b) g(|t|) prod L(t_i - d_i) dt, tensor Gauss on 8 cells."""
    x, w = np.polynomial.legendre.leggauss(p)
    s, ws = 0.5 * (x + 1.0), 0.5 * w
    total = 0.0 + 0.0j
    for cell in itertools.product((0, 1), repeat=3):
        axes, wts = [], []
        for i in range(3):
            lo = d[i] - 1 + cell[i]
            axes.append(lo + s)
            wts.append(ws * (1.0 - np.abs(lo + s - d[i])))
        T = np.meshgrid(*axes, indexing='ij')
        Wt = np.einsum('i,j,k->ijk', *wts)
        R = np.sqrt(T[0] ** 2 + T[1] ** 2 + T[2] ** 2)
        ra, rb = T[a] / R, T[b] / R
        e = np.exp(-1j * kappa * R) / (4 * np.pi * R ** 3)
        dd = e * ((3 * ra * rb - (1.0 if a == b else 0.0)) * (1 + 1j * kappa * R)
                  - kappa ** 2 * R ** 2 * ra * rb)
        if a == b:
            dd = dd + kappa ** 2 * np.exp(-1j * kappa * R) / (4 * np.pi * R)
        total += np.sum(dd * Wt)
    return total


@pytest.mark.parametrize("kappa", KAPPAS)
@pytest.mark.parametrize("d", [(2, 0, 0), (0, 2, 1), (2, 2, 2), (3, 1, 0), (5, 4, 1), (12, 3, 2),
                               (40, 7, 3)])
def test_far_field_face_form_equals_volume_form(d, kappa):
    for a, b in G.COMPONENTS:
        v = G.generator_entry(a, b, d, kappa)
        ref = _dyadic_volume(a, b, d, kappa)
        assert abs(v - ref) < 1e-12 * max(abs(ref), 1e-3), (a, b, d, v, ref)


@pytest.mark.parametrize("d", [(1, 2, 0), (1, 1, 1), (2, 1, 3), (0, 1, 2)])
def test_parity_and_symmetry_by_direct_evaluation(d):
    kappa = KAPPAS[0]
    for signs in itertools.product((1, -1), repeat=3):
        ds = tuple(s * v for s, v in zip(signs, d))
        for a in range(3):
            for b in range(3):
                direct = G.generator_entry(a, b, ds, kappa)
                lo, hi = min(a, b), max(a, b)
                octant = G.generator_entry(lo, hi, d, kappa)
                assert abs(direct - G.parity_sign(a, b, ds) * octant) < 1e-14, (a, b, ds)


def test_quadrature_order_converged():
    kappa = KAPPAS[0]
    for d in [(0, 0, 0), (1, 1, 0), (2, 1, 1), (6, 0, 0)]:
        for a, b in G.COMPONENTS:
            v1 = G.generator_entry(a, b, d, kappa)
            p, ps = G._orders(d)
            v2 = G.generator_entry(a, b, d, kappa, order=(p + 8, ps + 8))
            assert abs(v1 - v2) < 1e-13


def test_octant_table_matches_entries():
    kappa = KAPPAS[1]
    K = G.generator_octant((3, 2, 2), kappa)
    for dz, dy, dx in itertools.product(range(2), range(2), range(3)):
        for c, (a, b) in enumerate(G.COMPONENTS):
            assert K[c, dz, dy, dx] == G.generator_entry(a, b, (dx, dy, dz), kappa)
