"""Whole-chain physics pin of the oracle: a voxelised dielectric sphere against the Mie series.

The oracle's generator (Galerkin K of Sec. 2, eq. op_N), contrast M = chi/(1 + chi) (eq. JVIE)
and operator I - M N are solved densely on the voxels inside a sphere of radius 1 with
k a = 1 (voxels outside have M = 0, so w = 0 there exactly and the system restricts to the
inside).  The voxel field e = w / chi is compared at the voxel centres with the interior
Mie field (tests/mie.py) of the sphere of equal volume (the staircase body's volume).
Expected behaviour of a correct discretisation: the error falls with the voxel size, at
about first order in the core (|r| < a/2) and at about half order over all voxels (the
staircase boundary layer holds O(h) of the volume with O(1) error).  A sign error in the
Green's function phase, a missing identity in N or a wrong contrast breaks the bounds.
"""
import numpy as np
import pytest

from oracle import contrast as CT
from oracle import generator as G

import mie

KA = 1.0


def _sphere_fields(n, eps_list):
    a, k = 1.0, KA
    delta = 2 * a / n
    K = G.generator_octant((n, n, n), k * delta)
    c = (np.arange(n) + 0.5) * delta - a
    Z, Y, X = np.meshgrid(c, c, c, indexing='ij')
    inside = (X ** 2 + Y ** 2 + Z ** 2) < a * a
    idx = np.nonzero(inside.reshape(-1))[0]
    pts = np.stack([X.reshape(-1)[idx], Y.reshape(-1)[idx], Z.reshape(-1)[idx]], 1)
    iv = np.rint((pts + a) / delta - 0.5).astype(int)
    ni = len(idx)
    N = np.eye(3 * ni, dtype=complex)
    for p in range(3):
        for q in range(3):
            d = [iv[:, t][:, None] - iv[:, t][None, :] for t in range(3)]
            N[p * ni:(p + 1) * ni, q * ni:(q + 1) * ni] += G.generator_signed(K, p, q, d[0], d[1], d[2])
    a_eq = (3 * ni * delta ** 3 / (4 * np.pi)) ** (1 / 3)
    out = {}
    for eps in eps_list:
        chi = np.full(ni, eps - 1.0, dtype=complex)
        M = CT.contrast_from_chi(chi)
        Mt = np.tile(M, 3)
        e_inc = np.zeros(3 * ni, dtype=complex)
        e_inc[:ni] = np.exp(-1j * k * pts[:, 2])
        w = np.linalg.solve(np.eye(3 * ni) - Mt[:, None] * N, Mt * e_inc)
        e = (w / np.tile(chi, 3)).reshape(3, ni).T
        e_mie = mie.internal_field(pts, eps, k * a_eq, radius=a_eq)
        core = np.linalg.norm(pts, axis=1) < 0.5 * a
        err = np.linalg.norm(e - e_mie) / np.linalg.norm(e_mie)
        err_core = np.linalg.norm(e[core] - e_mie[core]) / np.linalg.norm(e_mie[core])
        out[eps] = (err, err_core)
    return out


def test_mie_series_limits():
    """The series itself: m = 1 gives the incident wave; k a -> 0 gives 3/(eps+2) x^."""
    rng = np.random.default_rng(0)
    P = rng.uniform(-0.7, 0.7, (150, 3))
    P = P[np.linalg.norm(P, axis=1) < 0.95]
    E = mie.internal_field(P, 1.0, KA)
    inc = np.zeros_like(E)
    inc[:, 0] = np.exp(-1j * KA * P[:, 2])
    assert np.abs(E - inc).max() < 1e-12
    for eps in (2.0, 5.81):   # the incident phase adds O(k a) inside: k a = 1e-6
        E = mie.internal_field(P * 1e-6, eps, 1e-6, radius=1e-6)
        assert np.abs(E[:, 0] - 3 / (eps + 2)).max() < 1e-5
        assert np.abs(E[:, 1:]).max() < 1e-5


@pytest.fixture(scope='module')
def sphere_errors():
    return {n: _sphere_fields(n, (2.0, 5.81)) for n in (6, 10, 14)}


def test_sphere_matches_mie_within_discretisation_error(sphere_errors):
    for n, res in sphere_errors.items():
        print('n=%d: eps 2 err %.4f core %.4f | eps 5.81 err %.4f core %.4f'
              % (n, res[2.0][0], res[2.0][1], res[5.81][0], res[5.81][1]))
    # low contrast: accurate at every size
    for n, res in sphere_errors.items():
        assert res[2.0][0] < 0.07 and res[2.0][1] < 0.01
    # silicon-like contrast: errors fall monotonically with the voxel size
    e = [sphere_errors[n][5.81] for n in (6, 10, 14)]
    assert e[0][0] > e[1][0] > e[2][0] and e[0][1] > e[1][1] > e[2][1]
    assert e[2][0] < 0.2 and e[2][1] < 0.08
    # core convergence order >= 0.8
    order = np.log(e[0][1] / e[2][1]) / np.log(14 / 6)
    print('core convergence order (eps 5.81): %.2f' % order)
    assert order >= 0.8
