"""Contrast and homogenisation (oracle; test infrastructure only).

* M = (eps_r - 1)/eps_r, the local medium operator of the JVIE (Sec. 2,
  definition following eq. JVIE).  Permittivities are relative to the
  background medium (Sec. 3, Table ref_ind uses the ratio 12.1/2.085 for Si in
  SiO2), so with chi = eps_r - 1 the contrast is M = chi / (1 + chi).
* The three homogenised contrasts of Sec. 5.2 (enumerated list):
  1. mode  -- the modal value of all entries of M in the box (a scalar);
  2. mean  -- the arithmetic mean of M along x, per (y, z);
  3. realmean -- the real part of that mean.
  Reading: "mode" of complex values is exact-equality mode; ties go to the
  value whose first occurrence in x-fastest order is earliest.

Arrays are indexed [z, y, x] (x fastest in memory), matching the unknown
ordering of eq. sys_mat.
"""
import numpy as np


def contrast_from_chi(chi):
    """M = chi/(1+chi) elementwise, chi = eps_r - 1 (Sec. 2, after eq. JVIE)."""
    chi = np.asarray(chi, dtype=np.complex128)
    return chi / (1.0 + chi)


def homogenize(M, kind):
    """Return the x-invariant contrast M~(y, z) used to build a box's circulant.

    ``M`` is the box's contrast array [nz, ny, nx].  ``kind``:
      'none'     -- M itself; only valid when M does not vary along x,
      'mode'     -- Sec. 5.2 item 1 (scalar, broadcast over (y, z)),
      'mean'     -- Sec. 5.2 item 2,
      'realmean' -- Sec. 5.2 item 3.
    Returns an [nz, ny] complex array.
    """
    M = np.asarray(M, dtype=np.complex128)
    nz, ny, nx = M.shape
    if kind == 'none':
        if not np.all(M == M[:, :, :1]):
            raise ValueError("homogenisation 'none' needs an x-invariant contrast")
        return M[:, :, 0].copy()
    if kind == 'mode':
        flat = M.reshape(-1)  # x fastest, then y, then z
        counts = {}
        first = {}
        for i, v in enumerate(flat):
            key = (float(v.real), float(v.imag))
            counts[key] = counts.get(key, 0) + 1
            if key not in first:
                first[key] = i
        best = max(counts, key=lambda k: (counts[k], -first[k]))
        return np.full((nz, ny), complex(best[0], best[1]), dtype=np.complex128)
    if kind == 'mean':
        return M.sum(axis=2) / nx
    if kind == 'realmean':
        return (M.sum(axis=2) / nx).real.astype(np.complex128)
    raise ValueError("unknown homogenisation %r" % (kind,))
