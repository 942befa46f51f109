"""Circulant preconditioners (oracle; test infrastructure only).

* ``chan``                -- T. Chan's optimal circulant, Sec. 4 eq. Chan:
                             c_i = ((n-i)/n) t_i + (i/n) t_{-(n-i)}, 0 <= i < n,
                             with t_i the entries of the Toeplitz matrix
                             T_n = {t_{i-j}} (first column t_0..t_{n-1}).
* ``chan_olkin_blocks``   -- the 1-level block circulant C_B of Sec. 4: the
                             Chan circulant of every x-level Toeplitz block of
                             I - M~ N, diagonalised by F along x and permuted
                             to diag(D_1..D_n) (eq. Di).  F_{kl} = exp(-2 pi i k l / n)
                             (Sec. 4: C = F^{-1} diag(F c) F), modes in natural
                             order k = 0..n-1.
* ``BlockCirculantInverse`` -- C_B^{-1} = F^{-1} P^T diag(D_k^{-1}) P F
                             (Sec. 4, inverse after eq. Di), blocks by dense LU
                             with partial pivoting.
* ``reduction_keep``      -- the memory reduction of Sec. 5.1.1 (eqs. proxy1,
                             proxy2): keep D_k where |v_k|/||v||_inf > tol, every
                             other mode uses the central block D_{ceil(n/2)}.
* ``chan_transform_2level``, ``BlockCirculantInverse2`` -- the 2-level circulant
                             C_B2 of Sec. 4: the Chan approximation applied again,
                             along y, to the Toeplitz blocks of every D_k; one
                             3nz x 3nz block per mode pair (kx, ky).  Needs a
                             homogenised contrast that does not vary along x or y.
* ``share_runs``          -- a stronger compression read from the outlook of Sec. 6: runs
                             of consecutive kept modes with close proxy values share one block.
* ``BlockedPreconditioner`` -- the blocked-circulant preconditioner of Sec. 5.3:
                             one circulant preconditioner per box, block
                             diagonal; voxels outside every box are left as is.

Readings (the paper is silent or ambiguous):
* Within a box the cross-section block index is r = a*(ny*nz) + y + ny*z
  (component slowest, then z, then y), so m = 3 ny nz.
* Proxy entry "D_i(1, ceil(ny/2) ceil(nz/2))": row 1 is (x-component, y=0,
  z=0); the column is the 1-based linear cross-section index
  ceil(ny/2)*ceil(nz/2) (y fastest) of the x-component (default reading), or,
  as an alternative reading, the voxel (ceil(ny/2), ceil(nz/2)) at the
  cross-section centre.  It is read from the
  Chan/DFT transform of the generator K alone (no M~, no identity), so it stays
  defined where M~ vanishes.  The keep test is strict (>), the central block is
  mode ceil(n/2) - 1 (0-based) and is always stored.
* Each box uses its own length n in the Chan weights and its own M~; the
  generator is shared (translation invariant).
"""
import numpy as np
import scipy.linalg

from .generator import generator_signed


def chan(t):
    """Chan first column c_0..c_{n-1} from t_l, l = -(n-1)..(n-1) given as t[l + n - 1]."""
    t = np.asarray(t)
    n = (t.shape[0] + 1) // 2
    c = np.empty((n,) + t.shape[1:], dtype=np.complex128)
    c[0] = t[n - 1]
    for i in range(1, n):
        c[i] = ((n - i) / n) * t[i + n - 1] + (i / n) * t[i - n + n - 1]
    return c


def dft_matrix(n):
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n)


def _n_sequences(Koct, n, ny, nz):
    """N^{ab}(l, dy, dz) for l in (-n, n), dy in (-ny, ny), dz in (-nz, nz).

    Returns array [3, 3, 2n-1, 2ny-1, 2nz-1] indexed by (l+n-1, dy+ny-1, dz+nz-1).
    """
    l = np.arange(-(n - 1), n)
    dy = np.arange(-(ny - 1), ny)
    dz = np.arange(-(nz - 1), nz)
    L, DY, DZ = np.meshgrid(l, dy, dz, indexing='ij')
    out = np.zeros((3, 3) + L.shape, dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            out[a, b] = generator_signed(Koct, a, b, L, DY, DZ)
            if a == b:
                out[a, b][n - 1, ny - 1, nz - 1] += 1.0  # N = I + K
    return out


def chan_transform(Koct, n, ny, nz, include_identity=True):
    """C^_k^{ab}(dy, dz) = sum_l c_l exp(-2 pi i k l/n), c = Chan(N^{ab}(., dy, dz)).

    Array [n, 3, 3, 2ny-1, 2nz-1]; with include_identity=False it is built from
    K alone (used by the memory-reduction proxy).
    """
    seq = _n_sequences(Koct, n, ny, nz)
    if not include_identity:
        for a in range(3):
            seq[a, a][n - 1, ny - 1, nz - 1] -= 1.0
    seq = np.moveaxis(seq, 2, 0)  # [2n-1, 3, 3, dy, dz]
    c = chan(seq)                 # [n, 3, 3, dy, dz]
    F = dft_matrix(n)
    return np.tensordot(F, c, axes=(1, 0))


def chan_olkin_blocks(Koct, Mt, n, ny, nz):
    """D_k = I - diag(M~) C^_k, k = 0..n-1, each m x m with m = 3 ny nz.

    ``Mt`` is the box's homogenised contrast [nz, ny].  Entry
    D_k[(a,y,z),(b,y',z')] = delta - M~(y,z) C^_k^{ab}(y-y', z-z').
    """
    Ch = chan_transform(Koct, n, ny, nz)
    m = 3 * ny * nz
    D = np.zeros((n, m, m), dtype=np.complex128)
    Mt = np.asarray(Mt, dtype=np.complex128)
    for a in range(3):
        for y in range(ny):
            for z in range(nz):
                r = a * ny * nz + y + ny * z
                for b in range(3):
                    for yp in range(ny):
                        for zp in range(nz):
                            c = b * ny * nz + yp + ny * zp
                            D[:, r, c] = -Mt[z, y] * Ch[:, a, b, y - yp + ny - 1, z - zp + nz - 1]
                D[:, r, r] += 1.0
    return D


def proxy_column(ny, nz, reading='product'):
    """(y', z') of the proxy entry's column (x-component).

    'product': the 1-based linear cross-section index ceil(ny/2)*ceil(nz/2), y fastest;
    'centre' : the voxel (ceil(ny/2), ceil(nz/2)) (1-based), i.e. the cross-section centre.
    """
    if reading == 'centre':
        return int(np.ceil(ny / 2.0)) - 1, int(np.ceil(nz / 2.0)) - 1
    col = int(np.ceil(ny / 2.0)) * int(np.ceil(nz / 2.0)) - 1   # 0-based linear index
    return col % ny, col // ny


def proxy_values(Koct, n, ny, nz, reading='product'):
    """v_k of eq. proxy1 (reading in the module header); returns v [n]."""
    yp, zp = proxy_column(ny, nz, reading)
    Ch = chan_transform(Koct, n, ny, nz, include_identity=False)
    return Ch[:, 0, 0, 0 - yp + ny - 1, 0 - zp + nz - 1]


def reduction_keep(v, tol):
    """Keep mask (eq. proxy2: |v / ||v||_inf| > tol) and the central mode index."""
    v = np.asarray(v)
    vhat = np.abs(v / np.max(np.abs(v)))
    keep = vhat > tol
    centre = int(np.ceil(len(v) / 2.0)) - 1
    keep[centre] = True
    return keep, centre


def share_runs(v, keep, share_tol, centre=None):
    """Stronger compression (a reading of the outlook of Sec. 6, not a method the paper gives):
    walking the kept modes in ascending k, a mode joins the current run while its proxy value
    is within share_tol (relative) of the run's first mode, |v_k - v_rep| <= share_tol |v_rep|,
    else it starts a new run.  Under the memory reduction the central mode (whose block the
    discarded modes use) always starts a run of its own.  Returns rep [n]: the representative
    mode of every kept mode (-1 for discarded ones).  share_tol = 0 keeps every kept mode on its
    own block."""
    v = np.asarray(v)
    rep = np.full(len(v), -1)
    cur = -1
    for k in range(len(v)):
        if not keep[k]:
            continue
        if cur >= 0 and share_tol > 0 and k != centre and abs(v[k] - v[cur]) <= share_tol * abs(v[cur]):
            rep[k] = cur
        else:
            cur = k
            rep[k] = k
    return rep


class BlockCirculantInverse:
    """z = C_B^{-1} r for one box (Sec. 4), optionally memory reduced (Sec. 5.1.1) and with
    runs of similar kept modes sharing one block (share_runs)."""

    def __init__(self, Koct, Mt, n, ny, nz, reduce_tol=None, proxy='product', share_tol=0.0):
        self.n, self.ny, self.nz = n, ny, nz
        D = chan_olkin_blocks(Koct, Mt, n, ny, nz)
        if reduce_tol is not None:
            keep, centre = reduction_keep(proxy_values(Koct, n, ny, nz, proxy), reduce_tol)
            self.keep, self.centre = keep, centre
            self.block_of_mode = np.where(keep, np.arange(n), centre)
        else:
            self.keep = np.ones(n, dtype=bool)
            self.centre = int(np.ceil(n / 2.0)) - 1
            self.block_of_mode = np.arange(n)
        if share_tol > 0:
            rep = share_runs(proxy_values(Koct, n, ny, nz, proxy), self.keep, share_tol,
                             self.centre if reduce_tol is not None else None)
            self.block_of_mode = np.where(self.keep, rep, self.block_of_mode)
        self.lu = {}
        for k in np.unique(self.block_of_mode):
            self.lu[int(k)] = scipy.linalg.lu_factor(D[k])
        self.D = D

    def apply(self, r):
        """r: [3, nz, ny, n] (box-local) -> z of the same shape."""
        n, ny, nz = self.n, self.ny, self.nz
        m = 3 * ny * nz
        F = dft_matrix(n)
        r = np.asarray(r, dtype=np.complex128).reshape(m, n)   # row = (a, z, y) = a*ny*nz + y + ny*z
        rh = r @ F.T                                            # DFT along x of every line
        zh = np.empty_like(rh)
        for k in range(n):
            zh[:, k] = scipy.linalg.lu_solve(self.lu[int(self.block_of_mode[k])], rh[:, k])
        z = zh @ np.conj(F).T / n                               # inverse DFT
        return z.reshape(3, nz, ny, n)


def chan_transform_2level(Koct, nx, ny, nz):
    """C^_{kx,ky}^{ab}(dz) of the 2-level circulant (Sec. 4): the x-level table of
    chan_transform, then T. Chan's circulant of each of its Toeplitz sequences along y
    (dy in (-ny, ny)) and a DFT along y.  Array [nx, ny, 3, 3, 2nz-1], modes in natural order.
    """
    Ch = chan_transform(Koct, nx, ny, nz)                # [nx, 3, 3, 2ny-1, 2nz-1]
    seq = np.moveaxis(Ch, 3, 0)                          # [2ny-1, nx, 3, 3, 2nz-1]
    c = chan(seq)                                        # [ny, nx, 3, 3, 2nz-1]
    out = np.tensordot(dft_matrix(ny), c, axes=(1, 0))   # [ky, nx, 3, 3, 2nz-1]
    return np.moveaxis(out, 0, 1)


def chan_olkin_blocks_2level(Koct, Mz, nx, ny, nz):
    """D_{kx,ky} = I - diag(M~) C^_{kx,ky}, each 3nz x 3nz with row (a, z) -> a*nz + z;
    ``Mz`` is the homogenised contrast per z layer [nz]."""
    Ch = chan_transform_2level(Koct, nx, ny, nz)
    m = 3 * nz
    Mz = np.asarray(Mz, dtype=np.complex128)
    D = np.zeros((nx, ny, m, m), dtype=np.complex128)
    for a in range(3):
        for z in range(nz):
            r = a * nz + z
            for b in range(3):
                for zp in range(nz):
                    D[:, :, r, b * nz + zp] = -Mz[z] * Ch[:, :, a, b, z - zp + nz - 1]
            D[:, :, r, r] += 1.0
    return D


class BlockCirculantInverse2:
    """z = C_B2^{-1} r for one box (Sec. 4, 2-level): DFTs along x and y, one dense solve per
    mode pair (kx, ky), inverse DFTs."""

    def __init__(self, Koct, Mz, n, ny, nz):
        self.n, self.ny, self.nz = n, ny, nz
        D = chan_olkin_blocks_2level(Koct, Mz, n, ny, nz)
        self.lu = [[scipy.linalg.lu_factor(D[kx, ky]) for ky in range(ny)] for kx in range(n)]
        self.D = D
        self.keep = np.ones(n * ny, dtype=bool)

    def apply(self, r):
        """r: [3, nz, ny, n] (box-local) -> z of the same shape."""
        n, ny, nz = self.n, self.ny, self.nz
        Fx, Fy = dft_matrix(n), dft_matrix(ny)
        r = np.asarray(r, dtype=np.complex128).reshape(3, nz, ny, n)
        rh = np.einsum('kx,azyx->azyk', Fx, r)
        rh = np.einsum('jy,azyk->azjk', Fy, rh)                 # [3, nz, ky, kx]
        zh = np.empty_like(rh)
        for kx in range(n):
            for ky in range(ny):
                zh[:, :, ky, kx] = scipy.linalg.lu_solve(self.lu[kx][ky], rh[:, :, ky, kx].reshape(-1)).reshape(3, nz)
        z = np.einsum('jy,azjk->azyk', np.conj(Fy), zh) / ny
        z = np.einsum('kx,azyk->azyx', np.conj(Fx), z) / n
        return z


class BlockedPreconditioner:
    """Block-diagonal circulant preconditioner over boxes (Sec. 5.3).

    ``boxes`` = list of (x0, y0, z0, nx, ny, nz); ``homog`` = one of
    'none', 'mode', 'mean', 'realmean' (Sec. 5.2), applied per box.
    """

    def __init__(self, Koct, M, grid, boxes=None, homog='none', reduce_tol=None, proxy='product', levels=1,
                 share_tol=0.0):
        """``homog`` and ``levels`` apply to every box, or are lists with one entry per box."""
        from .contrast import homogenize
        nx, ny, nz = grid
        self.grid = grid
        self.boxes = boxes or [(0, 0, 0, nx, ny, nz)]
        M = np.asarray(M, dtype=np.complex128)
        nb = len(self.boxes)
        homogs = list(homog) if isinstance(homog, (list, tuple)) else [homog] * nb
        levs = list(levels) if isinstance(levels, (list, tuple)) else [levels] * nb
        self.parts = []
        for (x0, y0, z0, bx, by, bz), hk, lev in zip(self.boxes, homogs, levs):
            Mt = homogenize(M[z0:z0 + bz, y0:y0 + by, x0:x0 + bx], hk)
            if lev == 2:
                Mt = np.broadcast_to(Mt, (bz, by))
                if not np.all(Mt == Mt[:, :1]):
                    raise ValueError('the 2-level circulant needs a contrast that does not vary along y')
                self.parts.append(BlockCirculantInverse2(Koct, Mt[:, 0], bx, by, bz))
            else:
                self.parts.append(BlockCirculantInverse(Koct, Mt, bx, by, bz, reduce_tol, proxy, share_tol))

    def apply(self, r):
        nx, ny, nz = self.grid
        r = np.asarray(r, dtype=np.complex128).reshape(3, nz, ny, nx)
        z = r.copy()
        for (x0, y0, z0, bx, by, bz), part in zip(self.boxes, self.parts):
            sub = r[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx]
            z[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx] = part.apply(sub)
        return z.reshape(-1)
