"""Pins of the oracle's circulant preconditioners (Sec. 4, Sec. 5.1.1-5.3).

* Chan's formula is the Frobenius-nearest circulant (Sec. 4, after eq. Chan):
  checked against a brute-force least-squares fit over all circulants.
* A circulant is its own Chan circulant; C = F^{-1} diag(F c) F (Sec. 4).
* The 1-level block circulant built elementwise from Chan(T_ij) of the dense
  operator's Toeplitz blocks (no FFT, no permutation), inverted densely,
  equals the oracle's DFT + permuted block solves (eq. Di and its inverse).
* If the operator is circulant along x, the preconditioner is exact and
  preconditioned GMRES converges in one step.  Zero contrast gives P = I.
* Memory reduction (Sec. 5.1.1): tol 0 keeps everything (identical result),
  tol > 1 keeps only the central block, kept count monotone in tol.
* Blocked preconditioner (Sec. 5.3): one box is the 1-level preconditioner;
  several boxes equal a dense block-diagonal build.
* Homogenisations (Sec. 5.2 list) on hand-made arrays.
* 2-level circulant (Sec. 4): equals the block-circulant-circulant matrix built elementwise
  from T. Chan's weights in x and y (no DFT, no blocks) and inverted densely; with one y
  layer it is the 1-level preconditioner; zero contrast gives the identity.
* Reflection along x: the xy and xz couplings are odd in the x offset and the others even, so
  D_{n-k} = S D_k S with S = -1 on the x-component rows (the identity the GPU path uses to
  solve modes k > n/2 with the factors of mode n - k), for odd and even n.
* Cross-section rows with M~ = 0 are identity rows of every D_k (eq. Di), so the block
  solve reduces exactly to the other rows S plus the coupling M~_S C^_SC r^_C, and to the
  S x S solve alone when r^_C = 0 (the reduction the GPU path takes for cladding rows).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import circulant as C
from oracle import contrast as CT
from oracle import generator as G
from oracle import gmres as GM
from oracle import matvec as MV

KAPPA = 0.2926652804732217


def test_chan_is_frobenius_optimal():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 8):
        t = rng.standard_normal(2 * n - 1) + 1j * rng.standard_normal(2 * n - 1)
        T = np.array([[t[i - j + n - 1] for j in range(n)] for i in range(n)])
        # design matrix: vec(circ(c)) = E c
        E = np.zeros((n * n, n))
        for i in range(n):
            for j in range(n):
                E[i * n + j, (i - j) % n] = 1.0
        c_ls = np.linalg.lstsq(E, T.reshape(-1), rcond=None)[0]
        assert np.allclose(C.chan(t), c_ls, rtol=1e-13, atol=1e-14)


def test_circulant_fixed_point_and_diagonalisation():
    rng = np.random.default_rng(1)
    n = 7
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    t = np.array([c[l % n] for l in range(-(n - 1), n)])
    assert np.allclose(C.chan(t), c, rtol=1e-14)
    Cm = np.array([[c[(i - j) % n] for j in range(n)] for i in range(n)])
    F = C.dft_matrix(n)
    assert np.allclose(np.linalg.inv(F) @ np.diag(F @ c) @ F, Cm, atol=1e-13)


@pytest.fixture(scope="module")
def box():
    grid = (6, 3, 2)
    K = G.generator_octant(grid, KAPPA)
    rng = np.random.default_rng(7)
    Mt = 0.8 + 0.1 * rng.standard_normal((2, 3)) + 0.05j * rng.standard_normal((2, 3))
    return grid, K, Mt


def _dense_block_circulant(K, Mt, grid):
    """C_B elementwise: Chan of every x-level Toeplitz block of I - M~ N (no FFT)."""
    nx, ny, nz = grid
    M3 = np.broadcast_to(Mt[:, :, None], (nz, ny, nx))
    A = MV.operator_matrix(K, M3, grid)     # rows/cols: (a, z, y, x), x fastest
    m = 3 * ny * nz
    A4 = A.reshape(m, nx, m, nx)
    CB = np.zeros_like(A4)
    for r in range(m):
        for c in range(m):
            T = A4[r, :, c, :]
            t = np.array([T[l, 0] if l >= 0 else T[0, -l] for l in range(-(nx - 1), nx)])
            cc = C.chan(t)
            CB[r, :, c, :] = np.array([[cc[(i - j) % nx] for j in range(nx)] for i in range(nx)])
    return CB.reshape(m * nx, m * nx), A


def test_block_circulant_inverse_matches_dense(box):
    grid, K, Mt = box
    nx, ny, nz = grid
    CB, _ = _dense_block_circulant(K, Mt, grid)
    inv = C.BlockCirculantInverse(K, Mt, nx, ny, nz)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(3 * nx * ny * nz) + 1j * rng.standard_normal(3 * nx * ny * nz)
    z = inv.apply(r.reshape(3, nz, ny, nx)).reshape(-1)
    assert np.allclose(z, np.linalg.solve(CB, r), rtol=1e-12, atol=1e-12)


def test_blocks_are_the_permuted_fourier_diagonal(box):
    grid, K, Mt = box
    nx, ny, nz = grid
    m = 3 * ny * nz
    CB, _ = _dense_block_circulant(K, Mt, grid)
    F = C.dft_matrix(nx)
    FF = np.kron(np.eye(m), F)
    L = FF @ CB @ np.linalg.inv(FF)                      # [Lambda_ij], each diagonal
    L4 = L.reshape(m, nx, m, nx)
    D = C.chan_olkin_blocks(K, Mt, nx, ny, nz)
    for k in range(nx):
        assert np.allclose(L4[:, k, :, k], D[k], atol=1e-12)
        for k2 in range(nx):
            if k2 != k:
                assert np.abs(L4[:, k, :, k2]).max() < 1e-12


def test_x_circulant_operator_gives_exact_preconditioner():
    grid = (5, 2, 2)
    nx, ny, nz = grid
    Kfull = G.generator_octant(grid, KAPPA)
    K = np.zeros_like(Kfull)
    K[:, :, :, 0] = Kfull[:, :, :, 0]         # no coupling along x: T blocks are diagonal
    M = np.full((nz, ny, nx), 0.8 + 0.05j)
    A = MV.operator_matrix(K, M, grid)
    P = C.BlockedPreconditioner(K, M, grid, homog='none')
    b = np.random.default_rng(4).standard_normal(3 * 20) + 0j
    x, info = GM.gmres(lambda v: A @ v, b, M=P.apply, tol=1e-12)
    assert info['iters'] == 1 and info['relres'] < 1e-12


def test_zero_contrast_gives_identity(box):
    grid, K, _ = box
    nx, ny, nz = grid
    inv = C.BlockCirculantInverse(K, np.zeros((nz, ny)), nx, ny, nz)
    r = np.random.default_rng(5).standard_normal((3, nz, ny, nx)) + 0j
    assert np.allclose(inv.apply(r), r, rtol=1e-14, atol=1e-14)


def test_zero_contrast_rows_reduce_exactly(box):
    grid, K, Mt = box
    nx, ny, nz = grid
    Mt = Mt.copy()
    Mt[0, 1] = 0.0
    Mt[1, 2] = 0.0
    D = C.chan_olkin_blocks(K, Mt, nx, ny, nz)
    Ch = C.chan_transform(K, nx, ny, nz)
    m = 3 * ny * nz
    zero = np.array([Mt[(i % (ny * nz)) // ny, i % ny] == 0 for i in range(m)])
    S, Cr = np.nonzero(~zero)[0], np.nonzero(zero)[0]
    assert len(Cr) == 6
    eye = np.eye(m)
    for k in range(nx):
        assert np.array_equal(D[k][Cr], eye[Cr])     # identity rows, exactly
    rng = np.random.default_rng(12)
    for k in range(nx):
        rh = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        full = np.linalg.solve(D[k], rh)
        # coupling from the Chan table itself: M~(y,z) C^_k[(a,y,z),(b,y',z')] r^_C
        cpl = np.zeros(len(S), dtype=complex)
        for ii, i in enumerate(S):
            a, y, z = i // (ny * nz), i % ny, (i % (ny * nz)) // ny
            for j in Cr:
                b, yp, zp = j // (ny * nz), j % ny, (j % (ny * nz)) // ny
                cpl[ii] += Mt[z, y] * Ch[k, a, b, y - yp + ny - 1, z - zp + nz - 1] * rh[j]
        zs = np.linalg.solve(D[k][np.ix_(S, S)], rh[S] + cpl)
        assert np.abs(zs - full[S]).max() < 1e-12 * np.abs(full).max()
        assert np.array_equal(full[Cr], rh[Cr]) or np.abs(full[Cr] - rh[Cr]).max() < 1e-14
        rh[Cr] = 0.0
        full = np.linalg.solve(D[k], rh)
        zs = np.linalg.solve(D[k][np.ix_(S, S)], rh[S])
        assert np.abs(full[Cr]).max() < 1e-14 and np.abs(zs - full[S]).max() < 1e-12 * np.abs(full).max()


def test_reduction_limits_and_monotone(box):
    grid, K, Mt = box
    nx, ny, nz = grid
    full = C.BlockCirculantInverse(K, Mt, nx, ny, nz)
    r = np.random.default_rng(6).standard_normal((3, nz, ny, nx)) + 0j
    red0 = C.BlockCirculantInverse(K, Mt, nx, ny, nz, reduce_tol=0.0)
    assert red0.keep.all()
    assert np.array_equal(red0.apply(r), full.apply(r))
    red2 = C.BlockCirculantInverse(K, Mt, nx, ny, nz, reduce_tol=2.0)
    assert red2.keep.sum() == 1 and red2.keep[int(np.ceil(nx / 2)) - 1]
    v = C.proxy_values(K, nx, ny, nz)
    counts = [C.reduction_keep(v, tol)[0].sum() for tol in (0.0, 1e-3, 1e-2, 0.1, 0.5, 2.0)]
    assert all(a >= b for a, b in zip(counts, counts[1:]))


def test_proxy_entry_location():
    # ny=16, nz=8 -> column ceil(16/2)*ceil(8/2) = 32 (1-based) -> y'=15, z'=1
    grid = (4, 16, 8)
    K = np.zeros((6, 8, 16, 4), dtype=complex)
    K[0, 1, 15, :] = np.array([1.0, 2.0, 3.0, 4.0])
    v = C.proxy_values(K, 4, 16, 8)
    # t_l = K^{xx}(l, -15, -1) = K(|l|, 15, 1); Chan + DFT by hand
    t = np.array([4.0, 3.0, 2.0, 1.0, 2.0, 3.0, 4.0])
    c = C.chan(t)
    assert np.allclose(v, C.dft_matrix(4) @ c)


def test_blocked_single_box_equals_one_level(box):
    grid, K, Mt = box
    nx, ny, nz = grid
    M = np.broadcast_to(Mt[:, :, None], (nz, ny, nx))
    P = C.BlockedPreconditioner(K, M, grid)
    inv = C.BlockCirculantInverse(K, Mt, nx, ny, nz)
    r = np.random.default_rng(8).standard_normal(3 * nx * ny * nz) + 0j
    assert np.array_equal(P.apply(r), inv.apply(r.reshape(3, nz, ny, nx)).reshape(-1))


def test_blocked_boxes_equal_dense_block_diagonal():
    grid = (8, 3, 2)
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    rng = np.random.default_rng(9)
    M = 0.7 + 0.2 * rng.standard_normal((nz, ny, nx)) + 0.01j
    boxes = [(0, 0, 0, 3, 3, 2), (3, 0, 0, 4, 2, 2)]       # last x column and one y row uncovered
    P = C.BlockedPreconditioner(K, M, grid, boxes=boxes, homog='mean')
    n = nx * ny * nz
    Pd = np.eye(3 * n, dtype=complex)
    idx = lambda a, x, y, z: a * n + x + nx * (y + ny * z)
    for (x0, y0, z0, bx, by, bz) in boxes:
        Mt = CT.homogenize(M[z0:z0 + bz, y0:y0 + by, x0:x0 + bx], 'mean')
        CB, _ = _dense_block_circulant(K, Mt, (bx, by, bz))
        Cinv = np.linalg.inv(CB)
        loc = [idx(a, x0 + x, y0 + y, z0 + z) for a in range(3) for z in range(bz)
               for y in range(by) for x in range(bx)]
        Pd[np.ix_(loc, loc)] = Cinv
    r = rng.standard_normal(3 * n) + 1j * rng.standard_normal(3 * n)
    assert np.allclose(P.apply(r), Pd @ r, rtol=1e-12, atol=1e-12)


def test_homogenisations():
    M = np.zeros((1, 2, 4), dtype=complex)
    M[0, 0] = [1 + 1j, 2, 1 + 1j, 3]
    M[0, 1] = [2, 2, 0.5j, 1 + 1j]
    assert np.allclose(CT.homogenize(M, 'mode'), 1 + 1j)      # 3 x (1+1j) vs 3 x 2: earlier first
    assert np.allclose(CT.homogenize(M, 'mean'), [[(7 + 2j) / 4, (5 + 1.5j) / 4]])
    assert np.allclose(CT.homogenize(M, 'realmean'), [[7 / 4, 5 / 4]])
    with pytest.raises(ValueError):
        CT.homogenize(M, 'none')
    U = np.ones((2, 2, 3)) * (0.5 + 0.1j)
    assert np.allclose(CT.homogenize(U, 'none'), 0.5 + 0.1j)


def test_proxy_centre_reading_location():
    # centre reading: ny=16, nz=8 -> voxel (8, 4) 1-based -> y'=7, z'=3
    assert C.proxy_column(16, 8, 'centre') == (7, 3)
    assert C.proxy_column(16, 8, 'product') == (15, 1)
    assert C.proxy_column(1, 1, 'product') == (0, 0) and C.proxy_column(1, 1, 'centre') == (0, 0)
    K = np.zeros((6, 8, 16, 4), dtype=complex)
    K[0, 3, 7, :] = np.array([1.0, -2.0, 0.5, 4.0])
    v = C.proxy_values(K, 4, 16, 8, reading='centre')
    t = np.array([4.0, 0.5, -2.0, 1.0, -2.0, 0.5, 4.0])
    assert np.allclose(v, C.dft_matrix(4) @ C.chan(t))


def _dense_two_level(K, Mz, grid):
    """C_B2 elementwise: c(dx, dy) = sum over the four wrapped quadrants of T. Chan's weights in
    x and y times T(dx - s nx, dy - t ny), T = I - M~ N (no DFT, no blocks)."""
    nx, ny, nz = grid
    n3 = 3 * nz * ny * nx

    def T(a, b, dx, dy, z, zp):
        v = -Mz[z] * G.generator_signed(K, a, b, np.array(dx), np.array(dy), np.array(z - zp))
        if a == b and dx == 0 and dy == 0 and z == zp:
            v = v + 1.0 - Mz[z]  # N = I + K
        return complex(v)

    A = np.zeros((n3, n3), dtype=complex)
    idx = lambda a, z, y, x: ((a * nz + z) * ny + y) * nx + x
    for a in range(3):
        for b in range(3):
            for z in range(nz):
                for zp in range(nz):
                    for lx in range(nx):
                        for ly in range(ny):
                            c = 0.0
                            for s_, wx in ((0, (nx - lx) / nx), (1, lx / nx)):
                                for t_, wy in ((0, (ny - ly) / ny), (1, ly / ny)):
                                    if wx and wy:
                                        c += wx * wy * T(a, b, lx - s_ * nx, ly - t_ * ny, z, zp)
                            for x in range(nx):
                                for y in range(ny):
                                    A[idx(a, z, y, x), idx(b, zp, (y - ly) % ny, (x - lx) % nx)] = c
    return A


def test_two_level_matches_dense_twin():
    grid = (5, 4, 2)
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    Mz = np.array([0.83 - 0.02j, 0.61 + 0.05j])
    inv = C.BlockCirculantInverse2(K, Mz, nx, ny, nz)
    A = _dense_two_level(K, Mz, grid)
    r = np.random.default_rng(21).standard_normal(A.shape[0]) + 1j * np.random.default_rng(22).standard_normal(A.shape[0])
    z = inv.apply(r.reshape(3, nz, ny, nx)).reshape(-1)
    ref = np.linalg.solve(A, r)
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) < 1e-12


def test_two_level_with_one_y_layer_is_one_level():
    grid = (6, 1, 3)
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    Mz = np.array([0.8, 0.7 + 0.1j, 0.5])
    r = np.random.default_rng(23).standard_normal((3, nz, ny, nx)) + 0j
    z2 = C.BlockCirculantInverse2(K, Mz, nx, ny, nz).apply(r)
    z1 = C.BlockCirculantInverse(K, Mz[:, None], nx, ny, nz).apply(r)
    assert np.abs(z2 - z1).max() < 1e-13 * np.abs(z1).max()
    z0 = C.BlockCirculantInverse2(K, np.zeros(nz), nx, ny, nz).apply(r)
    assert np.abs(z0 - r).max() < 1e-14


def test_blocked_boxes_of_different_shapes_and_levels_equal_dense_block_diagonal():
    """A 1-level box (mean contrast) beside a 2-level box of another shape (modal contrast), with
    voxels outside both: the blocked apply equals the dense block-diagonal of the per-box dense
    circulant inverses (the 1-level one built elementwise, the 2-level one from its twin)."""
    grid = (7, 6, 2)
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    rng = np.random.default_rng(31)
    M = 0.7 + 0.2 * rng.standard_normal((nz, ny, nx)) - 0.03j
    M[:, 2:, 1:6] = 0.65 - 0.01j                       # the 2-level box: one dominant value (its mode)
    boxes = [(0, 0, 0, 7, 2, 2), (1, 2, 0, 5, 4, 2)]   # x column 0 and 6 of rows 2.. uncovered
    P = C.BlockedPreconditioner(K, M, grid, boxes=boxes, homog=['mean', 'mode'], levels=[1, 2])
    n = nx * ny * nz
    Pd = np.eye(3 * n, dtype=complex)
    idx = lambda a, x, y, z: a * n + x + nx * (y + ny * z)
    for (x0, y0, z0, bx, by, bz), hk, lev in zip(boxes, ['mean', 'mode'], [1, 2]):
        Mt = CT.homogenize(M[z0:z0 + bz, y0:y0 + by, x0:x0 + bx], hk)
        if lev == 1:
            CB, _ = _dense_block_circulant(K, Mt, (bx, by, bz))
        else:
            CB = _dense_two_level(K, Mt[:, 0], (bx, by, bz))
        Cinv = np.linalg.inv(CB)
        loc = [idx(a, x0 + x, y0 + y, z0 + z) for a in range(3) for z in range(bz)
               for y in range(by) for x in range(bx)]
        Pd[np.ix_(loc, loc)] = Cinv
    r = rng.standard_normal(3 * n) + 1j * rng.standard_normal(3 * n)
    assert np.allclose(P.apply(r), Pd @ r, rtol=1e-12, atol=1e-12)


def test_share_runs_rule():
    """Runs of kept modes: exact grouping on hand-made proxies, tolerance 0 = no sharing,
    discarded modes untouched, stored count non-increasing in the tolerance."""
    v = np.array([1.0, 1.004, 1.012, 2.0, 2.01, 0.001, 2.02, 5.0])
    keep = np.array([True, True, True, True, True, False, True, True])
    assert list(C.share_runs(v, keep, 0.0)) == [0, 1, 2, 3, 4, -1, 6, 7]
    assert list(C.share_runs(v, keep, 0.005)) == [0, 0, 2, 3, 3, -1, 6, 7]
    assert list(C.share_runs(v, keep, 0.02)) == [0, 0, 0, 3, 3, -1, 3, 7]
    counts = [len(set(C.share_runs(v, keep, t)[keep])) for t in (0.0, 0.005, 0.02, 0.5, 5.0)]
    assert counts == sorted(counts, reverse=True) and counts[-1] == 1
    # the central mode of the memory reduction starts its own run
    assert list(C.share_runs(v, keep, 0.02, centre=4)) == [0, 0, 0, 3, 4, -1, 4, 7]


def test_share_runs_apply_uses_the_representative_blocks(box):
    """With sharing the apply equals the per-mode solve with each run's representative block."""
    grid, K, Mt = box
    nx, ny, nz = grid
    inv = C.BlockCirculantInverse(K, Mt, nx, ny, nz, share_tol=0.3)
    v = C.proxy_values(K, nx, ny, nz)
    rep = C.share_runs(v, np.ones(nx, dtype=bool), 0.3)
    assert list(inv.block_of_mode) == list(rep) and len(set(rep)) < nx
    r = np.random.default_rng(41).standard_normal((3, nz, ny, nx)) + 0j
    F = C.dft_matrix(nx)
    rh = r.reshape(3 * ny * nz, nx) @ F.T
    zh = np.stack([np.linalg.solve(inv.D[rep[k]], rh[:, k]) for k in range(nx)], axis=1)
    z = (zh @ np.conj(F).T / nx).reshape(3, nz, ny, nx)
    assert np.abs(inv.apply(r) - z).max() < 1e-12 * np.abs(z).max()
    plain = C.BlockCirculantInverse(K, Mt, nx, ny, nz, share_tol=0.0)
    assert list(plain.block_of_mode) == list(range(nx))


@pytest.mark.parametrize('grid', [(6, 3, 2), (7, 2, 3)])
def test_reflected_modes_are_sign_conjugate(grid):
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    rng = np.random.default_rng(11)
    Mt = 0.8 + 0.1 * rng.standard_normal((nz, ny)) + 0.05j * rng.standard_normal((nz, ny))
    D = C.chan_olkin_blocks(K, Mt, nx, ny, nz)
    m = 3 * ny * nz
    S = np.diag(np.where(np.arange(m) < ny * nz, -1.0, 1.0))
    scale = np.abs(D).max()
    for k in range(1, nx):
        assert np.abs(D[nx - k] - S @ D[k] @ S).max() < 1e-13 * scale, k
    # not a tautology: the couplings that change sign are there
    assert np.abs(D[1][:ny * nz, ny * nz:]).max() > 1e-3 * scale


@pytest.mark.parametrize('grid', [(6, 5, 2), (5, 4, 3)])
def test_two_level_reflected_modes_are_sign_conjugate(grid):
    """2-level: the Chan circulant along y keeps the y parities, so D_{kx,ny-ky} = S_y D S_y as
    well as D_{nx-kx,ky} = S_x D S_x (S_x, S_y: -1 on the x / y component rows)."""
    nx, ny, nz = grid
    K = G.generator_octant(grid, KAPPA)
    Mz = 0.8 + 0.1j + 0.05 * np.arange(nz)
    D = C.chan_olkin_blocks_2level(K, Mz, nx, ny, nz)
    m = 3 * nz
    Sx = np.diag(np.where(np.arange(m) < nz, -1.0, 1.0))
    Sy = np.diag(np.where((np.arange(m) >= nz) & (np.arange(m) < 2 * nz), -1.0, 1.0))
    scale = np.abs(D).max()
    for kx in range(nx):
        for ky in range(ny):
            assert np.abs(D[(nx - kx) % nx, ky] - Sx @ D[kx, ky] @ Sx).max() < 1e-13 * scale, (kx, ky)
            assert np.abs(D[kx, (ny - ky) % ny] - Sy @ D[kx, ky] @ Sy).max() < 1e-13 * scale, (kx, ky)
    assert np.abs(D[1, 1][nz:2 * nz, :nz]).max() > 1e-3 * scale   # the xy coupling is there
