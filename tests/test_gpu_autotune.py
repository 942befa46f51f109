"""Autotuned launches against the oracle.

Every candidate of each tuned kernel family is forced in turn through vie_autotune_set and its
results are compared with the oracle, not only with the default launch:

* operator products (right-hand sides per workgroup of the register plane pass x threads of
  the LDS x-line passes) on a 64x8x4 grid (LDS x lines) and a 512x16x8 grid (register x lines),
  FP64 and complex64, entry by entry against the oracle's FFT reference operator;
* the batched LU's sub-panels per macro panel (1, 2, 4, 8) x sub-panel width (32, 16) on
  384 x 384 blocks, FP64 and complex64 factors, and the block solves' per-mode and matrix-core candidates, each as the
  preconditioner's apply against the oracle's blocked preconditioner;
* a lockstep solve with every family tuned by timing, each column against the dense solution.

A choice that is not one of the shape's candidates is rejected with VIE_EARG before any launch.
Bars: products FP64 1e-10 / complex64 1e-5 of the largest entry; applies FP64 1e-10 /
complex64 1e-4 in norm.
"""
import numpy as np
import pytest

from oracle import circulant as OC
from oracle import contrast as OCT
from oracle import fftref as FR
from oracle import generator as OG
from oracle import matvec as OM
from paper_1903_07884_amd import workloads as W

pytestmark = pytest.mark.gpu

KB = W.k_background()


def _entrywise(y, ref):
    return max(np.abs(y[i] - ref[i]).max() / np.abs(ref[i]).max() for i in range(ref.shape[0]))


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _keys(gpu_lib, prefix, *parts):
    return [k for k in gpu_lib.autotune_entries() if k.startswith(prefix) and all(p in k for p in parts)]


def _ncand(gpu_lib, key):
    """Candidates the tuner timed for `key` (read before any entry is forced)."""
    for line in gpu_lib.autotune_report().splitlines():
        if line.startswith(key + ' ->'):
            return int(line.rsplit(',', 1)[1].split()[0])
    raise KeyError(key)


def _forced(gpu_lib, key, choice, run):
    """run() with `choice` stored under `key`; None if the library rejects the choice as not a
    candidate of the shape (VIE_EARG)."""
    gpu_lib.autotune_set(key, choice)
    try:
        return run()
    except gpu_lib.VieError as e:
        if 'not one of' not in str(e):
            raise
        return None


@pytest.mark.parametrize("grid,R", [((64, 8, 4), 12), ((512, 16, 8), 5)])
def test_every_matvec_candidate_matches_oracle(gpu_lib, grid, R):
    import torch
    nx, ny, nz = grid
    K = W.synthetic_generator(grid, 41, scale=0.2)
    chi = W.waveguide(grid)
    M = OCT.contrast_from_chi(chi)
    x = W.random_field((R, 3 * nx * ny * nz), 42)
    ref = FR.FftOperator(K, M, grid).matvec(x)
    xd = _dev(x)
    x32 = xd.to(torch.complex64)
    gdesc = 'grid=%dx%dx%d nrhs=%d ' % (nx, ny, nz, R)

    def products():
        op = gpu_lib.Operator(grid, 25e-9, KB, chi, generator=K, build_c64=True)
        try:
            y64, y32 = torch.empty_like(xd), torch.empty_like(x32)
            op.matvec(xd, y64, nrhs=R)
            op.matvec(x32, y32, nrhs=R)
            return y64.cpu().numpy(), y32.cpu().numpy().astype(np.complex128)
        finally:
            op.close()

    gpu_lib.autotune(True)
    keys = []
    try:
        products()  # tunes both precisions by timing
        keys = _keys(gpu_lib, 'matvec ', gdesc)
        assert len(keys) == 2, gpu_lib.autotune_report()
        counts = {key: _ncand(gpu_lib, key) for key in keys}
        # register plane pass on both grids: 0 (default grouping) and powers of two up to R
        planes = [0] + [rb for rb in (1, 2, 4, 8, 16) if rb <= R]
        xs = [0, 32, 64, 128, 256, 512, 1024]
        for key in keys:
            tried = []
            for rb in planes:
                for tx in xs:
                    out = _forced(gpu_lib, key, [rb, tx], products)
                    if out is None:
                        continue
                    y = out[0] if 'esz=16' in key else out[1]
                    err = _entrywise(y, ref)
                    tried.append((rb, tx))
                    print('%s -> %d %d: entry-wise %.2e' % (key, rb, tx, err))
                    assert err < (1e-10 if 'esz=16' in key else 1e-5)
            # every candidate the tuner timed ran once more, forced, and no other
            assert len(tried) == counts[key] and sorted({t[0] for t in tried}) == planes, tried
            gpu_lib.autotune_set(key, [])
        # a choice outside the candidates is refused before anything runs
        with pytest.raises(gpu_lib.VieError, match='not one of'):
            gpu_lib.autotune_set(keys[0], [3, 7])
            products()
    finally:
        for key in keys:
            gpu_lib.autotune_set(key, [])
        gpu_lib.autotune(False)


def test_every_lu_and_block_solve_candidate_matches_oracle(gpu_lib):
    import torch
    grid, delta = (32, 16, 8), 40e-9
    nx, ny, nz = grid
    K = OG.generator_octant(grid, KB * delta)
    chi = W.waveguide(grid)
    M = OCT.contrast_from_chi(chi)
    ref_pc = OC.BlockedPreconditioner(K, M, grid)
    n = 3 * nx * ny * nz
    m = 3 * ny * nz
    out = []
    try:
        gpu_lib.autotune(True)
        op = gpu_lib.Operator(grid, delta, KB, chi, generator=K, build_c64=True)
        for fprec, real, bar in ((gpu_lib.VIE_C128, 64, 1e-10), (gpu_lib.VIE_C64, 32, 1e-4)):
            for R in (2, 9):
                r = W.random_field((R, n), 50 + R)
                z_ref = np.stack([ref_pc.apply(r[i]) for i in range(R)])
                rd = _dev(r if fprec == gpu_lib.VIE_C128 else r.astype(np.complex64))

                def apply():
                    pc = gpu_lib.Preconditioner(op, factor_prec=fprec)
                    try:
                        z = torch.empty_like(rd)
                        pc.apply(rd, z, nrhs=R)
                        return z.cpu().numpy().astype(np.complex128)
                    finally:
                        pc.close()

                apply()  # tunes the LU and this right-hand-side count's block solve by timing
                lu = _keys(gpu_lib, 'lu_factor ', 'real=%d m=%d ' % (real, m))
                bs = _keys(gpu_lib, 'block_solve ', 'prec=%d m=%d ' % (fprec, m), 'nrhs=%d ' % R)
                assert len(lu) == 1 and len(bs) == 1, gpu_lib.autotune_report()
                nbs = _ncand(gpu_lib, bs[0])
                tried = 0
                for ns in (1, 2, 4, 8):
                    for wsub in (32, 16):
                        z = _forced(gpu_lib, lu[0], [ns, wsub], apply)
                        assert z is not None  # m = 384: all eight are candidates
                        err = _rel(z, z_ref)
                        print('%s -> %d %d: apply error %.2e' % (lu[0], ns, wsub, err))
                        assert err < bar
                cands = [[0, 0, rc, 1 << 30] for rc in (1, 2, 4, 8, 16, 32, 64)]
                fp32 = fprec != gpu_lib.VIE_C128
                cands += [[g, nw, 0, 8] for g in (16, 32, 64) for nw in ((8, 16) if fp32 else (4, 8))]
                for c in cands:
                    z = _forced(gpu_lib, bs[0], c, apply)
                    if z is None:
                        continue
                    tried += 1
                    err = _rel(z, z_ref)
                    print('%s -> %s: apply error %.2e' % (bs[0], c, err))
                    assert err < bar
                # 2 right-hand sides: the per-mode solve's candidates; 9: those and the six
                # matrix-core candidates
                assert tried == nbs and (R == 2 or tried > 6), (tried, nbs)
                out += lu + bs
        op.close()
    finally:
        for key in set(out):
            gpu_lib.autotune_set(key, [])
        gpu_lib.autotune(False)


def test_tuned_solve_matches_dense_solution(gpu_lib):
    """64x8x4 guide, 6 right-hand sides, FP64 to 1e-10 with every family tuned by timing."""
    import torch
    cfg = W.CONFIGS[1]
    grid, delta = cfg['grid'], cfg['delta']
    K = OG.generator_octant(grid, KB * delta)
    chi = W.make_chi(cfg)
    M = OCT.contrast_from_chi(chi)
    R = 6
    B = np.tile(M.reshape(-1), 3)[None] * W.device_sources(dict(geometry='waveguide', grid=grid, delta=delta),
                                                            R, 63).reshape(R, -1)
    A = OM.operator_matrix(K, M, grid)
    X_ref = np.linalg.solve(A, B.T).T
    try:
        gpu_lib.autotune(True)
        op = gpu_lib.Operator(grid, delta, KB, chi)
        pc = gpu_lib.Preconditioner(op)
        Bd = _dev(B)
        Xd = torch.zeros_like(Bd)
        st = gpu_lib.solve(op, pc, Bd, Xd, nrhs=R, tol=1e-10)
        pc.close()
        op.close()
    finally:
        gpu_lib.autotune(False)
    rep = gpu_lib.autotune_report()
    assert 'matvec ' in rep and 'block_solve ' in rep and 'lu_factor ' in rep, rep
    X = Xd.cpu().numpy()
    for q in range(R):
        res = np.linalg.norm(B[q] - A @ X[q]) / np.linalg.norm(B[q])
        err = _rel(X[q], X_ref[q])
        print('tuned solve column %d: iters %d, oracle-evaluated residual %.2e, error %.2e'
              % (q, st[q]['iters'], res, err))
        assert st[q]['status'] == 0 and res <= 2e-10 and err < 1e-7
