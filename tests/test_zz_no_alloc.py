"""The allocation-free product (vie_matvec_noalloc) called through the C ABI: its output equals
vie_matvec's on the same inputs, on consecutive calls of shrinking size (the fixed per-GPU
scratch keeps the previous call's contents), and within 1e-10 of the oracle's explicit sums on
the small grids; a product larger than the fixed scratch is refused before any device work."""
import ctypes

import numpy as np
import pytest

from oracle import contrast as OCT
from oracle import generator as OG
from oracle import matvec as OM
from paper_1903_07884_amd import workloads as W

pytestmark = pytest.mark.gpu

KB = W.k_background()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(vie, op, x, nrhs):
    """(vie_matvec result, vie_matvec_noalloc result) on x, both through the raw C ABI."""
    import torch
    lib = vie.load()
    prec = vie.VIE_C128 if x.dtype == torch.complex128 else vie.VIE_C64
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, float('nan'))
    assert lib.vie_matvec(op.h, _ptr(x), _ptr(y_ref), nrhs, prec, _stream()) == 0, lib.vie_last_error()
    st = lib.vie_matvec_noalloc(op.h, _ptr(x), _ptr(y_na), nrhs, prec, _stream())
    assert st == 0, lib.vie_last_error()
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_noalloc_matvec_equals_matvec_on_shrinking_calls(gpu_lib):
    import torch
    vie = gpu_lib
    delta = 50e-9
    cases = []
    # (grid, nrhs, precision, split plane): the second call of each operator is smaller
    for grid, split in (((40, 6, 4), False), ((24, 5, 3), True)):
        K = OG.generator_octant(grid, KB * delta)
        rng = np.random.default_rng(sum(grid))
        nx, ny, nz = grid
        chi = 3.0 + rng.standard_normal((nz, ny, nx)) + 0.2j * rng.standard_normal((nz, ny, nx))
        M = OCT.contrast_from_chi(chi)
        op = vie.Operator(grid, delta, KB, chi, build_c64=True, split_plane=split)
        for nrhs, dtype in ((3, torch.complex128), (1, torch.complex128), (2, torch.complex64), (1, torch.complex64)):
            x = W.random_field((nrhs, 3 * nx * ny * nz), 7 + nrhs)
            xd = torch.from_numpy(x).cuda().to(dtype)
            y_ref, y_na = _both(vie, op, xd, nrhs)
            ref = OM.matvec(K, M, grid, x)
            err = _rel(y_na.astype(np.complex128), ref)
            bar = 1e-10 if dtype == torch.complex128 else 1e-5
            print('noalloc', grid, 'split' if split else 'fused', nrhs, dtype, 'equal to vie_matvec:',
                  bool(np.array_equal(y_na, y_ref)), 'oracle %.2e' % err)
            assert np.array_equal(y_na, y_ref)
            assert err < bar
            cases.append(err)
        op.close()


def test_noalloc_matvec_full_size_and_refusal(gpu_lib):
    """2048x16x8 guide (25 MB of x-spectra per right-hand side): two calls equal vie_matvec's;
    three right-hand sides need more than the fixed scratch and are refused with VIE_EARG."""
    import torch
    vie = gpu_lib
    cfg = W.CONFIGS[2]
    grid = cfg['grid']
    nx, ny, nz = grid
    op = vie.Operator(grid, cfg['delta'], KB, W.make_chi(cfg))
    n = 3 * nx * ny * nz
    for nrhs in (2, 1):
        xd = torch.from_numpy(W.random_field((nrhs, n), 40 + nrhs)).cuda()
        y_ref, y_na = _both(vie, op, xd, nrhs)
        assert np.array_equal(y_na, y_ref)
    lib = vie.load()
    xd = torch.from_numpy(W.random_field((3, n), 43)).cuda()
    yd = torch.empty_like(xd)
    st = lib.vie_matvec_noalloc(op.h, _ptr(xd), _ptr(yd), 3, vie.VIE_C128, _stream())
    assert st == -1 and b'scratch bytes' in lib.vie_last_error()
    torch.cuda.synchronize()
    op.close()
