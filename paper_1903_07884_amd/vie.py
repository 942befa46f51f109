"""Thin ctypes binding of libvie.so (the C ABI declared in include/vie.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device vectors are torch tensors (complex128 or complex64, contiguous, on the
GPU); the current torch stream is passed as the HIP stream.  Host inputs
(contrast, generator, boxes) are numpy arrays.  If the library is missing,
``load`` raises: there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libvie.so')

VIE_C128, VIE_C64, VIE_BF16C = 0, 1, 2
VIE_OK, VIE_NOT_CONVERGED = 0, 1
STATUS = {0: 'VIE_OK', 1: 'VIE_NOT_CONVERGED', -1: 'VIE_EARG', -2: 'VIE_EOOM', -3: 'VIE_EDEVICE',
          -4: 'VIE_ESINGULAR', -5: 'VIE_ENONFINITE', -6: 'VIE_EBUDGET'}
HOMOG = {'none': 0, 'mode': 1, 'mean': 2, 'realmean': 3}
MODE = {'fp64': 0, 'mixed': 1, 'mixed_pc': 2}

EXPORTS = ('vie_create', 'vie_destroy', 'vie_generator', 'vie_rhs', 'vie_matvec', 'vie_matvec_noalloc',
           'precond_setup',
           'precond_info', 'precond_destroy', 'precond_apply', 'vie_solve', 'vie_profile_begin',
           'vie_profile_kernel', 'vie_profile_end', 'vie_last_error', 'vie_footprint', 'vie_autotune',
           'vie_autotune_report', 'vie_autotune_set', 'vie_device_bytes', 'vie_trim', 'vie_server_create', 'vie_server_submit',
           'vie_server_wait', 'vie_server_query', 'vie_server_info_get', 'vie_server_destroy')


class VieError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__('%s: %s' % (STATUS.get(status, status), msg))
        self.status = status


class CreateOpts(ctypes.Structure):
    _fields_ = [('build_c64', ctypes.c_int32), ('generator', ctypes.c_void_p), ('split_plane', ctypes.c_int32)]


class PcOpts(ctypes.Structure):
    _fields_ = [('homog', ctypes.c_int32), ('nboxes', ctypes.c_int32), ('boxes', ctypes.c_void_p),
                ('reduce', ctypes.c_int32), ('reduce_tol', ctypes.c_double), ('factor_prec', ctypes.c_int32),
                ('proxy', ctypes.c_int32), ('refine_steps', ctypes.c_int32), ('keep_zero_rows', ctypes.c_int32),
                ('levels', ctypes.c_int32), ('box_levels', ctypes.c_void_p), ('box_homog', ctypes.c_void_p),
                ('share_tol', ctypes.c_double), ('no_mirror', ctypes.c_int32)]


class PcInfo(ctypes.Structure):
    _fields_ = [('nboxes', ctypes.c_int32), ('box_nx', ctypes.c_int32), ('block_m', ctypes.c_int32),
                ('modes', ctypes.c_int32), ('stored_blocks', ctypes.c_int32), ('factor_bytes', ctypes.c_int64),
                ('active_m', ctypes.c_int32), ('levels', ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [('tol', ctypes.c_double), ('restart', ctypes.c_int32), ('maxit', ctypes.c_int32),
                ('mode', ctypes.c_int32), ('x0_given', ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [('workers', ctypes.c_int32), ('max_batch_rhs', ctypes.c_int32), ('hbm_budget', ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [('grid', ctypes.c_int32 * 3), ('voxel_size', ctypes.c_double), ('k_background', ctypes.c_double),
                ('chi', ctypes.c_void_p), ('e_inc', ctypes.c_void_p), ('nrhs', ctypes.c_int32),
                ('precond', ctypes.c_int32), ('pc', PcOpts), ('solve', SolveOpts)]


class RequestTimes(ctypes.Structure):
    _fields_ = [('queue_ms', ctypes.c_double), ('run_ms', ctypes.c_double), ('total_ms', ctypes.c_double),
                ('cache_hit', ctypes.c_int32), ('merged', ctypes.c_int32), ('joined', ctypes.c_int32)]


class ServerInfo(ctypes.Structure):
    _fields_ = [('submitted', ctypes.c_int64), ('completed', ctypes.c_int64), ('solves', ctypes.c_int64),
                ('cache_hits', ctypes.c_int64), ('evictions', ctypes.c_int64), ('cached_entries', ctypes.c_int32),
                ('queued', ctypes.c_int32), ('running', ctypes.c_int32), ('committed_bytes', ctypes.c_uint64),
                ('peak_committed_bytes', ctypes.c_uint64), ('budget_bytes', ctypes.c_uint64),
                ('shared_runs', ctypes.c_int64), ('cache_trims', ctypes.c_int64)]


class SolveStats(ctypes.Structure):
    _fields_ = [('iters', ctypes.c_int32), ('restarts', ctypes.c_int32), ('relres', ctypes.c_double),
                ('status', ctypes.c_int32)]


_lib = None


def load(path=None):
    """Load libvie.so (raises if it is missing or lacks a declared symbol)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError('libvie.so not built (%s); run paper_1903_07884_amd.build' % path)
    lib = ctypes.CDLL(path)
    for name in EXPORTS:
        getattr(lib, name)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.vie_create.argtypes = [ctypes.POINTER(i32), dbl, dbl, vp, ctypes.POINTER(CreateOpts), vp,
                               ctypes.POINTER(vp)]
    lib.vie_destroy.argtypes = [vp]
    lib.vie_generator.argtypes = [vp, vp]
    lib.vie_rhs.argtypes = [vp, vp, vp, i32, vp]
    lib.vie_matvec.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.vie_matvec_noalloc.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.precond_setup.argtypes = [vp, ctypes.POINTER(PcOpts), vp, ctypes.POINTER(vp)]
    lib.precond_info.argtypes = [vp, ctypes.POINTER(PcInfo)]
    lib.precond_destroy.argtypes = [vp]
    lib.precond_apply.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.vie_solve.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
    lib.vie_profile_begin.argtypes = []
    lib.vie_profile_kernel.argtypes = [ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64)]
    lib.vie_profile_end.argtypes = []
    lib.vie_autotune.argtypes = [i32]
    lib.vie_trim.argtypes = []
    lib.vie_device_bytes.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), i32]
    lib.vie_footprint.argtypes = [vp, ctypes.POINTER(PcOpts), i32, ctypes.POINTER(SolveOpts),
                                  ctypes.POINTER(ctypes.c_uint64)]
    lib.vie_autotune_report.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.vie_autotune_set.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32), i32]
    lib.vie_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.vie_server_submit.argtypes = [vp, ctypes.POINTER(Request), vp, ctypes.POINTER(SolveStats),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.vie_server_wait.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(RequestTimes)]
    lib.vie_server_query.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(i32)]
    lib.vie_server_info_get.argtypes = [vp, ctypes.POINTER(ServerInfo)]
    lib.vie_server_destroy.argtypes = [vp]
    for name in EXPORTS:
        getattr(lib, name).restype = ctypes.c_int
    lib.vie_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, allow=(VIE_OK,)):
    if status not in allow:
        raise VieError(status, _lib.vie_last_error().decode())
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError('expected a contiguous CUDA tensor of %s' % dtype)
    return ctypes.c_void_p(t.data_ptr())


def _prec(t):
    import torch
    return VIE_C128 if t.dtype == torch.complex128 else VIE_C64


class Operator:
    """vie_op: I - M N on a voxel grid (see include/vie.h)."""

    def __init__(self, grid, voxel_size, k_background, chi, build_c64=False, generator=None, split_plane=False,
                 stream=None):
        """``chi``: numpy array (host) or contiguous complex128 CUDA tensor (device), [nz, ny, nx]."""
        lib = load()
        nx, ny, nz = (int(v) for v in grid)
        self.grid = (nx, ny, nz)
        if hasattr(chi, 'is_cuda') and chi.is_cuda:
            import torch
            if chi.numel() != nx * ny * nz:
                raise ValueError('chi has the wrong size')
            chi_ptr = _dev(chi, torch.complex128)
        else:
            chi = np.ascontiguousarray(np.asarray(chi, dtype=np.complex128).reshape(nz, ny, nx))
            chi_ptr = chi.ctypes.data
        g3 = (ctypes.c_int32 * 3)(nx, ny, nz)
        opts = CreateOpts(1 if build_c64 else 0, None, 1 if split_plane else 0)
        if generator is not None:
            gen = np.ascontiguousarray(np.asarray(generator, dtype=np.complex128).reshape(6, nz, ny, nx))
            opts.generator = gen.ctypes.data
        h = ctypes.c_void_p()
        _check(lib.vie_create(g3, float(voxel_size), float(k_background), chi_ptr, ctypes.byref(opts),
                              _stream(stream), ctypes.byref(h)))
        self.h = h

    @property
    def n(self):
        nx, ny, nz = self.grid
        return 3 * nx * ny * nz

    def generator(self):
        nx, ny, nz = self.grid
        out = np.empty((6, nz, ny, nx), dtype=np.complex128)
        _check(_lib.vie_generator(self.h, out.ctypes.data))
        return out

    def rhs(self, e_inc, b, nrhs=1, stream=None):
        import torch
        _check(_lib.vie_rhs(self.h, _dev(e_inc, torch.complex128), _dev(b, torch.complex128), nrhs,
                            _stream(stream)))

    def matvec(self, x, y, nrhs=1, stream=None):
        _check(_lib.vie_matvec(self.h, _dev(x, x.dtype), _dev(y, x.dtype), nrhs, _prec(x), _stream(stream)))

    def matvec_noalloc(self, x, y, nrhs=1, stream=None):
        """The product through the allocation-free entry point (fixed per-GPU scratch)."""
        _check(_lib.vie_matvec_noalloc(self.h, _dev(x, x.dtype), _dev(y, x.dtype), nrhs, _prec(x),
                                       _stream(stream)))

    def close(self):
        if self.h:
            _lib.vie_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Preconditioner:
    """vie_pc: blocked Chan-Olkin circulant preconditioner (see include/vie.h)."""

    def __init__(self, op, homog='none', boxes=None, reduce_tol=None, factor_prec=VIE_C128, proxy='product',
                 refine=None, keep_zero_rows=False, levels=1, share_tol=0.0, mirror=True, stream=None):
        """``factor_prec``: VIE_C128 (FP64 solves), VIE_C64 or VIE_BF16C (mixed-precision
        solves, complex64 vectors); ``proxy``: 'product' or 'centre' reading of the
        memory-reduction proxy column; ``refine``: refinement steps of the bfloat16 block
        solves (default 1 for VIE_BF16C, else 0); ``homog`` and ``levels`` may be lists with
        one entry per box; ``share_tol``: runs of kept modes with close proxy values share one
        block (0 = off); ``keep_zero_rows``: factorise the full
        cross-section even where the homogenised contrast is zero; ``levels``: 1 or 2 (the
        2-level circulant, one 3*bz block per (x-mode, y-mode) pair); ``mirror``: solve the modes
        k > n/2 with the factors of mode n - k through the reflection symmetry along x (and, for
        the 2-level blocks, along y; not with ``share_tol``); False factorises every mode."""
        lib = load()
        self.op = op
        bx = None
        if refine is None:
            refine = 1 if factor_prec == VIE_BF16C else 0
        per_box_h = isinstance(homog, (list, tuple))
        per_box_l = isinstance(levels, (list, tuple))
        o = PcOpts(0 if per_box_h else HOMOG[homog], 0, None, 0, 0.0, factor_prec,
                   {'product': 0, 'centre': 1}[proxy], int(refine), 1 if keep_zero_rows else 0,
                   0 if per_box_l else int(levels))
        if boxes is not None:
            bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
            o.nboxes = bx.shape[0]
            o.boxes = bx.ctypes.data
        o.share_tol = float(share_tol)
        o.no_mirror = 0 if mirror else 1
        self._keep = []
        if per_box_h:
            hb = np.ascontiguousarray([HOMOG[h] for h in homog], dtype=np.int32)
            o.box_homog = hb.ctypes.data
            self._keep.append(hb)
        if per_box_l:
            lb = np.ascontiguousarray(levels, dtype=np.int32)
            o.box_levels = lb.ctypes.data
            self._keep.append(lb)
        if reduce_tol is not None:
            o.reduce = 1
            o.reduce_tol = float(reduce_tol)
        h = ctypes.c_void_p()
        _check(lib.precond_setup(op.h, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.h = h

    def info(self):
        i = PcInfo()
        _check(_lib.precond_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PcInfo._fields_}

    def apply(self, r, z, nrhs=1, stream=None):
        _check(_lib.precond_apply(self.h, _dev(r, r.dtype), _dev(z, r.dtype), nrhs, _prec(r), _stream(stream)))

    def close(self):
        if self.h:
            _lib.precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(op, pc, b, x, nrhs=1, tol=1e-6, restart=50, maxit=5000, mode='fp64', x0_given=False, stream=None):
    """vie_solve; returns a list of per-RHS stats dicts (status VIE_NOT_CONVERGED does not raise).
    ``mode``: 'fp64', 'mixed' (complex64 products and preconditioner) or 'mixed_pc' (complex64
    preconditioner only)."""
    import torch
    lib = load()
    o = SolveOpts(float(tol), int(restart), int(maxit), MODE[mode], 1 if x0_given else 0)
    st = (SolveStats * nrhs)()
    _check(lib.vie_solve(op.h, pc.h if pc is not None else None, _dev(b, torch.complex128),
                         _dev(x, torch.complex128), nrhs, ctypes.byref(o), st, _stream(stream)),
           allow=(VIE_OK, VIE_NOT_CONVERGED))
    return [{f: getattr(s, f) for f, _ in SolveStats._fields_} for s in st]


def footprint(op, nrhs=1, homog='none', boxes=None, reduce_tol=None, factor_prec=None, refine=None,
              restart=50, mode='fp64', solve=True):
    """vie_footprint: upper bound of the device bytes of op + preconditioner (factor_prec not
    None) + one solve of nrhs right-hand sides (solve=True)."""
    lib = load()
    po = None
    bx = None
    if factor_prec is not None:
        if refine is None:
            refine = 1 if factor_prec == VIE_BF16C else 0
        po = PcOpts(HOMOG[homog], 0, None, 0, 0.0, factor_prec, 0, int(refine))
        if boxes is not None:
            bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
            po.nboxes = bx.shape[0]
            po.boxes = bx.ctypes.data
        if reduce_tol is not None:
            po.reduce, po.reduce_tol = 1, float(reduce_tol)
    so = SolveOpts(1e-6, int(restart), 5000, MODE[mode], 0) if solve else None
    out = ctypes.c_uint64()
    _check(lib.vie_footprint(op.h, ctypes.byref(po) if po is not None else None, int(nrhs),
                             ctypes.byref(so) if so is not None else None, ctypes.byref(out)))
    return int(out.value)


def device_bytes(reset_peak=False):
    """(current, peak) device bytes held by the library (vie_device_bytes)."""
    cur, pk = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().vie_device_bytes(ctypes.byref(cur), ctypes.byref(pk), 1 if reset_peak else 0))
    return int(cur.value), int(pk.value)


def trim():
    """Return the library's cache of released device memory to the driver (vie_trim)."""
    _check(load().vie_trim())


def autotune(enable=True):
    """Process-wide switch of the launch-parameter autotuner (vie_autotune)."""
    _check(load().vie_autotune(1 if enable else 0))


def autotune_report():
    """The autotuner cache as text, one 'key -> choice (ms, candidates)' line per shape."""
    lib = load()
    need = ctypes.c_int64()
    _check(lib.vie_autotune_report(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(max(int(need.value), 1))
    _check(lib.vie_autotune_report(buf, len(buf), ctypes.byref(need)))
    return buf.value.decode()


def autotune_set(key, choice):
    """Store `choice` (a sequence of ints; empty removes the entry) under an autotuner key as
    autotune_report prints it (vie_autotune_set)."""
    vals = (ctypes.c_int32 * max(len(choice), 1))(*choice)
    _check(load().vie_autotune_set(key.encode(), vals, len(choice)))


def autotune_entries():
    """The autotuner cache as {key: [values]}."""
    out = {}
    for line in autotune_report().splitlines():
        if ' -> ' not in line:
            continue
        key, rest = line.split(' -> ', 1)
        out[key] = [int(v) for v in rest.split('  (', 1)[0].split()]
    return out


def profile_begin():
    _check(load().vie_profile_begin())


def profile_kernel(name):
    """(total_ms, launches) recorded for one kernel since profile_begin()."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().vie_profile_kernel(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def profile_end():
    _check(load().vie_profile_end())


class Server:
    """vie_server: queue, admission by footprint, resident operator/preconditioner cache and
    worker streams for a stream of solve requests (see include/vie.h)."""

    def __init__(self, workers=4, max_batch_rhs=64, hbm_budget=0):
        lib = load()
        o = ServerOpts(int(workers), int(max_batch_rhs), int(hbm_budget))
        h = ctypes.c_void_p()
        _check(lib.vie_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._pending = {}

    def submit(self, grid, voxel_size, k_background, chi, e_inc, precond=True, homog='none', boxes=None,
               reduce_tol=None, factor_prec=VIE_C128, refine=None, keep_zero_rows=False, tol=1e-6, restart=50,
               maxit=5000, mode='fp64', levels=1, proxy='product', share_tol=0.0, mirror=True):
        """Queue one request; ``chi`` [nz, ny, nx] and ``e_inc`` [nrhs, 3, nz, ny, nx] are host
        arrays (copied).  The preconditioner options are those of ``Preconditioner`` (``homog``
        and ``levels`` may be lists with one entry per box).  Returns the request id;
        ``wait(id)`` returns (x, stats, times)."""
        nx, ny, nz = (int(v) for v in grid)
        chi = np.ascontiguousarray(np.asarray(chi, dtype=np.complex128).reshape(nz, ny, nx))
        e = np.ascontiguousarray(np.asarray(e_inc, dtype=np.complex128).reshape(-1, 3 * nx * ny * nz))
        nrhs = e.shape[0]
        if refine is None:
            refine = 1 if factor_prec == VIE_BF16C else 0
        per_box_h = isinstance(homog, (list, tuple))
        per_box_l = isinstance(levels, (list, tuple))
        pc = PcOpts(0 if per_box_h else HOMOG[homog], 0, None, 0, 0.0, factor_prec,
                    {'product': 0, 'centre': 1}[proxy], int(refine), 1 if keep_zero_rows else 0,
                    0 if per_box_l else int(levels))
        pc.share_tol = float(share_tol)
        pc.no_mirror = 0 if mirror else 1
        keep = []
        bx = None
        if boxes is not None:
            bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
            pc.nboxes = bx.shape[0]
            pc.boxes = bx.ctypes.data
        if per_box_h:
            hb = np.ascontiguousarray([HOMOG[h] for h in homog], dtype=np.int32)
            pc.box_homog = hb.ctypes.data
            keep.append(hb)
        if per_box_l:
            lb = np.ascontiguousarray(levels, dtype=np.int32)
            pc.box_levels = lb.ctypes.data
            keep.append(lb)
        if reduce_tol is not None:
            pc.reduce, pc.reduce_tol = 1, float(reduce_tol)
        req = Request((ctypes.c_int32 * 3)(nx, ny, nz), float(voxel_size), float(k_background), chi.ctypes.data,
                      e.ctypes.data, nrhs, 1 if precond else 0, pc,
                      SolveOpts(float(tol), int(restart), int(maxit), MODE[mode], 0))
        x = np.empty((nrhs, 3 * nx * ny * nz), dtype=np.complex128)
        st = (SolveStats * nrhs)()
        rid = ctypes.c_int64()
        _check(_lib.vie_server_submit(self.h, ctypes.byref(req), x.ctypes.data, st, ctypes.byref(rid)))
        self._pending[rid.value] = (x, st)
        return rid.value

    def done(self, rid):
        d = ctypes.c_int32()
        _check(_lib.vie_server_query(self.h, int(rid), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, rid):
        """(x [nrhs, 3N], per-RHS stats dicts, times dict); VIE_NOT_CONVERGED does not raise."""
        t = RequestTimes()
        _check(_lib.vie_server_wait(self.h, int(rid), ctypes.byref(t)), allow=(VIE_OK, VIE_NOT_CONVERGED))
        x, st = self._pending.pop(rid)
        return (x, [{f: getattr(s, f) for f, _ in SolveStats._fields_} for s in st],
                {f: getattr(t, f) for f, _ in RequestTimes._fields_})

    def info(self):
        i = ServerInfo()
        _check(_lib.vie_server_info_get(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in ServerInfo._fields_}

    def close(self):
        if self.h:
            _lib.vie_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
