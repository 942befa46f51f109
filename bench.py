"""Time-to-1e-6-residual benchmark of the preconditioned voxel VIE solver on one MI355X.

A step is one complete solve from inputs resident in HBM: operator build
(FP64 generator quadrature + kernel transform), Chan-Olkin preconditioner
setup (Chan table, block assembly, batched LU), right-hand sides b = M e_inc
and right-preconditioned (flexible) GMRES(50) until every right-hand side
reaches a 1e-6 FP64 relative residual.

Default workload: the directional coupler, 1024 x 48 x 8 voxels of 25 nm with
64 right-hand sides (seeded Gaussian sources of varied core, offset,
polarisation and phase), solved in FP64 (complex128 operator, factors and
basis).  The same line carries the comparison the metric names: the same 64
right-hand sides solved in mixed precision (complex64 products, bfloat16
factors with one FP32 refinement step, or complex64 factors; FP64 Arnoldi and
true residual), the 4096 x 24 x 8 Bragg grating and the 2048 x 16 x 8 guide
solved both ways, with times as medians of whole steps, iterations, FP64
residuals and each mixed solution's distance to the FP64 one.

Prints one JSON line.  ``value`` is solves per second (1 / time-to-1e-6 of the
whole 64-RHS batch).  Per-kernel durations come from HIP events recorded by the
library on the stream each kernel runs on; ``roofline`` is reported for the
kernel with the largest total time, against the peak of its own arithmetic.
``cpu_baseline`` times the CPU oracle on a bounded sample of the same workload
(the FFT reference operator at full size, the rest sampled) and scales it to
one solve.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
METRIC = "time-to-1e-6 residual, mixed vs FP64 solve; matvec HBM GB/s; p50/p99"


# Sources that define each profiled kernel family (the kernel file and the headers it includes):
# a counter summary applies while these are unchanged.
KERNEL_SOURCES = {
    'block_solve': ('block_solve.hip', 'fft_device.h', 'vie_internal.h'),
}


def kernel_sources_digest(kernel='block_solve'):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, 'paper_1903_07884_amd', 'csrc')
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(csrc, f), 'rb').read())
    return h.hexdigest()[:16]


def good_length(n):
    """Smallest 2^a 3^b 5^c >= n (the circulant period the library uses)."""
    L = max(1, n)
    while True:
        q = L
        for p in (2, 3, 5):
            while q % p == 0:
                q //= p
        if q == 1:
            return L
        L += 1


def algorithmic_models(cfg, info, R, mode, factor='c128', refine=0, iters=0, restart=50):
    """Per-launch algorithmic work of the dominant kernels: (bound, amount, unit).

    block_solve at few right-hand sides: every stored factor read once + rhat in + zhat out
    + the permutation (HBM bytes); from 8 right-hand sides on the solves run on the matrix
    cores and the bound is their FP32 (FP64) rate: 8 m^2 real flops per (mode, rhs) column
    (L and U halves), three times that with one refinement step (two solves + the residual
    product).  matvec: x in, y out and M per right-hand side, plus the octant transform once;
    its plane pass alone: the x-spectra of the cross-section rows in and out, and the transform."""
    nx, ny, nz = cfg['grid']
    N = nx * ny * nz
    v = 16 if mode in ('fp64', 'mixed_pc') else 8   # product vector bytes per complex
    vp = 16 if mode == 'fp64' else 8                # preconditioner vector bytes
    f = {'c128': 16, 'c64': 8, 'bf16': 4}[factor]
    m = info['active_m']     # order of the solved blocks (identity rows of every D_k left out)
    modes = info['modes']
    stored = info['stored_blocks']
    Hx, Hy, Hz = (good_length(2 * n - 1) // 2 + 1 for n in (nx, ny, nz))
    khat = 6 * Hx * Hy * Hz * v
    if R >= 8:
        bs = ('mfma', 8.0 * m * m * modes * R * (3 if refine else 1), 'flops')
    else:
        bs = ('hbm', stored * m * m * f + R * modes * (2 * m * vp + 4 * m), 'bytes')
    models = {'block_solve': bs, 'matvec': ('hbm', R * (3 * N + 3 * N + N) * v + khat, 'bytes')}
    # plane pass of one product: the 3 ny nz rows of every x-frequency's spectra read and
    # written once, and the kernel transform ((x, y) octant with nz real offsets when nz <= 16)
    Px = good_length(2 * nx - 1)
    kplane = 6 * Hx * Hy * nz * v if nz <= 16 else khat
    models['matvec_plane'] = ('hbm', R * 2 * 3 * ny * nz * Px * v + kplane, 'bytes')
    if nz <= 16:
        # the plane pass with the direct z sum is bound by its arithmetic (counters: VALU issue):
        # per (x-frequency, right-hand side) the z coupling, 9 nz^2 complex multiply-adds per
        # y-frequency (8 real flops each), and the forward + inverse y-FFTs of the 3 nz rows
        # (5 Py log2 Py real flops each)
        Py = good_length(2 * ny - 1)
        fl = 9 * nz * nz * Py * 8 + 2 * 3 * nz * 5 * Py * np.log2(Py)
        models['matvec_plane'] = ('alu', R * Px * fl, 'flops')
        models['_plane_bytes'] = R * 2 * 3 * ny * nz * Px * v + kplane
    if iters:
        # Arnoldi step j (index within its cycle), one reduction and one update pass: the
        # reduction reads q_0..q_{j-1}, u_j (j + 1 basis vectors) and w; the update reads the same
        # and writes q_j and u_{j+1} (plus u_{j+1}'s complex64 copy when only the preconditioner
        # runs in complex64).  Average per launch.
        pv = 8 if mode == 'mixed' else 16
        js = [it % restart for it in range(iters)]
        n3 = 3 * N
        extra = 8 if mode == 'mixed_pc' else 0
        models['arnoldi_dots'] = ('hbm', sum(((j + 1) * pv + 16) * n3 * R for j in js) / len(js), 'bytes')
        models['arnoldi_update'] = ('hbm', sum(((j + 3) * pv + 16 + extra) * n3 * R for j in js) / len(js), 'bytes')
    return models


def copy_gbps(dev, nbytes=1 << 30, reps=5):
    """Bytes moved per second by torch's elementwise negation over `nbytes` of float32 (reads
    and writes nbytes each), timed with events on torch's stream; the best of `reps`."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.neg(src, out=dst)
        b.record()
        b.synchronize()
        t = a.elapsed_time(b) * 1e-3
        best = t if best is None else min(best, t)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


WORKLOAD_FILES = {2: 'guide_2048x16x8', 3: 'grating_4096x24x8', 4: 'coupler_1024x48x8', 5: 'disk_160x160x8'}


def counter_traffic(kernel, workload_tag, factor='c128'):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this kernel, workload
    and factor precision, if it matches the sources."""
    prec = {'c128': 'fp64', 'c64': 'c64', 'bf16': 'bf16'}.get(factor, factor)
    path = os.path.join(ROOT, 'profiles', '%s_%s_%s_counters.txt' % (kernel, WORKLOAD_FILES.get(workload_tag, '?'),
                                                                     prec))
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if '=' in line and not line.startswith('#'):
            k, v = line.split('=', 1)
            vals[k.strip()] = v.strip()
    if kernel not in KERNEL_SOURCES or vals.get('kernel_sources') != kernel_sources_digest(kernel):
        return None
    try:
        return float(vals['hbm_bytes_per_launch'])
    except (KeyError, ValueError):
        return None


def serving_bench(vie, n_burst=24, streams=((0.5, 40),), seed=11, workers=4, pool=4, small=False):
    """The request scheduler on a seeded stream of catalogue devices (waveguides, Bragg gratings
    and couplers of 256-8192 voxels along x with cross-sections 16x8-48x8, and the 2 um disk on
    160x160x8; 1-16 right-hand sides; mixed precision with complex64 factors; memory-reduced
    preconditioners from 2048 voxels on, the 2-level one for the disk).  Each device is visited
    once to fill the resident cache; a closed burst of n_burst requests measures the capacity;
    then open-loop Poisson streams at the given fractions of it.  Latency = scheduled arrival ->
    result on the host."""
    import queue as _queue
    import threading

    from paper_1903_07884_amd import workloads as W
    devs = W.serving_devices(small=small)
    kb = W.k_background()
    chis = [W.device_chi(d) for d in devs]
    srcs = [W.device_sources(d, pool, 1000 + i).reshape(pool, -1) for i, d in enumerate(devs)]
    solver = [W.device_solver(d) for d in devs]

    def submit(srv, i, nrhs, k):
        d = devs[i]
        e = srcs[i][[(k + j) % pool for j in range(nrhs)]]
        return srv.submit(d['grid'], d['delta'], kb, chis[i], e, precond=True, factor_prec=vie.VIE_C64,
                          mode='mixed', restart=50, **solver[i])

    def run(srv, stream, label):
        q = _queue.Queue()
        rec = [None] * len(stream)

        def collect():
            for c in range(len(stream)):
                if c:
                    r = rec[k]
                    print('bench: serving %s: %d of %d collected (request %d, %d RHS, %s)'
                          % (label, c, len(stream), k, r['nrhs'],
                             '%.0f ms' % r['lat'] if r['lat'] is not None else 'failed'), file=sys.stderr, flush=True)
                k, rid, late_ms, nrhs = q.get()
                try:
                    _, st, tm = srv.wait(rid)
                except vie.VieError as err:  # a failed request is recorded, not fatal
                    rec[k] = dict(lat=None, queue=None, hit=0, merged=0, joined=0, nrhs=nrhs, ok=False,
                                  error=str(err), done=time.perf_counter())
                    continue
                rec[k] = dict(lat=late_ms + tm['total_ms'], queue=tm['queue_ms'], hit=tm['cache_hit'],
                              merged=tm['merged'], joined=tm['joined'], nrhs=nrhs,
                              ok=all(x['status'] == 0 for x in st),
                              done=time.perf_counter())

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for k, (t, i, nrhs) in enumerate(stream):
            dt = t0 + t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            late = max(0.0, time.perf_counter() - (t0 + t)) * 1000.0
            q.put((k, submit(srv, i, nrhs, k), late, nrhs))
        th.join()
        span = max(r['done'] for r in rec) - t0
        good = [r for r in rec if r['lat'] is not None]
        lat = np.array([r['lat'] for r in good]) if good else np.array([float('nan')])
        return dict(requests=len(rec), failed=len(rec) - len(good),
                    errors=sorted({r['error'] for r in rec if 'error' in r})[:5], seconds=span,
                    requests_per_s=len(good) / span, rhs_per_s=sum(r['nrhs'] for r in good) / span,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_queue_ms=float(np.mean([r['queue'] for r in good])) if good else None,
                    cache_hit_fraction=float(np.mean([r['hit'] for r in rec])),
                    mean_merged=float(np.mean([r['merged'] for r in rec])),
                    joined_fraction=float(np.mean([r['joined'] for r in rec])),
                    all_converged=all(r['ok'] for r in rec))

    vie.autotune(False)
    vie.trim()
    srv = vie.Server(workers=workers, max_batch_rhs=64)
    warm = run(srv, [(0.0, i, 1) for i in range(len(devs))], 'cache fill')
    print('bench: serving cache filled (%d devices, %.2f s)' % (len(devs), warm['seconds']), file=sys.stderr,
          flush=True)
    g = np.random.default_rng(seed)
    burst = run(srv, [(0.0, int(g.integers(0, len(devs))), int(g.integers(1, 17))) for _ in range(n_burst)],
                'burst')
    cap = burst['requests_per_s']
    print('bench: serving capacity %.1f requests/s' % cap, file=sys.stderr, flush=True)
    out = dict(workers=workers, devices=len(devs), capacity_requests_per_s=cap, burst=burst, streams=[])
    for frac, n in streams:
        st = run(srv, W.serving_stream(n, frac * cap, seed + int(100 * frac), ndev=len(devs)),
                 'stream at %.1fx capacity' % frac)
        st['offered_fraction_of_capacity'] = frac
        st['offered_requests_per_s'] = frac * cap
        out['streams'].append(st)
        print('bench: serving stream at %.1fx capacity: p50 %.1f ms, p99 %.1f ms' % (frac, st['p50_ms'], st['p99_ms']),
              file=sys.stderr, flush=True)
    out['server'] = srv.info()
    srv.close()
    out['mix'] = ('catalogue of %d devices (waveguide / Bragg / coupler; n_x %d-%d; cross-sections %dx%d-%dx%d; '
                  '25 nm%s), 1-16 RHS per request, mixed precision with complex64 factors, GMRES(50) to 1e-6 '
                  '(memory-reduced preconditioner from n_x %d on%s)'
                  % (len(devs), min(d['grid'][0] for d in devs if d['geometry'] != 'disk'),
                     max(d['grid'][0] for d in devs if d['geometry'] != 'disk'),
                     min(d['grid'][1] for d in devs if d['geometry'] != 'disk'), devs[0]['grid'][2],
                     max(d['grid'][1] for d in devs if d['geometry'] != 'disk'), devs[0]['grid'][2],
                     '' if small else '; plus the 2 um Si disk on 160x160x8', W.SERVE_REDUCE_FROM_NX,
                     '' if small else '; the disk: 2-level over the modal-average contrast, to 1e-4'))
    return out


def lu_flops(m, nblocks, nb=32):
    """Real flops of the trailing updates of a right-looking LU (8 per complex multiply-add)."""
    f = 0
    for j0 in range(0, m, nb):
        w = min(nb, m - j0)
        rest = m - j0 - w
        f += 8 * rest * rest * w
    return f * nblocks


def workload_plan(cfg, tag):
    """Solver settings per workload: precision mode, preconditioner boxes / homogenisation."""
    nx, ny, nz = cfg['grid']
    if tag == 3:   # Bragg: 16 equal x-segments, real part of the mean contrast, FP32 factors
        seg = nx // 16
        return dict(mode='mixed', homog='realmean', reduce_tol=None, factor='c64',
                    boxes=[(i * seg, 0, 0, seg, ny, nz) for i in range(16)],
                    label='16 x-boxes, real-mean contrast')
    if tag == 4:   # coupler: one box over the full cross-section (contrast is x-invariant),
        # bfloat16 factors with one FP32 refinement step of every block solve
        return dict(mode='mixed', homog='none', reduce_tol=None, boxes=None, factor='bf16',
                    label='full cross-section, BF16 factors + FP32 refinement')
    if tag == 5:   # disk: 2-level circulant (blocks per (x-mode, y-mode) pair), modal-average contrast
        return dict(mode='fp64', homog='mode', reduce_tol=None, boxes=None, levels=2, tol=1e-4, maxit=20000,
                    label='2-level, modal-average contrast (tolerance 1e-4, as the paper reports its disks)')
    return dict(mode='fp64', homog='none', reduce_tol=None, boxes=None, label='full 1-level')


def cpu_baseline(cfg, iters, restarts, R, factor_blocks):
    """The CPU oracle timed on a bounded sample of this workload (about 20-30 s of CPU work),
    scaled to one whole solve of R right-hand sides.

    Measured at full size: the oracle's FFT reference operator (the transform of the embedded
    generator, and one product).  Sampled: the generator quadrature on a few hundred octant
    offsets, T. Chan's weights and the explicit x-DFT on sampled x-sequences, dense LU on two
    blocks, block solves of R right-hand sides on one block, MGS against 4 basis vectors.
    Scaling: generator x N offsets, Chan table x its sequence count, LU x the blocks the
    oracle factorises (every mode), solves x the modes; per iteration R products + one
    preconditioner apply + MGS against the average basis length, plus one product per restart."""
    import scipy.linalg

    from oracle import circulant as OC
    from oracle import contrast as OCT
    from oracle import fftref as FR
    from oracle import generator as OG
    from oracle import gmres as OGM  # noqa: F401  (the solver whose steps are timed)
    from paper_1903_07884_amd import workloads as W

    nx, ny, nz = cfg['grid']
    N = nx * ny * nz
    n3 = 3 * N
    m = 3 * ny * nz
    kappa = W.k_background() * cfg['delta']
    rng = np.random.default_rng(5)
    parts = {}

    def per_call(fn, reps):
        # seconds per call of a small sampled step: one untimed call (library threads and caches
        # warm), then the fastest of `reps` timed calls, since the step is scaled up many times
        fn()
        best = float('inf')
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            best = min(best, time.perf_counter() - t0)
        return best

    # generator: all 6 components on sampled octant offsets
    offs = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(100)]
    offs += [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0)]
    OG._MEMO.clear()
    t = time.perf_counter()
    for d in offs:
        for a, b in OG.COMPONENTS:
            OG.generator_entry(a, b, d, kappa)
    parts['generator'] = (time.perf_counter() - t) / len(offs) * N
    # FFT reference operator at full size: transform of the embedded generator, then products
    K = W.synthetic_generator(cfg['grid'], 3)
    M = OCT.contrast_from_chi(W.make_chi(cfg))
    t = time.perf_counter()
    op = FR.FftOperator(K, M, cfg['grid'])
    parts['kernel_transform'] = time.perf_counter() - t
    x = rng.standard_normal(n3) + 1j * rng.standard_normal(n3)
    op.matvec(x)
    t = time.perf_counter()
    for _ in range(2):
        op.matvec(x)
    t_mv = (time.perf_counter() - t) / 2
    # Chan table: Chan weights + explicit DFT of sampled x-sequences (6 (2ny-1)(2nz-1) in all)
    nseq = 6 * (2 * ny - 1) * (2 * nz - 1)
    F = OC.dft_matrix(nx)
    seq = rng.standard_normal(2 * nx - 1) + 0j
    parts['chan_table'] = per_call(lambda: F @ OC.chan(seq), 20) * nseq
    # LU of sampled blocks (the oracle factorises every mode's block)
    D = np.eye(m) + 0.1 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    lu = scipy.linalg.lu_factor(D)
    parts['lu'] = per_call(lambda: scipy.linalg.lu_factor(D), 2) * factor_blocks
    # preconditioner apply: explicit DFT of sampled lines + block solves of R columns
    r = rng.standard_normal((8, nx)) + 0j
    t_dft = per_call(lambda: r @ F.T, 5) / 8 * m * R * 2
    rhs = rng.standard_normal((m, R)) + 0j
    t_sol = per_call(lambda: scipy.linalg.lu_solve(lu, rhs), 4) * nx
    # modified Gram-Schmidt against an average of 25.5 basis vectors, per right-hand side
    V = rng.standard_normal((4, n3)) + 0j
    w0 = rng.standard_normal(n3) + 0j

    def mgs4():
        w = w0
        for i in range(4):
            w = w - np.vdot(V[i], w) * V[i]
    t_mgs = per_call(mgs4, 3) / 4 * 25.5 * R
    per_iter = R * t_mv + t_dft + t_sol + t_mgs
    setup = sum(parts.values())
    total = setup + iters * per_iter + restarts * R * t_mv
    cores = len(os.sched_getaffinity(0))
    return {
        'value': 1.0 / total, 'unit': 'solves/s', 'cores': cores, 'kind': 'oracle',
        'sample': ('oracle on the %dx%dx%d workload, %d right-hand sides: FFT reference operator built and '
                   'applied at full size (%.2f s per product); generator quadrature on %d of %d offsets, Chan '
                   'weights + explicit DFT on 20 of %d x-sequences, dense LU of 2 of %d blocks, block solves '
                   'of %d columns on 1 of %d modes, MGS on 4 vectors; scaled to one solve with %d iterations '
                   'and %d restarts (the GPU solve\'s counts)'
                   % (nx, ny, nz, R, t_mv, len(offs), N, nseq, factor_blocks, R, nx, iters, restarts)),
        'seconds_estimated': total, 'setup_s': setup, 'per_iteration_s': per_iter, 'product_s': t_mv,
    }


def roofline_of(kern, models, mode, dev, copy=True):
    """Roofline object of the kernel with the largest total time among those with a model."""
    cands = [k for k in kern if kern[k]['total_ms'] > 0]
    if not cands:
        return None
    dom = max(cands, key=lambda k: kern[k]['total_ms'])
    if dom not in models:
        return dict(kernel=dom, bound='alu', achieved=None, peak=FP64_PEAK_TFLOPS, unit='TFLOP/s', frac=None,
                    traffic=None, note='no algorithmic model for this kernel')
    bound, amount, unit, peak = models[dom]
    avg_s = kern[dom]['avg_us'] * 1e-6
    if unit == 'flops_total':
        achieved = amount / (kern[dom]['total_ms'] * 1e-3) / 1e12
        roof = dict(kernel=dom, bound=bound, achieved=achieved, peak=peak, unit='TFLOP/s', frac=achieved / peak,
                    traffic=None, per_step_flops=amount)
    elif unit == 'flops':
        achieved = amount / avg_s / 1e12
        roof = dict(kernel=dom, bound=bound, achieved=achieved, peak=peak, unit='TFLOP/s', frac=achieved / peak,
                    traffic=counter_traffic(dom, models.get('_tag'), models.get('_factor')), per_launch_flops=amount)
        if dom == 'matvec_plane' and '_plane_bytes' in models:
            roof['hbm_gbps_algorithmic'] = models['_plane_bytes'] / avg_s / 1e9
    else:
        achieved = amount / avg_s / 1e9
        roof = dict(kernel=dom, bound=bound, achieved=achieved, peak=HBM_PEAK_GBS, unit='GB/s',
                    frac=achieved / HBM_PEAK_GBS, traffic=counter_traffic(dom, models.get('_tag'), models.get('_factor')),
                    per_launch_bytes=amount)
        if copy:   # context: what a plain device copy reaches on this HBM
            cp = copy_gbps(dev)
            roof.update(copy_gbps=cp, frac_of_copy=achieved / cp)
    roof['avg_us'] = kern[dom]['avg_us']
    roof['launches_per_step'] = kern[dom]['launches']
    return roof


PROFILED = ['generator', 'matvec_xfwd', 'matvec_plane', 'matvec_xinv', 'precond_xfft', 'block_solve',
            'refine_residual', 'precond_ixfft', 'precond_identity_rows', 'lu_panel', 'lu_swap_trsm', 'lu_update',
            'lu_invert_diag', 'arnoldi_dots', 'arnoldi_update']


class Workload:
    """Inputs of one configuration resident on the device, and a step = create + setup + solve."""

    def __init__(self, vie, tag, dev):
        import torch

        from paper_1903_07884_amd import workloads as W
        self.vie, self.tag = vie, tag
        self.cfg = W.CONFIGS[tag]
        self.grid, self.delta = self.cfg['grid'], self.cfg['delta']
        self.kb = W.k_background()
        self.chi_d = torch.from_numpy(W.make_chi(self.cfg)).to(dev)
        self.R = self.cfg['nrhs']
        self.e_d = torch.from_numpy(W.make_sources(self.cfg, tag).reshape(self.R, -1).copy()).to(dev)
        self.b_d = torch.empty_like(self.e_d)
        self.x_d = torch.empty_like(self.e_d)
        self.plan = workload_plan(self.cfg, tag)
        self.stream = torch.cuda.current_stream()

    def step(self, record, mode=None, reduce_tol='default', boxes='default', proxy='product', factor=None,
             keep_zero_rows=False, precond=True, share_tol=0.0, mirror=True, refine=None):
        import torch
        vie, plan, R = self.vie, self.plan, self.R
        mode = mode or plan['mode']
        bxs = plan['boxes'] if boxes == 'default' else boxes
        rt = plan['reduce_tol'] if reduce_tol == 'default' else reduce_tol
        factor = factor or (plan.get('factor', 'c64') if mode in ('mixed', 'mixed_pc') else 'c128')
        fp = {'c128': vie.VIE_C128, 'c64': vie.VIE_C64, 'bf16': vie.VIE_BF16C}[factor]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(self.stream)
        op = vie.Operator(self.grid, self.delta, self.kb, self.chi_d, build_c64=(mode == 'mixed'))
        ev[1].record(self.stream)
        pc = vie.Preconditioner(op, homog=plan['homog'], boxes=bxs, reduce_tol=rt, factor_prec=fp, proxy=proxy,
                                keep_zero_rows=keep_zero_rows, levels=plan.get('levels', 1),
                                share_tol=share_tol, mirror=mirror, refine=refine) if precond else None
        ev[2].record(self.stream)
        op.rhs(self.e_d, self.b_d, nrhs=R)
        st = vie.solve(op, pc, self.b_d, self.x_d, nrhs=R, tol=plan.get('tol', 1e-6), restart=50, mode=mode,
                       maxit=plan.get('maxit', 5000))
        ev[3].record(self.stream)
        info = pc.info() if pc is not None else dict(stored_blocks=0, active_m=0, block_m=0, modes=0)
        if pc is not None:
            pc.close()
        op.close()
        print('bench: c%d %s (%s factors) solve done: %d iterations, relres %.3e'
              % (self.tag, mode, factor, max(q['iters'] for q in st), max(q['relres'] for q in st)),
              file=sys.stderr, flush=True)
        if record is not None:
            torch.cuda.synchronize()
            record.append(dict(create_ms=ev[0].elapsed_time(ev[1]), setup_ms=ev[1].elapsed_time(ev[2]),
                               solve_ms=ev[2].elapsed_time(ev[3]),
                               iters=max(q['iters'] for q in st), restarts=max(q['restarts'] for q in st),
                               relres=max(q['relres'] for q in st),
                               status=max(q['status'] for q in st), info=info, mode=mode, factor=factor,
                               refine=(1 if factor == 'bf16' else 0) if refine is None else refine))
        return st

    def models(self, rec):
        """Algorithmic work of the dominant kernels of a recorded step: name -> (bound, amount,
        unit, peak), the peak that of the kernel's own arithmetic type."""
        mode, factor = rec['mode'], rec['factor']
        mdl = algorithmic_models(self.cfg, rec['info'], self.R, mode, factor, refine=rec['refine'],
                                 iters=rec['iters'])
        out = {'_tag': self.tag, '_factor': factor}
        for k, val in mdl.items():
            if k.startswith('_'):
                out[k] = val
                continue
            bound, amount, unit = val
            peak = HBM_PEAK_GBS
            if bound == 'alu':   # vector units of the product's precision
                peak = FP32_PEAK_TFLOPS if mode == 'mixed' else FP64_PEAK_TFLOPS
            elif unit == 'flops':
                # matrix-core block solves: FP64 operands in FP64 mode; complex64 factors on the FP32
                # units; bfloat16 factors: the off-diagonal products on the BF16 units, while the
                # diagonal tiles and the refinement residual run in FP32 -- priced at the FP32 peak
                # for the whole scope and, separately, at the BF16 peak for its products
                peak = FP64_PEAK_TFLOPS if mode == 'fp64' else FP32_PEAK_TFLOPS
            if unit == 'flops' and factor == 'bf16' and k == 'block_solve':
                # two solves (off-diagonal products on the BF16 units) + the FP32 residual: the time
                # each third of the flops takes at its own peak, summed; one solve alone: the BF16 peak
                peak = (1.0 / ((2.0 / 3.0) / BF16_PEAK_TFLOPS + (1.0 / 3.0) / FP32_PEAK_TFLOPS) if rec['refine']
                        else BF16_PEAK_TFLOPS)
            out[k] = (bound, amount, unit, peak)
        info = rec['info']
        if info.get('stored_blocks'):
            # trailing updates of the batched LU, summed over the step (launches differ in size)
            out['lu_update'] = ('mfma', lu_flops(info['active_m'], info['stored_blocks']), 'flops_total',
                                FP64_PEAK_TFLOPS if factor == 'c128' else FP32_PEAK_TFLOPS)
        return out

    def timed(self, reps, warm, label, **kw):
        """Median over `reps` timed steps (after `warm` untimed ones) with per-kernel timings of the
        last, and the solution's distance to a reference solution if one is set."""
        import torch
        for _ in range(warm):
            self.step(None, **kw)
        torch.cuda.synchronize()
        recs, walls = [], []
        for i in range(reps):
            if i == reps - 1:
                self.vie.profile_begin()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            self.step(recs, **kw)
            torch.cuda.synchronize()
            walls.append(1000.0 * (time.perf_counter() - ta))
        kern = {}
        for nm in PROFILED:
            ms, cnt = self.vie.profile_kernel(nm)
            kern[nm] = dict(total_ms=ms, launches=cnt, avg_us=(1000.0 * ms / cnt) if cnt else None)
        self.vie.profile_end()
        last = recs[-1]
        out = dict(label=label, ms=float(np.median(walls)), ms_all=walls, iterations=last['iters'],
                   restarts=last['restarts'], relres=last['relres'], status=last['status'], precision=last['mode'],
                   factors=last['factor'],
                   breakdown_ms={k: last[k] for k in ('create_ms', 'setup_ms', 'solve_ms')},
                   stored_blocks=last['info']['stored_blocks'], block_order=last['info']['active_m'])
        return out, kern, last


def leg_plan(tag, main_mode):
    """Comparison legs of the default run per workload: (label, kwargs)."""
    if tag == 4:
        legs = [('fp64', dict(mode='fp64')), ('mixed_bf16_refined', dict(mode='mixed', factor='bf16')),
                ('mixed_bf16_unrefined', dict(mode='mixed', factor='bf16', refine=0)),
                ('mixed_c64_factors', dict(mode='mixed', factor='c64')),
                ('mixed_pc_c64_factors', dict(mode='mixed_pc', factor='c64')),
                ('mixed_bf16_reduced_1e-3_centre_proxy', dict(mode='mixed', factor='bf16', reduce_tol=1e-3,
                                                               proxy='centre'))]
    elif tag == 3:
        legs = [('fp64', dict(mode='fp64')), ('mixed_c64_factors', dict(mode='mixed', factor='c64')),
                ('mixed_pc_c64_factors', dict(mode='mixed_pc', factor='c64')),
                ('fp64_single_box', dict(mode='fp64', boxes=None)),
                ('mixed_single_box', dict(mode='mixed', factor='c64', boxes=None)),
                ('mixed_pc_single_box', dict(mode='mixed_pc', factor='c64', boxes=None))]
    elif tag == 2:
        legs = [('fp64', dict(mode='fp64')), ('mixed_c64_factors', dict(mode='mixed', factor='c64')),
                ('mixed_pc_c64_factors', dict(mode='mixed_pc', factor='c64')),
                ('fp64_reduced_1e-3', dict(mode='fp64', reduce_tol=1e-3)),
                ('fp64_reduced_1e-3_centre_proxy', dict(mode='fp64', reduce_tol=1e-3, proxy='centre'))]
    elif tag == 5:
        legs = [('fp64', dict(mode='fp64')), ('unpreconditioned', dict(mode='fp64', precond=False))]
    else:
        legs = [('fp64', dict(mode='fp64')), ('unpreconditioned', dict(mode='fp64', precond=False))]
    return [l for l in legs if l[0] != main_mode]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--config', type=int, default=4,
                    help='workload of the timed steps (4: the 1024x48x8 coupler with 64 right-hand sides)')
    ap.add_argument('--precision', choices=('fp64', 'mixed', 'mixed_pc'), default='fp64',
                    help='precision of the timed steps (the other one is a comparison leg)')
    ap.add_argument('--legs', default='4,3,2',
                    help='workloads whose FP64 / mixed comparison legs the line carries ("" = none)')
    ap.add_argument('--leg-reps', type=int, default=3)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-compare', action='store_true', help='same as --legs ""')
    ap.add_argument('--no-autotune', action='store_true',
                    help='default launch parameters (otherwise the warm-up step autotunes them)')
    ap.add_argument('--copy-probe', type=int, default=0,
                    help='also run one plain device copy of this many bytes (calibrates HBM counters)')
    ap.add_argument('--no-serving', action='store_true', help='skip the short serving-stream measurement')
    ap.add_argument('--serve', action='store_true',
                    help='only the serving stream: Poisson arrivals at 0.5, 0.8 and 1.0 of the measured '
                         'capacity, 150 requests each (one JSON line)')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py runs on one GPU only (--gpus %d requested); sharding over several GPUs is '
              'a design note, not an implementation' % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_07884_amd import vie

    vie.load()
    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    if args.serve:
        t0 = time.perf_counter()
        sv = serving_bench(vie, n_burst=40, streams=((0.5, 150), (0.8, 150), (1.0, 150)))
        t1 = time.perf_counter()
        s08 = [x for x in sv['streams'] if x['offered_fraction_of_capacity'] == 0.8][0]
        print(json.dumps({
            'metric': 'serving latency p50/p99 (arrival -> result) and throughput on a seeded request stream',
            'value': s08['requests_per_s'], 'unit': 'requests/s', 'n_gpus': 1, 'steps': 1, 'warmup': 0,
            'ms_per_step': 1000.0 * (t1 - t0), 'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
            'dtype': 'c64+f64', 'data': 'synthetic',
            'config': {'workload': 'serving stream: ' + sv['mix'], 'workers': sv['workers']},
            'p50_ms': s08['p50_ms'], 'p99_ms': s08['p99_ms'], 'serving': sv}))
        return

    if args.copy_probe:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    wl = Workload(vie, args.config, dev)
    main_kw = dict(mode=args.precision)
    if args.precision != 'fp64':
        main_kw['factor'] = wl.plan.get('factor', 'c64')
    vie.autotune(not args.no_autotune)
    for _ in range(max(args.warmup, 0 if args.no_autotune else 1)):
        wl.step(None, **main_kw)
    torch.cuda.synchronize()
    vie.profile_begin()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step(recs, **main_kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    for nm in PROFILED:
        ms, cnt = vie.profile_kernel(nm)
        kern[nm] = dict(total_ms=ms / args.steps, launches=cnt // args.steps,
                        avg_us=(1000.0 * ms / cnt) if cnt else None)
    vie.profile_end()
    ms_per_step = 1000.0 * (t1 - t0) / args.steps
    last = recs[-1]
    x_main = wl.x_d.clone()
    per_step = sorted(r['create_ms'] + r['setup_ms'] + r['solve_ms'] for r in recs)
    latency = dict(p50=float(np.percentile(per_step, 50)), p99=float(np.percentile(per_step, 99)),
                   samples=len(per_step), what='create + setup + solve per step, HIP events')
    models = wl.models(last)
    roof = roofline_of(kern, models, last['mode'], dev, copy=not args.copy_probe)
    mv_us = sum(kern[k]['avg_us'] or 0 for k in ('matvec_xfwd', 'matvec_plane', 'matvec_xinv'))
    info = last['info']

    # comparison legs: the same workloads solved in the other precision / with other preconditioner
    # settings, each timed as a median of whole steps outside the main timed region
    compare, ratios = {}, {}
    legs = [] if args.no_compare else [int(t) for t in args.legs.split(',') if t.strip()]
    warm_leg = 0 if args.no_autotune else 1
    for tag in legs:
        w = wl if tag == args.config else Workload(vie, tag, dev)
        res = {}
        ref_x = x_main if tag == args.config and args.precision == 'fp64' else None
        main_label = args.precision if tag == args.config else None
        for label, kw in leg_plan(tag, main_label):
            # the 4096x24x8 grating's legs take seconds each: one timed run
            reps = args.leg_reps if tag != 3 else 1
            out, lk, lrec = w.timed(reps, warm_leg, label, **kw)
            lroof = roofline_of(lk, w.models(lrec), lrec['mode'], dev, copy=False)
            out['dominant_kernel'] = lroof
            if label == 'fp64' and ref_x is None:
                ref_x = w.x_d.clone()
            if ref_x is not None and label != 'fp64':
                # distance of this leg's solution to the FP64 solve's (each column, the largest)
                d = (w.x_d - ref_x).reshape(w.R, -1)
                out['error_vs_fp64_solution'] = float((d.norm(dim=1) / ref_x.reshape(w.R, -1).norm(dim=1)).max())
            res[label] = out
        if tag == args.config:
            res[args.precision + ' (timed steps)'] = dict(ms=ms_per_step, iterations=last['iters'],
                                                          relres=last['relres'])
        t64 = res['fp64']['ms'] if 'fp64' in res else (ms_per_step if args.precision == 'fp64' and
                                                          tag == args.config else None)
        for label in list(res):
            if not label.startswith('mixed'):
                continue
            rest = label[len('mixed_pc_'):] if label.startswith('mixed_pc_') else label[len('mixed_'):]
            twin = 'fp64_' + rest   # the FP64 leg of the same preconditioner, if any
            ref_ms = res[twin]['ms'] if twin in res else t64
            if ref_ms:
                ratios['c%d %s' % (tag, label)] = ref_ms / res[label]['ms']
        compare['c%d' % tag] = res
        if w is not wl:
            del w
            torch.cuda.empty_cache()
    dtype = {'fp64': 'c128', 'mixed': 'c64+bf16+f64' if last['factor'] == 'bf16' else 'c64+f64',
             'mixed_pc': 'c128+bf16' if last['factor'] == 'bf16' else 'c128+c64'}[last['mode']]
    cfg = wl.cfg
    out = {
        'metric': METRIC,
        'value': 1000.0 / ms_per_step,
        'unit': 'solves/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': ms_per_step,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': dtype,
        'data': 'synthetic',
        'config': {'workload': cfg['name'] + ', %s, %d-level Chan-Olkin %s (%d modes served by %d factorised blocks '
                   'of %dx%d: the %d rows of the %d-row block with nonzero contrast), GMRES(50) to %g; a solve '
                   'is all %d right-hand sides to that residual'
                   % (last['mode'], wl.plan.get('levels', 1), wl.plan['label'], info['modes'],
                      info['stored_blocks'], info['active_m'], info['active_m'], info['active_m'],
                      info['block_m'], wl.plan.get('tol', 1e-6), wl.R),
                   'grid': list(wl.grid), 'voxel_m': wl.delta, 'nrhs': wl.R, 'precision': last['mode']},
        'mixed_vs_fp64': ratios or None,
        'compare': compare or None,
        'time_to_solution_ms': ms_per_step,
        'breakdown_ms': {k: last[k] for k in ('create_ms', 'setup_ms', 'solve_ms')},
        'iterations': last['iters'], 'restarts': last['restarts'], 'relres': last['relres'],
        'matvec_gbps_algorithmic': models['matvec'][1] / (mv_us * 1e-6) / 1e9 if mv_us else None,
        'matvec_us': mv_us,
        'latency_ms': latency,
        'autotune': None if args.no_autotune else vie.autotune_report(),
        'kernels': kern,
        'roofline': roof,
        'kernel_sources': kernel_sources_digest(),
    }
    if not args.no_serving and not args.copy_probe:
        out['serving'] = serving_bench(vie)
    if not args.no_cpu_baseline and not args.copy_probe:
        out['cpu_baseline'] = cpu_baseline(cfg, last['iters'], last['restarts'], wl.R, wl.grid[0])
    print(json.dumps(out))


if __name__ == '__main__':
    main()
