"""Time-to-1e-6-residual benchmark of the preconditioned voxel VIE solver on one MI355X.

A step is one complete solve from inputs resident in HBM: operator build
(FP64 generator quadrature + kernel transform), 1-level Chan-Olkin
preconditioner setup (Chan table, block assembly, batched LU), right-hand
side b = M e_inc and right-preconditioned GMRES(50) to a 1e-6 relative
residual.  The workload is the long uniform Si waveguide (2048 x 16 x 8 voxels
of 25 nm, complex128, one 384 x 384 block per each of the 2048 modes; the blocks
of modes k > 1024 are S D_{2048-k} S by the reflection symmetry along x, so 1025
are factorised).

Prints one JSON line.  ``value`` is solves per second (1 / time-to-1e-6).
Per-kernel durations come from HIP events recorded by the library on the
stream each kernel runs on; ``roofline`` is reported for the kernel with the
largest total time.  ``cpu_baseline`` times the CPU oracle on a bounded sample
of the same workload and extrapolates to one solve.
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
    v = 16 if mode == 'fp64' else 8      # vector bytes per complex
    f = {'c128': 16, 'c64': 8, 'bf16': 4}[factor]
    m = info['active_m']     # order of the solved blocks (identity rows of every D_k left out)
    modes = info['modes']
    stored = info['stored_blocks']
    Hx, Hy, Hz = (good_length(2 * n - 1) // 2 + 1 for n in (nx, ny, nz))
    khat = 6 * Hx * Hy * Hz * v
    if R >= 8:
        bs = ('mfma', 8.0 * m * m * modes * R * (3 if refine else 1), 'flops')
    else:
        bs = ('hbm', stored * m * m * f + R * modes * (2 * m * v + 4 * m), 'bytes')
    models = {'block_solve': bs, 'matvec': ('hbm', R * (3 * N + 3 * N + N) * v + khat, 'bytes')}
    # plane pass of one product: the 3 ny nz rows of every x-frequency's spectra read and
    # written once, and the kernel transform ((x, y) octant with nz real offsets when nz <= 16)
    Px = good_length(2 * nx - 1)
    kplane = 6 * Hx * Hy * nz * v if nz <= 16 else khat
    models['matvec_plane'] = ('hbm', R * 2 * 3 * ny * nz * Px * v + kplane, 'bytes')
    if iters:
        # CGS2 per Arnoldi step j (index within its cycle): each of the two dot passes reads the
        # j+1 basis vectors and w once; each update pass also writes w.  Average per launch.
        pv = 16 if mode == 'fp64' else 8
        js = [it % restart for it in range(iters)]
        n3 = 3 * N
        models['arnoldi_dots'] = ('hbm', sum(((j + 1) * pv + 16) * n3 * R for j in js) / len(js), 'bytes')
        models['arnoldi_update'] = ('hbm', sum(((j + 1) * pv + 32) * n3 * R for j in js) / len(js), 'bytes')
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


def counter_traffic(kernel, workload_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches the sources."""
    path = os.path.join(ROOT, 'profiles', '%s_c%d_counters.txt' % (kernel, workload_tag))
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


def serving_bench(vie, n_burst=40, streams=((0.8, 120),), seed=11, workers=4, pool=4):
    """The request scheduler on a seeded stream of catalogue devices (waveguides, Bragg gratings,
    couplers; lengths 256-1024; cross-sections 16x8-32x8; 1-16 right-hand sides; mixed precision,
    complex64 factors, 1-level preconditioner).  Each device is visited once to fill the resident
    cache; a closed burst of n_burst requests measures the capacity; then open-loop Poisson streams
    at the given fractions of it.  Latency = scheduled arrival -> result on the host."""
    import queue as _queue
    import threading

    from paper_1903_07884_amd import workloads as W
    devs = W.serving_devices()
    kb = W.k_background()
    chis = [W.device_chi(d) for d in devs]
    srcs = [W.device_sources(d, pool, 1000 + i).reshape(pool, -1) for i, d in enumerate(devs)]

    def submit(srv, i, nrhs, k):
        d = devs[i]
        e = srcs[i][[(k + j) % pool for j in range(nrhs)]]
        return srv.submit(d['grid'], d['delta'], kb, chis[i], e, precond=True,
                          homog='realmean' if d['geometry'] == 'bragg' else 'none', factor_prec=vie.VIE_C64,
                          mode='mixed', tol=1e-6, restart=50)

    def run(srv, stream):
        q = _queue.Queue()
        rec = [None] * len(stream)

        def collect():
            for _ in range(len(stream)):
                k, rid, late_ms, nrhs = q.get()
                _, st, tm = srv.wait(rid)
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
        lat = np.array([r['lat'] for r in rec])
        return dict(requests=len(rec), seconds=span, requests_per_s=len(rec) / span,
                    rhs_per_s=sum(r['nrhs'] for r in rec) / span,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_queue_ms=float(np.mean([r['queue'] for r in rec])),
                    cache_hit_fraction=float(np.mean([r['hit'] for r in rec])),
                    mean_merged=float(np.mean([r['merged'] for r in rec])),
                    joined_fraction=float(np.mean([r['joined'] for r in rec])),
                    all_converged=all(r['ok'] for r in rec))

    vie.autotune(False)
    vie.trim()
    srv = vie.Server(workers=workers, max_batch_rhs=64)
    warm = run(srv, [(0.0, i, 1) for i in range(len(devs))])
    print('bench: serving cache filled (%d devices, %.2f s)' % (len(devs), warm['seconds']), file=sys.stderr,
          flush=True)
    g = np.random.default_rng(seed)
    burst = run(srv, [(0.0, int(g.integers(0, len(devs))), int(g.integers(1, 17))) for _ in range(n_burst)])
    cap = burst['requests_per_s']
    print('bench: serving capacity %.1f requests/s' % cap, file=sys.stderr, flush=True)
    out = dict(workers=workers, devices=len(devs), capacity_requests_per_s=cap, burst=burst, streams=[])
    for frac, n in streams:
        st = run(srv, W.serving_stream(n, frac * cap, seed + int(100 * frac)))
        st['offered_fraction_of_capacity'] = frac
        st['offered_requests_per_s'] = frac * cap
        out['streams'].append(st)
        print('bench: serving stream at %.1fx capacity: p50 %.1f ms, p99 %.1f ms' % (frac, st['p50_ms'], st['p99_ms']),
              file=sys.stderr, flush=True)
    out['server'] = srv.info()
    srv.close()
    out['mix'] = ('catalogue of %d devices (waveguide / Bragg / coupler; n_x 256-1024; cross-sections 16x8-32x8; '
                  '25 nm), 1-16 RHS per request, mixed precision with complex64 factors, GMRES(50) to 1e-6'
                  % len(devs))
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


def cpu_baseline(cfg, iters, restarts, seconds_budget=20.0):
    """Time the oracle on bounded samples of this workload and extrapolate to one solve."""
    import scipy.linalg

    from oracle import circulant as OC
    from oracle import contrast as OCT
    from oracle import generator as OG
    from oracle import matvec as OM
    from paper_1903_07884_amd import workloads as W

    nx, ny, nz = cfg['grid']
    N = nx * ny * nz
    n3 = 3 * N
    m = 3 * ny * nz
    kappa = W.k_background() * cfg['delta']
    rng = np.random.default_rng(5)
    parts = {}
    # generator: all 6 components on sampled octant offsets
    offs = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(150)]
    offs += [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0)]
    OG._MEMO.clear()
    t = time.perf_counter()
    for d in offs:
        for a, b in OG.COMPONENTS:
            OG.generator_entry(a, b, d, kappa)
    parts['generator'] = (time.perf_counter() - t) / len(offs) * N
    # Chan table: Chan weights + explicit DFT of sampled x-sequences (6 (2ny-1)(2nz-1) in all)
    nseq = 6 * (2 * ny - 1) * (2 * nz - 1)
    F = OC.dft_matrix(nx)
    t = time.perf_counter()
    for _ in range(40):
        seq = rng.standard_normal(2 * nx - 1) + 0j
        F @ OC.chan(seq)
    parts['chan_table'] = (time.perf_counter() - t) / 40 * nseq
    # LU of sampled blocks
    D = np.eye(m) + 0.1 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    t = time.perf_counter()
    for _ in range(3):
        lu = scipy.linalg.lu_factor(D)
    parts['lu'] = (time.perf_counter() - t) / 3 * nx
    # matvec by explicit summation: sampled rows
    K = (rng.standard_normal((6, nz, ny, nx)) + 1j * rng.standard_normal((6, nz, ny, nx))) * 1e-3
    M = OCT.contrast_from_chi(W.waveguide(cfg['grid']))
    x = rng.standard_normal(n3) + 1j * rng.standard_normal(n3)
    rows = rng.choice(n3, 300, replace=False)
    t = time.perf_counter()
    OM.matvec_rows(K, M, cfg['grid'], x, rows)
    t_mv = (time.perf_counter() - t) / len(rows) * n3
    # preconditioner apply: DFT of sampled lines + sampled block solves
    r = rng.standard_normal((8, nx)) + 0j
    t = time.perf_counter()
    r @ F.T
    t_dft = (time.perf_counter() - t) / 8 * m * 2
    rhs = rng.standard_normal(m) + 0j
    t = time.perf_counter()
    for _ in range(20):
        scipy.linalg.lu_solve(lu, rhs)
    t_sol = (time.perf_counter() - t) / 20 * nx
    # modified Gram-Schmidt against an average of 25 basis vectors
    V = rng.standard_normal((4, n3)) + 0j
    w = rng.standard_normal(n3) + 0j
    t = time.perf_counter()
    for i in range(4):
        h = np.vdot(V[i], w)
        w = w - h * V[i]
    t_mgs = (time.perf_counter() - t) / 4 * 25.5
    per_iter = t_mv + t_dft + t_sol + t_mgs
    setup = parts['generator'] + parts['chan_table'] + parts['lu']
    total = setup + iters * per_iter + restarts * t_mv
    cores = len(os.sched_getaffinity(0))
    return {
        'value': 1.0 / total, 'unit': 'solves/s', 'cores': cores, 'kind': 'oracle',
        'sample': ('oracle timed on samples of the %dx%dx%d workload and extrapolated: generator on %d '
                   'offsets (of %d), Chan+explicit DFT on 40 of %d x-sequences, dense LU of 3 of %d blocks, '
                   'explicit-sum matvec on 300 of %d rows, explicit DFT on 8 lines, 20 block solves, MGS on '
                   '4 vectors; %d iterations and %d restarts taken from the GPU solve'
                   % (nx, ny, nz, len(offs), N, nseq, nx, n3, iters, restarts)),
        'seconds_estimated': total,
        'setup_s': setup, 'per_iteration_s': per_iter,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--config', type=int, default=2)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-compare', action='store_true',
                    help='skip the comparison solves (FP64 / reduced / other factor precisions)')
    ap.add_argument('--no-autotune', action='store_true',
                    help='default launch parameters (otherwise the warm-up step autotunes them)')
    ap.add_argument('--copy-probe', type=int, default=0,
                    help='also run one plain device copy of this many bytes (calibrates HBM counters)')
    ap.add_argument('--no-serving', action='store_true', help='skip the short serving-stream measurement')
    ap.add_argument('--serve', action='store_true',
                    help='only the serving stream: Poisson arrivals at 0.5, 0.8 and 1.0 of the measured '
                         'capacity, 1000 requests each (one JSON line)')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py runs on one GPU only (--gpus %d requested); sharding over several GPUs is '
              'a design note, not an implementation' % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_07884_amd import vie, workloads as W

    vie.load()
    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    if args.serve:
        t0 = time.perf_counter()
        sv = serving_bench(vie, n_burst=60, streams=((0.5, 1000), (0.8, 1000), (1.0, 1000)))
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
    cfg = W.CONFIGS[args.config]
    grid, delta = cfg['grid'], cfg['delta']
    nx, ny, nz = grid
    kb = W.k_background()
    chi_d = torch.from_numpy(W.make_chi(cfg)).to(dev)
    stream = torch.cuda.current_stream()

    R = cfg['nrhs']
    e_d = torch.from_numpy(W.make_sources(cfg, args.config).reshape(R, -1).copy()).to(dev)
    b_d = torch.empty_like(e_d)
    x_d = torch.empty_like(e_d)
    plan = workload_plan(cfg, args.config)

    def step(record, mode=None, reduce_tol='default', boxes='default', proxy='product', factor=None,
             keep_zero_rows=False, precond=True, share_tol=0.0, mirror=True):
        mode = mode or plan['mode']
        bxs = plan['boxes'] if boxes == 'default' else boxes
        rt = plan['reduce_tol'] if reduce_tol == 'default' else reduce_tol
        factor = factor or (plan.get('factor', 'c64') if mode == 'mixed' else 'c128')
        fp = {'c128': vie.VIE_C128, 'c64': vie.VIE_C64, 'bf16': vie.VIE_BF16C}[factor]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        op = vie.Operator(grid, delta, kb, chi_d, build_c64=(mode == 'mixed'))
        ev[1].record(stream)
        print('bench: operator built', file=sys.stderr, flush=True)
        pc = vie.Preconditioner(op, homog=plan['homog'], boxes=bxs, reduce_tol=rt, factor_prec=fp, proxy=proxy,
                                keep_zero_rows=keep_zero_rows, levels=plan.get('levels', 1),
                                share_tol=share_tol, mirror=mirror) if precond else None
        ev[2].record(stream)
        print('bench: preconditioner set up (%s factors)' % factor, file=sys.stderr, flush=True)
        op.rhs(e_d, b_d, nrhs=R)
        st = vie.solve(op, pc, b_d, x_d, nrhs=R, tol=plan.get('tol', 1e-6), restart=50, mode=mode,
                       maxit=plan.get('maxit', 5000))
        ev[3].record(stream)
        info = pc.info() if pc is not None else dict(stored_blocks=0, active_m=0, block_m=0, modes=0)
        if pc is not None:
            pc.close()
        op.close()
        print('bench: %s solve done: %d iterations, relres %.3e' % (mode, max(q['iters'] for q in st),
                                                                     max(q['relres'] for q in st)),
              file=sys.stderr, flush=True)
        if record is not None:
            torch.cuda.synchronize()
            record.append(dict(create_ms=ev[0].elapsed_time(ev[1]), setup_ms=ev[1].elapsed_time(ev[2]),
                               solve_ms=ev[2].elapsed_time(ev[3]),
                               iters=max(q['iters'] for q in st), restarts=max(q['restarts'] for q in st),
                               relres=max(q['relres'] for q in st),
                               status=max(q['status'] for q in st), info=info, mode=mode, factor=factor))
        return st

    if args.copy_probe:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    vie.autotune(not args.no_autotune)
    for _ in range(max(args.warmup, 0 if args.no_autotune else 1)):
        step(None)
    torch.cuda.synchronize()
    vie.profile_begin()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    names = ['generator', 'matvec_xfwd', 'matvec_plane', 'matvec_xinv', 'precond_xfft', 'block_solve',
             'refine_residual', 'precond_ixfft', 'precond_identity_rows', 'lu_panel', 'lu_swap_trsm', 'lu_update', 'lu_invert_diag', 'arnoldi_dots',
             'arnoldi_update']
    kern = {}
    for nm in names:
        ms, cnt = vie.profile_kernel(nm)
        kern[nm] = dict(total_ms=ms / args.steps, launches=cnt // args.steps,
                        avg_us=(1000.0 * ms / cnt) if cnt else None)
    vie.profile_end()
    ms_per_step = 1000.0 * (t1 - t0) / args.steps
    last = recs[-1]
    per_step = sorted(r['create_ms'] + r['setup_ms'] + r['solve_ms'] for r in recs)
    latency = dict(p50=float(np.percentile(per_step, 50)), p99=float(np.percentile(per_step, 99)),
                   samples=len(per_step), what='create + setup + solve per step, HIP events')
    compare = {}
    if args.no_compare:
        pass
    elif plan['mode'] == 'fp64':
        # every mode factorised (no reflection pairing); memory-reduced 1-level preconditioner
        # (tolerance 1e-3), both readings of the proxy column; the 2-level disk against no
        # preconditioner
        legs = (('full_every_mode_factorised', dict(mirror=False)),
                ('reduced_1e-3', dict(reduce_tol=1e-3)),
                ('reduced_1e-3_centre_proxy', dict(reduce_tol=1e-3, proxy='centre')),
                ('reduced_1e-3_shared_runs_0.01', dict(reduce_tol=1e-3, share_tol=0.01)),
                ('reduced_1e-3_shared_runs_0.05', dict(reduce_tol=1e-3, share_tol=0.05)))
        if plan.get('levels') == 2:
            legs = (('unpreconditioned', dict(precond=False)),)
        for label, kw in legs:
            rr = []
            if not args.no_autotune:   # tune this leg's new shapes outside its timing, like the main run
                step(None, **kw)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            step(rr, **kw)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            compare[label] = dict(ms=1000.0 * (tb - ta), iterations=rr[0]['iters'], relres=rr[0]['relres'],
                                  breakdown_ms={k: rr[0][k] for k in ('create_ms', 'setup_ms', 'solve_ms')},
                                  stored_blocks=rr[0]['info']['stored_blocks'])
    if plan['mode'] == 'mixed' and not args.no_compare:
        # the same problem solved in plain FP64 (and, for the coupler, with the memory-reduced
        # preconditioner), timed the same way, outside the main timed region
        extra = ()
        if args.config == 4:
            extra = (('mixed_c64_factors', dict(factor='c64')),
                     ('mixed_bf16_full_cross_section', dict(keep_zero_rows=True)),
                     ('mixed_reduced_1e-3_centre_proxy', dict(reduce_tol=1e-3, proxy='centre')))
        if args.config == 3:
            extra = (('mixed_single_box', dict(boxes=None)), ('fp64_single_box', dict(mode='fp64', boxes=None)))
        for label, kw in (('fp64', dict(mode='fp64')),) + extra:
            rr = []
            if not args.no_autotune:   # tune this leg's new shapes outside its timing, like the main run
                step(None, **kw)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            step(rr, **kw)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            compare[label] = dict(ms=1000.0 * (tb - ta), iterations=rr[0]['iters'], relres=rr[0]['relres'],
                                  breakdown_ms={k: rr[0][k] for k in ('create_ms', 'setup_ms', 'solve_ms')},
                                  stored_blocks=rr[0]['info']['stored_blocks'],
                                  block_order=rr[0]['info']['active_m'])
        compare['fp64_over_mixed_time'] = compare['fp64']['ms'] / ms_per_step
    info = last['info']
    factor = last['factor']
    models = algorithmic_models(cfg, info, R, plan['mode'], factor, refine=1 if factor == 'bf16' else 0,
                                iters=last['iters'])

    # dominant kernel and its roofline
    dom = max(names, key=lambda k: kern[k]['total_ms'])
    roof = None
    if dom == 'lu_update':
        fl = lu_flops(info['active_m'], info['stored_blocks'])
        launches = max(1, kern[dom]['launches'])
        achieved = fl / (kern[dom]['total_ms'] * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS if plan['mode'] == 'fp64' else FP32_PEAK_TFLOPS
        roof = dict(kernel=dom, bound='alu', achieved=achieved, peak=peak, unit='TFLOP/s',
                    frac=achieved / peak, traffic=None,
                    per_launch_work='%.4g real flops summed over %d launches' % (fl, launches))
    elif dom in models and models[dom][0] == 'mfma':
        _, amount, _ = models[dom]
        achieved = amount / (kern[dom]['avg_us'] * 1e-6) / 1e12
        peak = FP64_PEAK_TFLOPS if plan['mode'] == 'fp64' else FP32_PEAK_TFLOPS
        roof = dict(kernel=dom, bound='mfma', achieved=achieved, peak=peak, unit='TFLOP/s',
                    frac=achieved / peak, traffic=counter_traffic(dom, args.config), per_launch_flops=amount)
    elif dom in models:
        bound, amount, _ = models[dom]
        avg_s = kern[dom]['avg_us'] * 1e-6
        achieved = amount / avg_s / 1e9
        roof = dict(kernel=dom, bound=bound, achieved=achieved, peak=HBM_PEAK_GBS, unit='GB/s',
                    frac=achieved / HBM_PEAK_GBS, traffic=counter_traffic(dom, args.config),
                    per_launch_bytes=amount)
        if not args.copy_probe:  # context: what a plain device copy reaches on this HBM
            cp = copy_gbps(dev)
            roof.update(copy_gbps=cp, frac_of_copy=achieved / cp)
    else:
        roof = dict(kernel=dom, bound='alu', achieved=None, peak=FP64_PEAK_TFLOPS, unit='TFLOP/s', frac=None,
                    traffic=None)
    # matvec GB/s (algorithmic bytes over the three passes of one product)
    mv_us = sum(kern[k]['avg_us'] or 0 for k in ('matvec_xfwd', 'matvec_plane', 'matvec_xinv'))
    mv_bytes = models['matvec'][1]
    bs = kern['block_solve']
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
        'dtype': 'c128' if plan['mode'] == 'fp64' else ('c64+bf16+f64' if factor == 'bf16' else 'c64+f64'),
        'data': 'synthetic',
        'config': {'workload': cfg['name'] + ', %s, %d-level Chan-Olkin %s (%d modes served by %d factorised blocks '
                   'of %dx%d: the %d rows of the %d-row block with nonzero contrast), GMRES(50) to %g'
                   % (plan['mode'], plan.get('levels', 1), plan['label'], info['modes'], info['stored_blocks'],
                      info['active_m'], info['active_m'],
                      info['active_m'], info['block_m'], plan.get('tol', 1e-6)),
                   'grid': list(grid), 'voxel_m': delta, 'nrhs': R, 'precision': plan['mode']},
        'compare': compare or None,
        'time_to_solution_ms': ms_per_step,
        'breakdown_ms': {k: last[k] for k in ('create_ms', 'setup_ms', 'solve_ms')},
        'iterations': last['iters'], 'restarts': last['restarts'], 'relres': last['relres'],
        'matvec_gbps_algorithmic': mv_bytes / (mv_us * 1e-6) / 1e9 if mv_us else None,
        'matvec_us': mv_us,
        'block_solve_rate_algorithmic': (models['block_solve'][1] / (bs['avg_us'] * 1e-6) /
                                         (1e9 if models['block_solve'][0] == 'hbm' else 1e12)) if bs['avg_us'] else None,
        'block_solve_rate_unit': 'GB/s' if models['block_solve'][0] == 'hbm' else 'TFLOP/s',
        'latency_ms': latency,
        'autotune': None if args.no_autotune else vie.autotune_report(),
        'kernels': kern,
        'roofline': roof,
        'kernel_sources': kernel_sources_digest(),
    }
    if not args.no_serving and not args.copy_probe:
        out['serving'] = serving_bench(vie)
    if not args.no_cpu_baseline and args.config == 2:
        out['cpu_baseline'] = cpu_baseline(cfg, last['iters'], last['restarts'])
    print(json.dumps(out))


if __name__ == '__main__':
    main()
