"""The request scheduler (vie_server_*): results alone and in a mix, merging, cache, budget.

Each result must not depend on what it is solved beside: a request solved alone (one
worker, no merging) and the same request solved while other devices run on other streams,
possibly merged with another request of its own device, agree to 1e-12 (FP64) / 1e-6
(mixed) relative, and every result meets its tolerance.  Merged requests equal the plain
library solve of each request.  Every served result's residual ||M e - (I - M N) x|| / ||M e||
is also evaluated by the oracle (its generator quadrature and FFT reference operator) and
must meet the request's tolerance.
"""
import numpy as np
import pytest

from oracle import contrast as OCT
from oracle import fftref as FR
from oracle import generator as OG
from paper_1903_07884_amd import workloads as W

pytestmark = pytest.mark.gpu

KB = W.k_background()


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _devices():
    """Three small devices: an FP64 guide with the 1-level preconditioner, a mixed-precision
    coupler cross-section, an unpreconditioned random-contrast block."""
    rng = np.random.default_rng(3)
    g1 = (32, 8, 4)
    g2 = (24, 12, 2)
    g3 = (12, 6, 3)
    chi3 = 2.0 + rng.standard_normal(g3[::-1]) + 0.3j * rng.standard_normal(g3[::-1])
    return {
        'guide': dict(grid=g1, voxel_size=50e-9, k_background=KB, chi=W.waveguide(g1), precond=True),
        'coupler': dict(grid=g2, voxel_size=25e-9, k_background=KB,
                        chi=W.coupler(g2, cores=((1, 5), (7, 11))), precond=True,
                        factor_prec=1, mode='mixed'),
        'block': dict(grid=g3, voxel_size=50e-9, k_background=KB, chi=chi3, precond=False),
    }


def _e(dev, nrhs, seed):
    nx, ny, nz = dev['grid']
    return W.random_field((nrhs, 3 * nx * ny * nz), seed)


def _tol(dev):
    return 1e-6 if dev.get('mode') == 'mixed' else 1e-12


_REF = {}


def _oracle_relres(dev, x, e):
    """Residuals of served solutions x [R, 3N] for incident fields e [R, 3N], by the oracle."""
    grid, delta = tuple(dev['grid']), dev['voxel_size']
    key = (grid, delta, dev['chi'].tobytes())
    if key not in _REF:
        K = OG.generator_octant(grid, dev['k_background'] * delta)
        _REF[key] = FR.FftOperator(K, OCT.contrast_from_chi(dev['chi']), grid)
    ref = _REF[key]
    b = np.tile(ref.M.reshape(-1), 3)[None] * np.atleast_2d(e)
    return ref.relres(np.atleast_2d(x), b)


def test_result_is_the_same_alone_and_in_the_mix(gpu_lib):
    devs = _devices()
    # alone: one worker, no merging, one request at a time
    srv = gpu_lib.Server(workers=1, max_batch_rhs=1)
    alone = {}
    for name, dev in devs.items():
        rid = srv.submit(e_inc=_e(dev, 2, 11), tol=1e-10 if dev.get('mode') != 'mixed' else 1e-6, **dev)
        alone[name] = srv.wait(rid)
    srv.close()
    # in the mix: four workers; every device submitted several times, the reference request
    # between others of other devices and one more of its own device (it may be merged)
    srv = gpu_lib.Server(workers=4, max_batch_rhs=64)
    ids = {}
    order = ['block', 'guide', 'coupler', 'guide', 'block', 'coupler', 'guide', 'coupler', 'block']
    seen = {}
    for k, name in enumerate(order):
        dev = devs[name]
        first = name not in seen
        seen[name] = True
        e = _e(dev, 2, 11) if first else _e(dev, 1, 100 + k)
        rid = srv.submit(e_inc=e, tol=1e-10 if dev.get('mode') != 'mixed' else 1e-6, **dev)
        if first:
            ids[name] = rid
        else:
            ids.setdefault(name + '_others', []).append(rid)
    results = {name: srv.wait(rid) for name, rid in ids.items() if not name.endswith('_others')}
    others = [srv.wait(r) for name, rs in ids.items() if name.endswith('_others') for r in rs]
    info = srv.info()
    srv.close()
    for name, dev in devs.items():
        xa, sa, ta = alone[name]
        xm, sm, tm = results[name]
        d = _rel(xm, xa)
        print('serve %s: alone %.1f ms, in the mix %.1f ms (queue %.1f, merged %d, cache hit %d); difference %.2e; '
              'relres %s' % (name, ta['total_ms'], tm['total_ms'], tm['queue_ms'], tm['merged'], tm['cache_hit'], d,
                             [s['relres'] for s in sm]))
        assert d <= _tol(dev)
        assert all(s['status'] == 0 for s in sa + sm)
        assert all(s['relres'] <= (1e-10 if dev.get('mode') != 'mixed' else 1e-6) for s in sm)
        ores = _oracle_relres(dev, xm, _e(dev, 2, 11))
        print('  oracle-evaluated residuals', ores)
        assert np.all(ores <= (1e-10 if dev.get('mode') != 'mixed' else 1e-6) * 1.01)
    assert all(all(s['status'] == 0 for s in st) for _, st, _ in others)
    print('server info', info)
    assert info['completed'] == len(order) and info['queued'] == 0 and info['running'] == 0
    assert info['peak_committed_bytes'] <= info['budget_bytes']


def test_queued_requests_of_one_device_are_merged_and_cached(gpu_lib):
    """One worker busy with a long solve; three requests of another device queue behind it and
    run as one 3-RHS solve, each column equal to the plain library solve of its request."""
    import torch
    devs = _devices()
    slow = dict(devs['guide'])
    slow['grid'] = (64, 8, 4)
    slow['chi'] = W.waveguide((64, 8, 4))
    slow['precond'] = False  # unpreconditioned: many iterations keep the worker busy
    dev = devs['block']
    srv = gpu_lib.Server(workers=1, max_batch_rhs=64)
    r_slow = srv.submit(e_inc=_e(slow, 1, 5), tol=1e-8, **slow)
    es = [_e(dev, 1, 20 + k) for k in range(3)]
    rids = [srv.submit(e_inc=e, tol=1e-10, **dev) for e in es]
    res = [srv.wait(r) for r in rids]
    srv.wait(r_slow)
    # the same device once more: operator from the cache
    r4 = srv.submit(e_inc=es[0], tol=1e-10, **dev)
    x4, _, t4 = srv.wait(r4)
    srv.close()
    merged = [t['merged'] for _, _, t in res]
    print('merged counts', merged, 'second visit cache hit', t4['cache_hit'])
    assert merged == [3, 3, 3]
    assert t4['cache_hit'] == 1
    # plain library solves of each request
    op = gpu_lib.Operator(dev['grid'], dev['voxel_size'], dev['k_background'], dev['chi'])
    for (x, st, _), e in zip(res, es):
        ed = torch.from_numpy(e).cuda()
        b = torch.empty_like(ed)
        op.rhs(ed, b, nrhs=1)
        xd = torch.zeros_like(b)
        gpu_lib.solve(op, None, b, xd, tol=1e-10)
        assert _rel(x, xd.cpu().numpy()) <= 1e-12
        assert st[0]['status'] == 0
        assert _oracle_relres(dev, x, e)[0] <= 1e-10 * 1.01
    assert _rel(x4, res[0][0]) <= 1e-12


def test_budget_admission_and_eviction(gpu_lib):
    devs = _devices()
    srv = gpu_lib.Server(workers=2, hbm_budget=1 << 20)
    with pytest.raises(gpu_lib.VieError) as ei:
        srv.submit(e_inc=_e(devs['guide'], 1, 1), **devs['guide'])
    assert ei.value.status == -6
    with pytest.raises(gpu_lib.VieError) as ei:
        srv.submit(e_inc=_e(devs['guide'], 1, 1), factor_prec=7,
                   **{k: v for k, v in devs['guide'].items() if k != 'factor_prec'})
    assert ei.value.status == -1
    srv.close()
    # a budget that holds one guide request at a time: the others wait, idle entries are evicted
    import ctypes
    lib = gpu_lib.load()
    g = devs['guide']
    nx, ny, nz = g['grid']
    pc = gpu_lib.PcOpts(0, 0, None, 0, 0.0, 0, 0, 0, 0)
    so = gpu_lib.SolveOpts(1e-10, 50, 5000, 0, 0)
    op = gpu_lib.Operator(g['grid'], g['voxel_size'], g['k_background'], g['chi'])
    need = ctypes.c_uint64()
    assert lib.vie_footprint(op.h, ctypes.byref(pc), 1, ctypes.byref(so), ctypes.byref(need)) == 0
    op.close()
    budget = int(1.3 * need.value)  # one request (resident + run) fits; a second needs an eviction
    srv = gpu_lib.Server(workers=2, hbm_budget=budget)
    rids = []
    for k in range(3):  # three different devices (contrast scaled): no cache reuse
        d = dict(g)
        d['chi'] = g['chi'] * (1.0 + 0.1 * k)
        rids.append(srv.submit(e_inc=_e(d, 1, 40 + k), tol=1e-10, **d))
    out = [srv.wait(r) for r in rids]
    info = srv.info()
    srv.close()
    print('budget %d bytes, one request %d; info %s' % (budget, need.value, info))
    assert all(st[0]['status'] == 0 for _, st, _ in out)
    for k, (x, _, _) in enumerate(out):
        d = dict(g)
        d['chi'] = g['chi'] * (1.0 + 0.1 * k)
        assert _oracle_relres(d, x, _e(d, 1, 40 + k))[0] <= 1e-10 * 1.01
    assert info['evictions'] >= 1
    assert info['peak_committed_bytes'] <= budget


def test_continuous_batching_completes_early_and_takes_joiners(gpu_lib):
    """Continuous batching: a solve's right-hand sides are slots.  A request whose columns end
    at the first restart boundary (a zero incident field) completes while its batch-mate goes
    on; a request submitted after the batch was admitted joins the freed slot at a later
    boundary.  Every result equals the plain library solve of its request."""
    import time
    import torch
    devs = _devices()
    busy = devs['block']
    dev = dict(devs['guide'])
    dev['grid'] = (128, 8, 4)
    dev['chi'] = W.waveguide((128, 8, 4))
    dev['precond'] = False  # unpreconditioned, GMRES(10): many restart cycles at 1e-10
    kw = dict(tol=1e-10, restart=10)
    srv = gpu_lib.Server(workers=1, max_batch_rhs=64)
    r_busy = srv.submit(e_inc=_e(busy, 1, 3), tol=1e-10, **busy)
    e_a = np.zeros_like(_e(dev, 1, 0))
    e_b = _e(dev, 1, 51)
    e_c = _e(dev, 1, 52)
    r_a = srv.submit(e_inc=e_a, **kw, **dev)  # queued behind the busy solve with r_b: merged
    r_b = srv.submit(e_inc=e_b, **kw, **dev)
    t0 = time.time()
    while True:  # until the (a, b) solve is admitted
        info = srv.info()
        if info['queued'] == 0 and info['running'] == 1 and srv.done(r_busy):
            break
        assert time.time() - t0 < 60
        time.sleep(0.001)
    r_c = srv.submit(e_inc=e_c, **kw, **dev)
    xa, sa, ta = srv.wait(r_a)
    xb, sb, tb = srv.wait(r_b)
    xc, sc, tc = srv.wait(r_c)
    srv.wait(r_busy)
    while srv.info()['running']:  # the worker's bookkeeping after the last result
        time.sleep(0.001)
    info = srv.info()
    srv.close()
    print('a: %s; b: %s (iters %d); c: %s (iters %d); server %s' % (ta, tb, sb[0]['iters'], tc, sc[0]['iters'], info))
    assert ta['merged'] >= 2 and tb['merged'] >= 2
    assert tc['joined'] == 1 and ta['joined'] == 0 and tb['joined'] == 0
    assert ta['total_ms'] < tb['total_ms']  # a returned while b was still being solved
    assert np.abs(xa).max() == 0.0 and sa[0]['iters'] == 0
    op = gpu_lib.Operator(dev['grid'], dev['voxel_size'], dev['k_background'], dev['chi'])
    for x, st, e in ((xb, sb, e_b), (xc, sc, e_c)):
        ed = torch.from_numpy(e).cuda()
        b = torch.empty_like(ed)
        op.rhs(ed, b, nrhs=1)
        xd = torch.zeros_like(b)
        ref = gpu_lib.solve(op, None, b, xd, tol=1e-10, restart=10)
        assert st[0]['status'] == 0 and st[0]['iters'] == ref[0]['iters']
        assert _rel(x, xd.cpu().numpy()) <= 1e-12
        assert _oracle_relres(dev, x, e)[0] <= 1e-10 * 1.01
    assert info['solves'] == 2  # the busy solve and the (a, b) solve, which c joined


def test_request_joins_a_running_cycle_at_the_next_step(gpu_lib):
    """Joins at Arnoldi-step granularity: a zero-field request merged with b frees its slot at
    once; with one long restart cycle (GMRES(200), unpreconditioned to 1e-10) a request
    submitted while b is being solved takes that slot after the next step, not at b's cycle
    end, so its wait is a small part of b's run.  Both results equal the plain library solve
    (same iterations) and pass the oracle's residual check."""
    import time
    import torch
    devs = _devices()
    busy = devs['block']
    dev = dict(devs['guide'])
    dev['grid'] = (128, 8, 4)
    dev['chi'] = W.waveguide((128, 8, 4))
    dev['precond'] = False
    kw = dict(tol=1e-10, restart=200)
    srv = gpu_lib.Server(workers=1, max_batch_rhs=64)
    r_busy = srv.submit(e_inc=_e(busy, 1, 3), tol=1e-10, **busy)
    e_b, e_c = _e(dev, 1, 81), _e(dev, 1, 82)
    r_a = srv.submit(e_inc=np.zeros_like(e_b), **kw, **dev)  # merged with b behind the busy solve
    r_b = srv.submit(e_inc=e_b, **kw, **dev)
    t0 = time.time()
    while True:  # until the (a, b) solve is admitted
        info = srv.info()
        if info['queued'] == 0 and info['running'] == 1 and srv.done(r_busy):
            break
        assert time.time() - t0 < 60
        time.sleep(0.001)
    time.sleep(0.01)  # b is stepping
    r_c = srv.submit(e_inc=e_c, **kw, **dev)
    srv.wait(r_a)
    xc, sc, tc = srv.wait(r_c)
    xb, sb, tb = srv.wait(r_b)
    srv.wait(r_busy)
    srv.close()
    print('b: %s (iters %d); c: %s (iters %d)' % (tb, sb[0]['iters'], tc, sc[0]['iters']))
    assert tc['joined'] == 1
    assert tc['queue_ms'] < 0.5 * tb['run_ms']
    op = gpu_lib.Operator(dev['grid'], dev['voxel_size'], dev['k_background'], dev['chi'])
    for x, st, e in ((xb, sb, e_b), (xc, sc, e_c)):
        ed = torch.from_numpy(e).cuda()
        b = torch.empty_like(ed)
        op.rhs(ed, b, nrhs=1)
        xd = torch.zeros_like(b)
        ref = gpu_lib.solve(op, None, b, xd, **kw)
        assert st[0]['status'] == 0 and st[0]['iters'] == ref[0]['iters']
        assert _rel(x, xd.cpu().numpy()) <= 1e-12
        assert _oracle_relres(dev, x, e)[0] <= 1e-10 * 1.01
    op.close()


def test_concurrent_solves_share_one_cached_entry(gpu_lib):
    """Requests of one device with different solver settings (so they are neither merged nor
    joined) run at the same time on several workers: they share one cached operator and
    preconditioner (built once), each stream with its own scratch, and every result equals the
    plain library solve of its request and passes the oracle's residual check."""
    import torch
    devs = _devices()
    dev = dict(devs['guide'])
    dev['grid'] = (96, 8, 4)
    dev['chi'] = W.waveguide((96, 8, 4))
    srv = gpu_lib.Server(workers=4, max_batch_rhs=64)
    tols = [1e-10, 1e-11, 2e-11, 5e-11, 1e-10 * 0.7, 3e-11]
    es = [_e(dev, 2, 70 + k) for k in range(len(tols))]
    rids = [srv.submit(e_inc=e, tol=t, **dev) for e, t in zip(es, tols)]
    out = [srv.wait(r) for r in rids]
    info = srv.info()
    srv.close()
    print('shared entry: %s' % info)
    assert info['cached_entries'] == 1 and info['evictions'] == 0
    assert info['shared_runs'] >= 1
    op = gpu_lib.Operator(dev['grid'], dev['voxel_size'], dev['k_background'], dev['chi'])
    pc = gpu_lib.Preconditioner(op)
    for (x, st, _), e, t in zip(out, es, tols):
        ed = torch.from_numpy(e).cuda()
        b = torch.empty_like(ed)
        op.rhs(ed, b, nrhs=2)
        xd = torch.zeros_like(b)
        ref = gpu_lib.solve(op, pc, b, xd, nrhs=2, tol=t)
        assert [q['iters'] for q in st] == [q['iters'] for q in ref]
        assert _rel(x, xd.cpu().numpy()) <= 1e-12
        assert np.all(_oracle_relres(dev, x, e) <= t * 1.01)


def test_admission_returns_cached_blocks_past_the_budget(gpu_lib):
    """With a budget just above one request's footprint, admitting the second device evicts the
    first and, since the blocks the first solve released are still cached for reuse, returns
    them to the driver before building (regression: the cache once filled the device)."""
    import ctypes
    lib = gpu_lib.load()
    g = _devices()['guide']
    pc = gpu_lib.PcOpts(0, 0, None, 0, 0.0, 0, 0, 0, 0)
    so = gpu_lib.SolveOpts(1e-10, 50, 5000, 0, 0)
    op = gpu_lib.Operator(g['grid'], g['voxel_size'], g['k_background'], g['chi'])
    need = ctypes.c_uint64()
    assert lib.vie_footprint(op.h, ctypes.byref(pc), 1, ctypes.byref(so), ctypes.byref(need)) == 0
    op.close()
    budget = int(need.value) + (1 << 20)
    srv = gpu_lib.Server(workers=1, hbm_budget=budget)
    devs = []
    for k in range(2):
        d = dict(g)
        d['chi'] = g['chi'] * (1.0 + 0.2 * k)
        devs.append(d)
    out = []
    for k, d in enumerate(devs):  # one after the other: the first solve's blocks are cached
        out.append(srv.wait(srv.submit(e_inc=_e(d, 1, 90 + k), tol=1e-10, **d)))
    info = srv.info()
    srv.close()
    print('budget %d, one request %d: %s' % (budget, need.value, info))
    assert info['cache_trims'] >= 1 and info['evictions'] >= 1
    assert info['peak_committed_bytes'] <= budget
    for k, (d, (x, st, _)) in enumerate(zip(devs, out)):
        assert st[0]['status'] == 0
        assert _oracle_relres(d, x, _e(d, 1, 90 + k))[0] <= 1e-10 * 1.01


def test_merge_past_the_budget_does_not_hold_the_queue(gpu_lib):
    """Regression: two queued 2-RHS requests of one device whose merged 4-RHS batch exceeds the
    budget (each alone fits), with eight small requests behind the first.  The scheduler once
    kept trying the merged batch at the head of the queue after the head had been overtaken its
    maximum number of times, and nothing was admitted again.  Now merged requests that cannot
    fit are left queued: every request completes, the two 2-RHS requests are never admitted as
    one batch, committed bytes stay within the budget, and every result passes the oracle's
    residual check."""
    import ctypes
    lib = gpu_lib.load()
    devs = _devices()
    g, blk = devs['guide'], devs['block']
    nx, ny, nz = g['grid']
    n3 = 3 * nx * ny * nz
    pc = gpu_lib.PcOpts(0, 0, None, 0, 0.0, 0, 0, 0, 0)
    so = gpu_lib.SolveOpts(1e-10, 50, 5000, 0, 0)
    op = gpu_lib.Operator(g['grid'], g['voxel_size'], g['k_background'], g['chi'])
    fp = {}
    for R in (2, 3):
        need = ctypes.c_uint64()
        assert lib.vie_footprint(op.h, ctypes.byref(pc), R, ctypes.byref(so), ctypes.byref(need)) == 0
        fp[R] = int(need.value)
    op.close()
    # the server adds the incident fields and right-hand sides (2 x 16 bytes per entry) to the
    # footprint: 2 right-hand sides fit, 4 do not
    budget = fp[2] + 2 * 32 * n3 + (fp[3] - fp[2])
    srv = gpu_lib.Server(workers=1, max_batch_rhs=64, hbm_budget=budget)
    # a first request (another guide: its build and solve) keeps the one worker busy while the
    # queue forms
    blocker = dict(g)
    blocker['chi'] = g['chi'] * 1.3
    subs = [(blocker, 1, 1e-12, 200)]
    subs.append((g, 2, 1e-10, 201))
    for k in range(8):  # eight different small devices (contrast scaled): no merging among them
        d = dict(blk)
        d['chi'] = blk['chi'] * (1.0 + 0.05 * k)
        subs.append((d, 1, 1e-10, 210 + k))
    subs.append((g, 2, 1e-10, 202))
    rids = [srv.submit(e_inc=_e(d, R, seed), tol=tol, **d) for d, R, tol, seed in subs]
    out = [srv.wait(r) for r in rids]
    info = srv.info()
    srv.close()
    print('budget %d (2 RHS: %d + %d): %s' % (budget, fp[2], 2 * 32 * n3, info))
    assert info['completed'] == len(subs)
    assert info['peak_committed_bytes'] <= budget
    for (d, R, tol, seed), (x, st, tm) in zip(subs, out):
        assert all(q['status'] == 0 for q in st)
        assert np.all(_oracle_relres(d, x, _e(d, R, seed)) <= tol * 1.01)
    # the second 2-RHS request either ran on its own or joined the first one's slots once those
    # had ended (a join takes freed slots, no new memory); it was never admitted merged with it
    assert out[-1][2]['joined'] == 1 or (out[1][2]['merged'] == 1 and out[-1][2]['merged'] == 1)


def test_submit_rejects_bad_solver_settings(gpu_lib):
    """Solver settings are validated on submit, as vie_solve does (unknown mode, tol, maxit)."""
    g = _devices()['guide']
    srv = gpu_lib.Server(workers=1)
    for kw in (dict(tol=0.0), dict(tol=float('nan')), dict(maxit=0), dict(restart=201)):
        with pytest.raises(gpu_lib.VieError) as ei:
            srv.submit(e_inc=_e(g, 1, 1), **kw, **g)
        assert ei.value.status == -1
    gpu_lib.MODE['bogus'] = 7
    try:
        with pytest.raises(gpu_lib.VieError) as ei:
            srv.submit(e_inc=_e(g, 1, 1), mode='bogus', **{k: v for k, v in g.items() if k != 'mode'})
        assert ei.value.status == -1
    finally:
        del gpu_lib.MODE['bogus']
    srv.close()
