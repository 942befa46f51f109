"""Seeded synthetic inputs: geometries, permittivity contrasts and incident fields.

This module holds no step of the solver's arithmetic.  It produces the inputs
that both the GPU library and the CPU oracle consume:

* the relative contrast chi = eps/eps_b - 1 per voxel ([nz, ny, nx], x fastest),
* incident fields e_inc ([R, 3, nz, ny, nx]),
* the background wavenumber k_b = 2 pi sqrt(eps_b) / lambda0,

for the silicon-photonics geometries the paper studies (Sec. 3, Sec. 5):
uniform Si waveguides in SiO2 cladding, Bragg gratings with an alternating
core width and directional couplers made of two parallel cores.  Material
values follow Table ref_ind (Si 12.1, SiO2 2.085); the operating wavelength is
1550 nm (Sec. 3).  The paper's adiabatic absorbers and dipole-generated beam
come from a cited work and are not reproduced; a Gaussian cross-section with a
propagating phase along x and a seeded global phase stands in for the source.
"""
import numpy as np

SEED = 190307884
LAMBDA0 = 1.55e-6
EPS_SI = 12.11
EPS_SIO2 = 2.085


def k_background(lambda0=LAMBDA0, eps_b=EPS_SIO2):
    return 2.0 * np.pi * np.sqrt(eps_b) / lambda0


def rng(tag):
    return np.random.default_rng([SEED, int(tag)])


def voxel_centres(grid, delta):
    """Centres (x, y, z) in metres; y and z are centred on the box axis."""
    nx, ny, nz = grid
    x = (np.arange(nx) + 0.5) * delta
    y = (np.arange(ny) + 0.5) * delta - 0.5 * ny * delta
    z = (np.arange(nz) + 0.5) * delta - 0.5 * nz * delta
    return x, y, z


def chi_from_mask(mask, eps_core=EPS_SI, eps_b=EPS_SIO2):
    chi = np.zeros(mask.shape, dtype=np.complex128)
    chi[mask] = eps_core / eps_b - 1.0
    return chi


def waveguide(grid, delta=None):
    """Uniform Si core filling the whole box (Sec. 5.1 without absorber)."""
    nx, ny, nz = grid
    return chi_from_mask(np.ones((nz, ny, nx), dtype=bool))


def bragg(grid, delta, w_narrow=0.5e-6, w_wide=0.6e-6, period=0.32e-6):
    """Bragg grating (Sec. 5.2): core width alternates narrow/wide each half period.

    Si where |y| < w(x)/2, w = w_narrow if (x mod period) < period/2 else w_wide,
    sampled at voxel centres, over all z layers.
    """
    nx, ny, nz = grid
    x, y, _ = voxel_centres(grid, delta)
    phase = np.mod(x + 1e-15, period)
    w = np.where(phase < 0.5 * period, w_narrow, w_wide)
    mask2 = np.abs(y)[:, None] < 0.5 * w[None, :]            # [ny, nx]
    return chi_from_mask(np.broadcast_to(mask2, (nz, ny, nx)).copy())


def coupler(grid, cores=((4, 20), (28, 44))):
    """Directional coupler cross-section: Si in the given y-voxel ranges, all z, all x."""
    nx, ny, nz = grid
    mask = np.zeros((nz, ny, nx), dtype=bool)
    for lo, hi in cores:
        mask[:, lo:hi, :] = True
    return chi_from_mask(mask)


def gaussian_source(grid, delta, r, y0=0.0, z0=0.0, wy=0.2e-6, wz=0.1e-6, pol=1,
                    phase=0.0, eps_core=EPS_SI, lambda0=LAMBDA0):
    """e_inc = p_hat exp(-((y-y0)/wy)^2 - ((z-z0)/wz)^2) exp(-j beta x) exp(j phase).

    beta = k0 sqrt(eps_core) (x-propagating under the exp(j w t) convention).
    Returns [3, nz, ny, nx] complex128 with only component ``pol`` non-zero.
    """
    del r
    nx, ny, nz = grid
    x, y, z = voxel_centres(grid, delta)
    beta = 2.0 * np.pi * np.sqrt(eps_core) / lambda0
    prof = np.exp(-((y[None, :, None] - y0) / wy) ** 2 - ((z[:, None, None] - z0) / wz) ** 2)
    wave = np.exp(-1j * beta * x)[None, None, :]
    e = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    e[pol] = prof * wave * np.exp(1j * phase)
    return e


CONFIGS = {
    1: dict(name='uniform Si waveguide 64x8x4 @ 50 nm', grid=(64, 8, 4), delta=50e-9,
            geometry='waveguide', nrhs=1, wy=0.2e-6, wz=0.1e-6),
    2: dict(name='long uniform Si waveguide 2048x16x8 @ 25 nm', grid=(2048, 16, 8), delta=25e-9,
            geometry='waveguide', nrhs=1, wy=0.2e-6, wz=0.1e-6),
    3: dict(name='Si Bragg grating 4096x24x8 @ 25 nm', grid=(4096, 24, 8), delta=25e-9,
            geometry='bragg', nrhs=1, wy=0.25e-6, wz=0.1e-6),
    4: dict(name='Si directional coupler 1024x48x8 @ 25 nm, 64 RHS', grid=(1024, 48, 8),
            delta=25e-9, geometry='coupler', nrhs=64, wy=0.2e-6, wz=0.1e-6),
    5: dict(name='Si disk 160x160x8 @ 25 nm (2 um radius)', grid=(160, 160, 8), delta=25e-9,
            geometry='disk', nrhs=1, wy=0.2e-6, wz=0.1e-6),
}


def make_chi(cfg):
    grid, delta = cfg['grid'], cfg['delta']
    geom = cfg['geometry']
    if geom == 'waveguide':
        return waveguide(grid, delta)
    if geom == 'bragg':
        return bragg(grid, delta)
    if geom == 'coupler':
        return coupler(grid)
    if geom == 'disk':
        return disk(grid, delta, 0.5 * min(grid[0], grid[1]) * delta)
    raise ValueError(geom)


def make_sources(cfg, tag):
    """Seeded incident fields [R, 3, nz, ny, nx] for a configuration."""
    g = rng(tag)
    grid, delta = cfg['grid'], cfg['delta']
    R = cfg['nrhs']
    out = np.zeros((R, 3) + tuple(reversed(grid)), dtype=np.complex128)
    if cfg['geometry'] == 'coupler':
        ny = grid[1]
        centres = [((lo + hi) / 2.0 - ny / 2.0) * delta for lo, hi in ((4, 20), (28, 44))]
        for r in range(R):
            core = int(g.integers(0, 2))
            y0 = centres[core] + g.uniform(-0.1e-6, 0.1e-6)
            z0 = g.uniform(-0.05e-6, 0.05e-6)
            pol = 1 if g.integers(0, 2) == 0 else 2
            ph = g.uniform(0.0, 2.0 * np.pi)
            out[r] = gaussian_source(grid, delta, r, y0=y0, z0=z0, wy=cfg['wy'], wz=cfg['wz'],
                                     pol=pol, phase=ph)
    else:
        for r in range(R):
            ph = g.uniform(0.0, 2.0 * np.pi)
            out[r] = gaussian_source(grid, delta, r, wy=cfg['wy'], wz=cfg['wz'], pol=1, phase=ph)
    return out


def random_field(shape, tag):
    """Seeded complex normal test vector."""
    g = rng(tag)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# ---------------------------------------------------------------- serving stream
SERVE_TYPES = ('waveguide', 'bragg', 'coupler')
SERVE_NX = (256, 512, 1024, 2048, 4096, 8192)
SERVE_CROSS = ((16, 8), (24, 8), (32, 8), (48, 8))
SERVE_DISK = dict(geometry='disk', grid=(160, 160, 8), radius=2e-6)
SERVE_REDUCE_FROM_NX = 2048   # longer devices are served with the memory-reduced preconditioner


def serving_devices(delta=25e-9, small=False):
    """Device catalogue of the serving stream: geometry x length x cross-section (lengths
    256-8192 voxels, cross-sections 16x8 to 48x8 at 25 nm), plus the 2 um Si disk on a
    160x160x8 grid.  small=True keeps lengths up to 1024 and cross-sections up to 32x8 (no
    disk), a catalogue whose every device fits the cache at once."""
    nxs = SERVE_NX[:3] if small else SERVE_NX
    cross = SERVE_CROSS[:3] if small else SERVE_CROSS
    out = [dict(geometry=t, grid=(nx, ny, nz), delta=delta) for t in SERVE_TYPES for nx in nxs for (ny, nz) in cross]
    if not small:
        out.append(dict(SERVE_DISK, delta=delta))
    return out


def device_solver(dev):
    """Solver settings of a catalogue device (mixed precision, complex64 factors, GMRES(50)):
    real-mean homogenisation for gratings; the memory-reduced preconditioner (tolerance 1e-3,
    centre reading of the proxy column) from SERVE_REDUCE_FROM_NX voxels on; the disk with the
    2-level circulant over its modal-average contrast, solved to 1e-4 as the paper reports its
    disks.  Returns keyword settings by name (no arithmetic)."""
    if dev['geometry'] == 'disk':
        return dict(homog='mode', levels=2, tol=1e-4)
    kw = dict(homog='realmean' if dev['geometry'] == 'bragg' else 'none', tol=1e-6)
    if dev['grid'][0] >= SERVE_REDUCE_FROM_NX:
        kw.update(reduce_tol=1e-3, proxy='centre')
    return kw


def coupler_cores(ny):
    """Two cores of width ny/3 with a gap of ny/6 (at least one voxel each), centred in y."""
    c, g = max(1, ny // 3), max(1, ny // 6)
    lo = (ny - 2 * c - g) // 2
    return ((lo, lo + c), (lo + c + g, lo + 2 * c + g))


def device_chi(dev):
    grid, delta = dev['grid'], dev['delta']
    if dev['geometry'] == 'waveguide':
        return waveguide(grid)
    if dev['geometry'] == 'bragg':
        return bragg(grid, delta)
    if dev['geometry'] == 'disk':
        return disk(grid, delta, dev['radius'])
    return coupler(grid, cores=coupler_cores(grid[1]))


def device_sources(dev, count, tag):
    """`count` seeded incident fields [count, 3, nz, ny, nx] for a catalogue device: Gaussian
    cross-section at a random offset (in a random core for couplers), random polarisation
    (y or z) and phase."""
    g = rng(tag)
    grid, delta = dev['grid'], dev['delta']
    ny = grid[1]
    out = np.zeros((count, 3) + tuple(reversed(grid)), dtype=np.complex128)
    for r in range(count):
        if dev['geometry'] == 'coupler':
            lo, hi = coupler_cores(ny)[int(g.integers(0, 2))]
            y0 = ((lo + hi) / 2.0 - ny / 2.0) * delta
        else:
            y0 = 0.0
        y0 += g.uniform(-0.05e-6, 0.05e-6)
        z0 = g.uniform(-0.03e-6, 0.03e-6)
        pol = 1 if g.integers(0, 2) == 0 else 2
        out[r] = gaussian_source(grid, delta, r, y0=y0, z0=z0, wy=0.2e-6, wz=0.1e-6, pol=pol,
                                 phase=g.uniform(0.0, 2.0 * np.pi))
    return out


def serving_stream(n, rate, tag, max_rhs=16, ndev=None):
    """Seeded request stream: Poisson arrivals at `rate` per second, a uniform catalogue device
    (of `ndev`, default the full catalogue) and U{1..max_rhs} right-hand sides per request.
    Returns [(t_arrival_s, device_index, nrhs)]."""
    g = rng(tag)
    ndev = ndev or len(serving_devices())
    t = 0.0
    out = []
    for _ in range(n):
        t += g.exponential(1.0 / rate)
        out.append((t, int(g.integers(0, ndev)), int(g.integers(1, max_rhs + 1))))
    return out


def disk(grid, delta, radius):
    """Si disk of the given radius centred in the (x, y) box, through every z layer (the disk of
    the resonator in Sec. 5.3, without its bus waveguide)."""
    nx, ny, nz = grid
    x = (np.arange(nx) + 0.5) * delta - 0.5 * nx * delta
    y = (np.arange(ny) + 0.5) * delta - 0.5 * ny * delta
    mask2 = (x[None, :] ** 2 + y[:, None] ** 2) < radius ** 2   # [ny, nx]
    return chi_from_mask(np.broadcast_to(mask2, (nz, ny, nx)).copy())


def guide_with_lossy_ends(grid, ramp, loss=0.3):
    """Uniform Si guide whose first and last `ramp` x-voxels carry a growing imaginary part of
    the contrast (a synthetic lossy termination: Im chi falls linearly to -loss at both ends).
    It exercises the complex contrast (mean vs real-mean homogenisation); it is not the paper's
    adiabatic absorber."""
    nx, ny, nz = grid
    chi = waveguide(grid).astype(np.complex128)
    w = np.zeros(nx)
    t = (np.arange(ramp) + 1) / ramp
    w[:ramp] = t[::-1]
    w[nx - ramp:] = t
    chi = chi - 1j * loss * w[None, None, :]
    return chi


def synthetic_generator(grid, tag, scale=5e-3, self_term=-1.0 / 3.0):
    """Seeded stand-in for the octant generator table [6, nz, ny, nx] (components xx, yy, zz,
    xy, xz, yz; offsets d >= 0), for parity checks on grids whose quadrature generator is too
    slow to evaluate on the CPU.  Entries are complex normal, scaled by scale / (1 + |d|)^3 (the
    fall-off of a dipole interaction), the three diagonal components hold `self_term` at zero
    offset, and an off-diagonal component is zero wherever the offset along either of its two
    axes is zero (its block is odd along them, so it vanishes there).  A test input only: it
    holds none of the solver's arithmetic."""
    nx, ny, nz = grid
    K = random_field((6, nz, ny, nx), tag)
    dz, dy, dx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing='ij')
    K *= scale / (1.0 + np.sqrt(dx * dx + dy * dy + dz * dz)) ** 3
    K[0:3, 0, 0, 0] += self_term
    for c, axes in ((3, (0, 1)), (4, (0, 2)), (5, (1, 2))):
        for ax in axes:
            sl = [c, slice(None), slice(None), slice(None)]
            sl[3 - ax] = 0                      # table axes are [z, y, x]
            K[tuple(sl)] = 0.0
    return K
