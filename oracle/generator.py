"""Galerkin generator of the voxel JVIE operator (oracle; test infrastructure only).

What is computed
----------------
The Galerkin entries N^{ab}_{ij} = <N p_j^b, p_i^a> (Sec. 2, eq. op_N) for the
orthonormal piecewise-constant voxel basis p_i^a = V^{-1/2} a_hat on voxel i
(Sec. 2), with N f = curl curl int g f and g(R) = exp(-j k R)/(4 pi R) (Sec. 2,
definition of the operator N; time convention exp(j w t)).

Reading (the paper cites the method for these integrals but does not give
it): since curl curl = grad div - Laplacian and (Laplacian + k^2) g = -delta,
N = I + (k^2 + grad div) G, so N^{ab}(d) = delta_ab delta_d0 + K^{ab}(d) with,
after integrating grad div by parts onto voxel faces and scaling lengths by the
voxel edge Delta (kappa = k Delta, offsets d = (i - j) in voxels):

    K^{ab}(d) = kappa^2 delta_ab I3(d) + F^{ab}(d)
    I3(d)     = int_{R^3} g(|t|) L(t_x - d_x) L(t_y - d_y) L(t_z - d_z) dt
    F^{aa}(d) = -[2 J(d_a) - J(d_a + 1) - J(d_a - 1)]      (parallel face pairs)
    J(h)      = int_{R^2} g(sqrt(h^2 + |v|^2)) L(v_1 - d_p) L(v_2 - d_q) dv
    F^{ab}(d) = -sum_{s, s' = +-1} s s' P(d_a + s/2, d_b - s'/2, d_c)   (a != b)
    P(a,b,c)  = int g(|t|) B(t_a - a) B(t_b - b) L(t_c - c) dt

L(s) = max(1 - |s|, 0) is the tent (the overlap length of two unit voxels)
and B the unit box [-1/2, 1/2]; (p, q) are the two axes other than a and c
the axis other than a, b.  g here is the dimensionless kernel
exp(-j kappa rho)/(4 pi rho).

Quadrature: every integral is split at the breakpoints of its weights and at
0 on each axis, so that each piece is either away from the singular point or
has it at a corner.  Pieces away from it use tensor Gauss-Legendre; pieces
with the singular corner are split into pyramids (triangles in 2-D) with the
apex at the origin and mapped by the Duffy transform, which cancels the 1/R
singularity.  The order is raised near the singular point.

Structure (Sec. 2, paragraph after eq. sys_mat): six of the nine blocks are
unique (K^{ab} = K^{ba}); K^{aa} is even in every offset component and
K^{ab} (a != b) is odd in d_a and d_b and even in the third.  The generator
is therefore returned on one octant d >= 0, components ordered
(xx, yy, zz, xy, xz, yz), and extended by these parities.
"""
import numpy as np

COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
_COMP_INDEX = {ab: c for c, ab in enumerate(COMPONENTS)}
_COMP_INDEX.update({(b, a): c for c, (a, b) in enumerate(COMPONENTS)})


def component_index(a, b):
    return _COMP_INDEX[(a, b)]


_RULES = {}


def _unit_rules(p, dim):
    """Unit-cube tensor rule and unit Duffy rule (origin at corner 0) of order p."""
    key = (p, dim)
    if key not in _RULES:
        x, w = np.polynomial.legendre.leggauss(p)
        s, ws = 0.5 * (x + 1.0), 0.5 * w
        grids = np.meshgrid(*([s] * dim), indexing='ij')
        wg = np.ones_like(grids[0])
        for wa in np.meshgrid(*([ws] * dim), indexing='ij'):
            wg = wg * wa
        tens = np.stack([g.reshape(-1) for g in grids], axis=1)
        tw = wg.reshape(-1)
        # Duffy: one pyramid per axis a with apex at the origin and base on the
        # face t_a = 1; t_a = lam, t_b = lam * eta_b, Jacobian lam^(dim-1).
        dpts, dwts = [], []
        lam = tens[:, 0]
        for a in range(dim):
            u = np.zeros_like(tens)
            u[:, a] = lam
            others = [b for b in range(dim) if b != a]
            for k, b in enumerate(others):
                u[:, b] = lam * tens[:, k + 1]
            dpts.append(u)
            dwts.append(tw * lam ** (dim - 1))
        _RULES[key] = (tens, tw, np.concatenate(dpts), np.concatenate(dwts))
    return _RULES[key]


def _kernel(rho, kappa):
    return np.exp(-1j * kappa * rho) / (4.0 * np.pi * rho)


# 1-D weights: ('L', c) tent centred at c, ('B', c) unit box centred at c.
def _support(w):
    kind, c = w
    return (c - 1.0, c + 1.0) if kind == 'L' else (c - 0.5, c + 0.5)


def _breaks(w):
    kind, c = w
    lo, hi = _support(w)
    pts = {lo, hi}
    if kind == 'L':
        pts.add(c)
    if lo < 0.0 < hi:
        pts.add(0.0)
    pts = sorted(pts)
    return list(zip(pts[:-1], pts[1:]))


def _weight(w, t):
    kind, c = w
    if kind == 'L':
        return 1.0 - np.abs(t - c)   # linear on each piece, which lies in the support
    return np.ones_like(t)


def _product(lists):
    if not lists:
        yield []
        return
    for head in lists[0]:
        for rest in _product(lists[1:]):
            yield [head] + rest


def _integrate(weights, kernel, p, p_sing, singular=True):
    """int kernel(t) * prod_a weights[a](t_a) dt over R^dim, piecewise.

    Each piece is a box between breakpoints.  A piece with the singular point
    (the origin) at a corner uses the Duffy rule when ``singular``; every other
    piece uses the tensor Gauss-Legendre rule.  All pieces are evaluated in one
    kernel call.
    """
    dim = len(weights)
    tens, tw, dpts, dwts = _unit_rules(p, dim)
    _, _, dpts_s, dwts_s = _unit_rules(p_sing, dim)
    pts_list, wts_list = [], []
    for pieces in _product([_breaks(w) for w in weights]):
        lo = np.array([a for a, b in pieces])
        hi = np.array([b for a, b in pieces])
        length = hi - lo
        if singular and all(a == 0.0 or b == 0.0 for a, b in pieces):
            sign = np.where(hi > 0.0, 1.0, -1.0)
            pts_list.append(dpts_s * (length * sign))
            wts_list.append(dwts_s * np.prod(length))
        else:
            pts_list.append(lo + tens * length)
            wts_list.append(tw * np.prod(length))
    pts = np.concatenate(pts_list)
    wts = np.concatenate(wts_list)
    f = kernel(pts) * wts
    for a, w in enumerate(weights):
        f = f * _weight(w, pts[:, a])
    return np.sum(f)


def _orders(d):
    """Gauss order by Chebyshev distance of the offset from the singular voxel."""
    r = max(abs(int(v)) for v in d)
    if r <= 2:
        return 14, 14
    if r <= 5:
        return 10, 10
    return 8, 8


def volume_term(d, kappa, order=None):
    """I3(d) = int g(|t|) prod L(t_a - d_a) dt (volume-volume integral / Delta^5)."""
    p, ps = order or _orders(d)
    return _integrate([('L', float(d[0])), ('L', float(d[1])), ('L', float(d[2]))],
                      lambda t: _kernel(np.sqrt(np.sum(t * t, axis=1)), kappa), p, ps)


_MEMO = {}


def face_parallel(h, dp, dq, kappa, order):
    """J(h) = int_{R^2} g(sqrt(h^2+|v|^2)) L(v1-dp) L(v2-dq) dv (two faces normal to one axis).

    J is even in h, dp, dq and symmetric in (dp, dq); values are memoised on that key.
    """
    key = ('J', abs(h), min(abs(dp), abs(dq)), max(abs(dp), abs(dq)), kappa, tuple(order))
    if key not in _MEMO:
        _MEMO[key] = _face_parallel(abs(h), abs(dp), abs(dq), kappa, order)
    return _MEMO[key]


def _face_parallel(h, dp, dq, kappa, order):
    p, ps = order
    h2 = float(h) * float(h)
    if h != 0:
        # smooth integrand: no singular corner even if 0 is a breakpoint
        return _integrate([('L', float(dp)), ('L', float(dq))],
                          lambda v: _kernel(np.sqrt(h2 + np.sum(v * v, axis=1)), kappa), p, ps,
                          singular=False)
    return _integrate([('L', float(dp)), ('L', float(dq))],
                      lambda v: _kernel(np.sqrt(np.sum(v * v, axis=1)), kappa), p, ps)


def face_perpendicular(a, b, ca, cb, cc, kappa, order):
    """P = int g(|t|) B(t_a - ca) B(t_b - cb) L(t_c - cc) dt (face normal to a vs face normal to b).

    P does not depend on which axes a, b, c are, is even in each centre and
    symmetric in (ca, cb); values are memoised on that key.
    """
    key = ('P', min(abs(ca), abs(cb)), max(abs(ca), abs(cb)), abs(cc), kappa, tuple(order))
    if key not in _MEMO:
        _MEMO[key] = _face_perpendicular(0, 1, min(abs(ca), abs(cb)), max(abs(ca), abs(cb)),
                                         abs(cc), kappa, order)
    return _MEMO[key]


def _face_perpendicular(a, b, ca, cb, cc, kappa, order):
    c = 3 - a - b
    weights = [None, None, None]
    weights[a] = ('B', float(ca))
    weights[b] = ('B', float(cb))
    weights[c] = ('L', float(cc))
    p, ps = order
    return _integrate(weights, lambda t: _kernel(np.sqrt(np.sum(t * t, axis=1)), kappa), p, ps)


def grad_div_term(a, b, d, kappa, order=None):
    """F^{ab}(d): the grad-div part of K, as a sum over voxel-face pairs."""
    order = order or _orders(d)
    d = [int(v) for v in d]
    if a == b:
        others = [c for c in range(3) if c != a]
        dp, dq = d[others[0]], d[others[1]]
        J = lambda h: face_parallel(h, dp, dq, kappa, order)
        return -(2.0 * J(d[a]) - J(d[a] + 1) - J(d[a] - 1))
    c = 3 - a - b
    total = 0.0 + 0.0j
    for s in (1, -1):
        for sp in (1, -1):
            total += s * sp * face_perpendicular(a, b, d[a] + 0.5 * s, d[b] - 0.5 * sp, d[c],
                                                 kappa, order)
    return -total


def generator_entry(a, b, d, kappa, order=None):
    """K^{ab}(d) for one signed offset d (N^{ab}(d) = delta_ab delta_d0 + K^{ab}(d))."""
    k = grad_div_term(a, b, d, kappa, order)
    if a == b:
        k += kappa * kappa * volume_term(d, kappa, order)
    return k


def generator_octant(grid, kappa):
    """K on the octant 0 <= d < (nx, ny, nz): array [6, nz, ny, nx] complex128.

    ``grid`` = (nx, ny, nz); ``kappa`` = k_background * Delta.
    """
    nx, ny, nz = grid
    out = np.zeros((6, nz, ny, nx), dtype=np.complex128)
    for dz in range(nz):
        for dy in range(ny):
            for dx in range(nx):
                d = (dx, dy, dz)
                order = _orders(d)
                vol = volume_term(d, kappa, order)
                for c, (a, b) in enumerate(COMPONENTS):
                    val = grad_div_term(a, b, d, kappa, order)
                    if a == b:
                        val += kappa * kappa * vol
                    out[c, dz, dy, dx] = val
    return out


def parity_sign(a, b, d):
    """Sign s with K^{ab}(d) = s K^{ab}(|d|) (Sec. 2: each block symmetric or antisymmetric)."""
    if a == b:
        return 1.0
    s = 1.0
    for axis in (a, b):
        if d[axis] < 0:
            s = -s
    return s


def generator_signed(Koct, a, b, dx, dy, dz):
    """K^{ab} at signed offset arrays (dx, dy, dz) from the octant table."""
    c = component_index(a, b)
    vals = Koct[c][np.abs(dz), np.abs(dy), np.abs(dx)]
    if a != b:
        d = (dx, dy, dz)
        vals = vals * np.where(d[a] < 0, -1.0, 1.0) * np.where(d[b] < 0, -1.0, 1.0)
    return vals
