// Galerkin generator of the voxel JVIE operator on the device, FP64.
//
// N^{ab}_{ij} = <N p_j^b, p_i^a> (Sec. 2, eq. op_N) depends only on the voxel
// offset d = i - j (three-level Toeplitz, Sec. 2 after eq. sys_mat).  With
// curl curl = grad div - Laplacian and (Laplacian + k^2) g = -delta, N = I + K,
// K = (k^2 + grad div) G.  Lengths are scaled by the voxel edge, kappa = k Delta,
// g(rho) = exp(-j kappa rho) / (4 pi rho), and L(s) = max(1 - |s|, 0) is the
// overlap length of two unit voxels along one axis.
//
// * Offsets at least two voxels apart along some axis (the support of L^3 then
//   avoids the singular point): the volume form
//       K^{ab}(d) = int (kappa^2 delta_ab + d_a d_b) g(|t|) prod_i L(t_i - d_i) dt
//   with tensor Gauss-Legendre on the 8 unit cells of the support, the order
//   falling with distance.
// * Offsets with every component in {0, 1}: grad div moved onto voxel faces,
//       K^{aa} = kappa^2 I3 - [2 J(d_a) - J(d_a + 1) - J(d_a - 1)]
//       K^{ab} = -sum_{s,s'} s s' P(d_a + s/2, d_b - s'/2, d_c)     (a != b)
//   with I3 the volume integral against L^3, J the parallel-face integral
//   against L^2 at normal distance h, P the perpendicular-face integral against
//   box x box x L; each is split at the breakpoints of its weights and at 0,
//   and pieces with the singular point at a corner use a Duffy transform.
#include <cmath>
#include <mutex>

#include "vie_internal.h"

#define GL_MAXP 24
__constant__ double gl_node[GL_MAXP * (GL_MAXP + 1) / 2];  // nodes on [0,1], order p at p(p-1)/2
__constant__ double gl_wt[GL_MAXP * (GL_MAXP + 1) / 2];

static std::once_flag gl_once;
static vie_status gl_status = VIE_OK;

// Gauss-Legendre nodes/weights on [-1,1] by Newton's method on P_p.
static void gauss_legendre(int p, double *x, double *w) {
    for (int i = 0; i < p; ++i) {
        long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (p + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= p; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (p == 1) { p1 = z; p0 = 1; }
            dp = p * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        long double p0 = 1, p1 = z;
        for (int k = 2; k <= p; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (p == 1) { p1 = z; p0 = 1; }
        dp = p * (z * p1 - p0) / (z * z - 1);
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
    }
}

static vie_status upload_gl() {
    std::call_once(gl_once, [] {
        const int n = GL_MAXP * (GL_MAXP + 1) / 2;
        std::vector<double> xs(n), ws(n);
        for (int p = 1; p <= GL_MAXP; ++p) {
            std::vector<double> x(p), w(p);
            gauss_legendre(p, x.data(), w.data());
            for (int i = 0; i < p; ++i) {
                xs[p * (p - 1) / 2 + i] = 0.5 * (x[i] + 1.0);
                ws[p * (p - 1) / 2 + i] = 0.5 * w[i];
            }
        }
        if (hipMemcpyToSymbol(HIP_SYMBOL(gl_node), xs.data(), sizeof(double) * n) != hipSuccess ||
            hipMemcpyToSymbol(HIP_SYMBOL(gl_wt), ws.data(), sizeof(double) * n) != hipSuccess)
            gl_status = VIE_EDEVICE;
    });
    if (gl_status != VIE_OK) vie_set_error("uploading Gauss-Legendre tables failed");
    return gl_status;
}

#define GEN_THREADS 256

__device__ __forceinline__ c128 block_sum(c128 v, c128 *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = GEN_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    c128 r = red[0];
    __syncthreads();
    return r;
}

// far field order by Chebyshev distance D >= 2
// The integrand's nearest complex singularity sits about 2D unit cells away, so the
// tensor rule error falls like (4D)^(-2p): p = 4 already reaches 1e-16 beyond D = 24.
__device__ __forceinline__ int far_order(int D) {
    if (D <= 2) return 14;
    if (D <= 3) return 10;
    if (D <= 5) return 8;
    if (D <= 11) return 7;
    if (D <= 23) return 5;
    return 4;
}

// ---- near field: generic piecewise integrator -----------------------------------
struct Wt {
    int kind;  // 0 tent L(t - c), 1 unit box centred at c
    double c;
};

__device__ int wt_breaks(const Wt &w, double *pts) {
    double lo = w.kind == 0 ? w.c - 1.0 : w.c - 0.5;
    double hi = w.kind == 0 ? w.c + 1.0 : w.c + 0.5;
    double cand[4];
    int n = 0;
    cand[n++] = lo;
    cand[n++] = hi;
    if (w.kind == 0) cand[n++] = w.c;
    if (lo < 0.0 && 0.0 < hi) cand[n++] = 0.0;
    // insertion sort + unique
    for (int i = 1; i < n; ++i) {
        double v = cand[i];
        int j = i - 1;
        while (j >= 0 && cand[j] > v) {
            cand[j + 1] = cand[j];
            --j;
        }
        cand[j + 1] = v;
    }
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (m == 0 || cand[i] != pts[m - 1]) pts[m++] = cand[i];
    return m;
}

__device__ __forceinline__ double wt_value(const Wt &w, double t) {
    return w.kind == 0 ? 1.0 - fabs(t - w.c) : 1.0;
}

__device__ __forceinline__ c128 green(double rho, double kappa) {
    double s, c;
    sincos(kappa * rho, &s, &c);
    double f = 1.0 / (4.0 * M_PI * rho);
    return mk(c * f, -s * f);
}

// int kernel * prod weights over R^dim (dim 2: kernel g(sqrt(h2 + |v|^2))).
__device__ c128 integrate(const Wt *w, int dim, double h2, bool singular, double kappa, int p, int ps,
                          c128 *red) {
    double br[3][4];
    int nb[3];
    for (int a = 0; a < dim; ++a) nb[a] = wt_breaks(w[a], br[a]) - 1;
    int npieces = 1;
    for (int a = 0; a < dim; ++a) npieces *= nb[a];
    const double *gx = gl_node + p * (p - 1) / 2, *gw = gl_wt + p * (p - 1) / 2;
    const double *sx = gl_node + ps * (ps - 1) / 2, *sw = gl_wt + ps * (ps - 1) / 2;
    c128 acc = czero<double>();
    for (int pc = 0; pc < npieces; ++pc) {
        double lo[3], hi[3], len[3], sg[3];
        int rem = pc;
        bool corner = singular;
        double jac = 1.0;
        for (int a = 0; a < dim; ++a) {
            int i = rem % nb[a];
            rem /= nb[a];
            lo[a] = br[a][i];
            hi[a] = br[a][i + 1];
            len[a] = hi[a] - lo[a];
            sg[a] = hi[a] > 0.0 ? 1.0 : -1.0;
            jac *= len[a];
            if (!(lo[a] == 0.0 || hi[a] == 0.0)) corner = false;
        }
        int q = corner ? ps : p;
        int npts = 1;
        for (int a = 0; a < dim; ++a) npts *= q;
        int total = corner ? dim * npts : npts;
        for (int t = threadIdx.x; t < total; t += GEN_THREADS) {
            double x[3], wq;
            if (!corner) {
                int r = t;
                wq = jac;
                for (int a = 0; a < dim; ++a) {
                    int i = r % q;
                    r /= q;
                    x[a] = lo[a] + len[a] * gx[i];
                    wq *= gw[i];
                }
            } else {
                // pyramid `ax`: apex at origin, base on the face |t_ax| = len[ax]
                int ax = t / npts, r = t % npts;
                int i0 = r % q;
                r /= q;
                double lam = sx[i0];
                wq = jac * sw[i0] * (dim == 3 ? lam * lam : lam);
                x[ax] = sg[ax] * lam * len[ax];
                for (int a = 0; a < dim; ++a) {
                    if (a == ax) continue;
                    int ii = r % q;
                    r /= q;
                    x[a] = sg[a] * lam * sx[ii] * len[a];
                    wq *= sw[ii];
                }
            }
            double rho2 = h2;
            for (int a = 0; a < dim; ++a) rho2 += x[a] * x[a];
            c128 gv = green(sqrt(rho2), kappa);
            double wv = wq;
            for (int a = 0; a < dim; ++a) wv *= wt_value(w[a], x[a]);
            acc = acc + mk(gv.re * wv, gv.im * wv);
        }
    }
    return block_sum(acc, red);
}

__device__ __forceinline__ c128 wave_sum64(c128 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_down(v.re, off);
        v.im += __shfl_down(v.im, off);
    }
    return v;
}

// Far offsets (some |d_a| >= 2): one wavefront per offset, volume form, all six components.
__global__ void __launch_bounds__(64) k_generator_far(c128 *gen, int nx, int ny, int nz, double kappa) {
    long long N = (long long)nx * ny * nz;
    long long o = blockIdx.x;
    int dx = (int)(o % nx), dy = (int)((o / nx) % ny), dz = (int)(o / ((long long)nx * ny));
    int d[3] = {dx, dy, dz};
    int D = max(dx, max(dy, dz));
    if (D < 2) return;  // near offsets: k_generator_near
    int p = far_order(D);
    const double *gx = gl_node + p * (p - 1) / 2, *gw = gl_wt + p * (p - 1) / 2;
    int p3 = p * p * p;
    c128 acc[6];
    for (int c = 0; c < 6; ++c) acc[c] = czero<double>();
    for (int t = threadIdx.x; t < 8 * p3; t += 64) {
        int cell = t / p3, r = t % p3;
        double x[3], wq = 1.0;
        for (int a = 0; a < 3; ++a) {
            int i = r % p;
            r /= p;
            double lo = d[a] - 1 + ((cell >> a) & 1);
            x[a] = lo + gx[i];
            wq *= gw[i] * (1.0 - fabs(x[a] - d[a]));
        }
        double R2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        double R = sqrt(R2);
        double sn, cs;
        sincos(kappa * R, &sn, &cs);
        double f = wq / (4.0 * M_PI * R2 * R);
        c128 e = mk(cs * f, -sn * f);            // exp(-j kappa R)/(4 pi R^3) * weight
        c128 A = mk(1.0, kappa * R);             // 1 + j kappa R
        double k2R2 = kappa * kappa * R2;
        double rh[3] = {x[0] / R, x[1] / R, x[2] / R};
        for (int a = 0; a < 3; ++a) {            // a == b: e [(3 r_a^2 - 1) A - k2R2 r_a^2 + k2R2]
            double q = 3.0 * rh[a] * rh[a] - 1.0;
            c128 br = mk(q * A.re - k2R2 * rh[a] * rh[a] + k2R2, q * A.im);
            acc[a] = acc[a] + e * br;
        }
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        for (int k = 0; k < 3; ++k) {            // a != b: e r_a r_b (3 A - k2R2)
            double rr = rh[pa[k]] * rh[pb[k]];
            c128 br = mk(rr * (3.0 * A.re - k2R2), rr * 3.0 * A.im);
            acc[3 + k] = acc[3 + k] + e * br;
        }
    }
    for (int c = 0; c < 6; ++c) acc[c] = wave_sum64(acc[c]);
    // off-diagonal blocks are odd in their two axes: exactly zero at zero offset there
    if (dx == 0 || dy == 0) acc[3] = czero<double>();
    if (dx == 0 || dz == 0) acc[4] = czero<double>();
    if (dy == 0 || dz == 0) acc[5] = czero<double>();
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) gen[c * N + o] = acc[c];
}

// Touching offsets d in {0,1}^3 (the support of the overlap weights reaches the singular
// point): face form.  Each offset needs 22 integrals: I3, J(h) for three normal distances per
// axis, and P for four face pairs of each of the three off-diagonal components.  One
// workgroup per (offset, integral) writes its value to parts[offset][22]; k_generator_near
// combines them.
#define NEAR_PARTS 22
__global__ void __launch_bounds__(GEN_THREADS) k_generator_near_parts(c128 *parts, int nx, int ny, int nz,
                                                                      double kappa) {
    __shared__ c128 red[GEN_THREADS];
    const int off = blockIdx.x / NEAR_PARTS, idx = blockIdx.x % NEAR_PARTS;
    const int dx = off & 1, dy = (off >> 1) & 1, dz = (off >> 2) & 1;
    if (dx >= nx || dy >= ny || dz >= nz) return;
    const int d[3] = {dx, dy, dz};
    const int p = 14, ps = 16;
    c128 v;
    if (idx == 0) {  // I3
        Wt w3[3] = {{0, (double)dx}, {0, (double)dy}, {0, (double)dz}};
        v = integrate(w3, 3, 0.0, true, kappa, p, ps, red);
    } else if (idx < 10) {  // J: axis a, normal distance d_a - 1 + k
        const int a = (idx - 1) / 3, k = (idx - 1) % 3;
        const int q0 = (a + 1) % 3, q1 = (a + 2) % 3;
        Wt w2[2] = {{0, (double)d[q0 < q1 ? q0 : q1]}, {0, (double)d[q0 < q1 ? q1 : q0]}};
        const int h = d[a] - 1 + k;
        v = integrate(w2, 2, (double)h * h, h == 0, kappa, p, ps, red);
    } else {  // P: component pair kk, face signs s, s'
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        const int kk = (idx - 10) / 4, si = ((idx - 10) / 2) % 2, spi = (idx - 10) % 2;
        const int a = pa[kk], b = pb[kk], c = 3 - a - b;
        const int sg = si ? -1 : 1, sgp = spi ? -1 : 1;
        Wt w[3];
        w[a] = {1, d[a] + 0.5 * sg};
        w[b] = {1, d[b] - 0.5 * sgp};
        w[c] = {0, (double)d[c]};
        v = integrate(w, 3, 0.0, true, kappa, p, ps, red);
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = v;
}

// K^{aa} = kappa^2 I3 - (2 J(d_a) - J(d_a - 1) - J(d_a + 1)); K^{ab} = -sum s s' P; the
// components odd in an axis with d = 0 there vanish.  One lane per touching offset.
__global__ void k_generator_near(c128 *gen, const c128 *parts, int nx, int ny, int nz, double kappa) {
    const int off = threadIdx.x;
    if (off >= 8) return;
    const int dx = off & 1, dy = (off >> 1) & 1, dz = (off >> 2) & 1;
    if (dx >= nx || dy >= ny || dz >= nz) return;
    const long long N = (long long)nx * ny * nz;
    const long long o = ((long long)dz * ny + dy) * nx + dx;
    const c128 *pt = parts + off * NEAR_PARTS;
    c128 out[6];
    const c128 I3 = pt[0];
    for (int a = 0; a < 3; ++a) {
        const c128 *J = pt + 1 + 3 * a;
        c128 F = mk(-(2.0 * J[1].re - J[0].re - J[2].re), -(2.0 * J[1].im - J[0].im - J[2].im));
        out[a] = F + mk(kappa * kappa * I3.re, kappa * kappa * I3.im);
    }
    for (int k = 0; k < 3; ++k) {
        c128 tot = czero<double>();
        for (int si = 0; si < 2; ++si)
            for (int spi = 0; spi < 2; ++spi) {
                const c128 P = pt[10 + 4 * k + 2 * si + spi];
                const double ss = (si == spi) ? 1.0 : -1.0;
                tot = tot + mk(ss * P.re, ss * P.im);
            }
        out[3 + k] = mk(-tot.re, -tot.im);
    }
    if (dx == 0 || dy == 0) out[3] = czero<double>();
    if (dx == 0 || dz == 0) out[4] = czero<double>();
    if (dy == 0 || dz == 0) out[5] = czero<double>();
    for (int c = 0; c < 6; ++c) gen[c * N + o] = out[c];
}

vie_status launch_generator(vie_op op, hipStream_t s) {
    VIE_CHECK(upload_gl());
    long long N = op->N;
    if (N > 0x7fffffffLL) {
        vie_set_error("grid too large for the generator launch");
        return VIE_EARG;
    }
    ProfScope ps("generator", s);
    hipLaunchKernelGGL(k_generator_far, dim3((unsigned)N), dim3(64), 0, s, op->gen.as<c128>(), op->nx, op->ny,
                       op->nz, op->kappa);
    VIE_HIP(hipGetLastError());
    DevBuf parts;
    VIE_CHECK(parts.ensure(sizeof(c128) * 8 * NEAR_PARTS));
    hipLaunchKernelGGL(k_generator_near_parts, dim3(8 * NEAR_PARTS), dim3(GEN_THREADS), 0, s, parts.as<c128>(),
                       op->nx, op->ny, op->nz, op->kappa);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_generator_near, dim3(1), dim3(64), 0, s, op->gen.as<c128>(), (const c128 *)parts.as<c128>(),
                       op->nx, op->ny, op->nz, op->kappa);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}
