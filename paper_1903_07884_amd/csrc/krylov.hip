// Restarted right-preconditioned (flexible) GMRES on the device (Sec. 1: the
// discrete JVIE is solved by GMRES; restart, side and orthogonalisation are
// this library's choices).
//
// Per Arnoldi step j: z_j = P^{-1} v_j (kept, so x += Z y at the end of a
// cycle), w = A z_j, classical Gram-Schmidt applied twice with wavefront
// reductions (two-stage: per-workgroup partials, then one reduction kernel),
// a single-lane kernel applies the previous complex Givens rotations to the
// new Hessenberg column, forms the next rotation and updates the residual
// estimate |g_{j+1}|, which is the only value read back by the host each step.
// Each cycle ends with the FP64 true residual r = b - A x.
#include <cmath>

#include "vie_internal.h"

#define KR_THREADS 256
#define KR_BLOCKS 512

__device__ __forceinline__ c128 wave_sum(c128 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_down(v.re, off);
        v.im += __shfl_down(v.im, off);
    }
    return v;
}

__device__ __forceinline__ c128 block_sum_kr(c128 v, c128 *sh) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    c128 r = czero<double>();
    if (threadIdx.x == 0)
        for (int i = 0; i < KR_THREADS / 64; ++i) r = r + sh[i];
    __syncthreads();
    return r;  // valid in thread 0
}

// partial[blk * (nv + self) + i] = sum_e conj(V_i[e]) w[e]; with `self` an extra |w|^2 entry.
__global__ void __launch_bounds__(KR_THREADS) k_dots(const c128 *V, long long ldv, int nv, const c128 *w, long long n,
                                                     int self, c128 *partial) {
    __shared__ c128 sh[KR_THREADS / 64];
    long long chunk = (n + gridDim.x - 1) / gridDim.x;
    long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    int stride = nv + self;
    for (int i = 0; i < nv; ++i) {
        const c128 *v = V + i * ldv;
        c128 acc = czero<double>();
        for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) acc = acc + cmulc(v[e], w[e]);
        c128 s = block_sum_kr(acc, sh);
        if (threadIdx.x == 0) partial[blockIdx.x * stride + i] = s;
    }
    if (self) {
        c128 acc = czero<double>();
        for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) acc.re += abs2(w[e]);
        c128 s = block_sum_kr(acc, sh);
        if (threadIdx.x == 0) partial[blockIdx.x * stride + nv] = s;
    }
}

// out[i] = sum_b partial[b * stride + i], i < cnt.  One workgroup per i.
__global__ void __launch_bounds__(KR_THREADS) k_reduce(const c128 *partial, int nb, int stride, c128 *out) {
    __shared__ c128 sh[KR_THREADS / 64];
    int i = blockIdx.x;
    c128 acc = czero<double>();
    for (int b = threadIdx.x; b < nb; b += KR_THREADS) acc = acc + partial[b * stride + i];
    c128 s = block_sum_kr(acc, sh);
    if (threadIdx.x == 0) out[i] = s;
}

// w -= sum_i V_i h[i]; optional partial |w|^2 into partial[blk] (norm != 0).
__global__ void __launch_bounds__(KR_THREADS) k_update(const c128 *V, long long ldv, int nv, const c128 *h, c128 *w,
                                                       long long n, c128 *partial) {
    __shared__ c128 hs[256];
    __shared__ c128 sh[KR_THREADS / 64];
    for (int i = threadIdx.x; i < nv; i += KR_THREADS) hs[i] = h[i];
    __syncthreads();
    long long chunk = (n + gridDim.x - 1) / gridDim.x;
    long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    c128 nrm = czero<double>();
    for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) {
        c128 acc = w[e];
        for (int i = 0; i < nv; ++i) acc = cfms(acc, V[i * ldv + e], hs[i]);
        w[e] = acc;
        nrm.re += abs2(acc);
    }
    if (partial) {
        c128 s = block_sum_kr(nrm, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// out = sum_i V_i y[i]  (x update direction)
__global__ void __launch_bounds__(KR_THREADS) k_combine(const c128 *V, long long ldv, int nv, const c128 *y, c128 *out,
                                                        long long n, int accumulate) {
    __shared__ c128 ys[256];
    for (int i = threadIdx.x; i < nv; i += KR_THREADS) ys[i] = y[i];
    __syncthreads();
    for (long long e = blockIdx.x * (long long)KR_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * KR_THREADS) {
        c128 acc = accumulate ? out[e] : czero<double>();
        for (int i = 0; i < nv; ++i) acc = acc + V[i * ldv + e] * ys[i];
        out[e] = acc;
    }
}

// v = w * (1/s), s = scal[0].re
__global__ void k_scale(const c128 *w, c128 *v, long long n, const double *scal) {
    double f = 1.0 / scal[0];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        v[e] = mk(w[e].re * f, w[e].im * f);
}

// r = b - r
__global__ void k_residual(const c128 *b, c128 *r, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        r[e] = b[e] - r[e];
}

// Arnoldi bookkeeping for step j (single lane).
// st: [0] = |g_{j+1}|, [1] = h_{j+1,j} (the new basis scale), [2] = breakdown flag,
// [3] = sqrt(|w_0|^2) before orthogonalisation.
struct GState {
    c128 *h1, *h2;     // [nv] two CGS passes, h1[nv] = |w0|^2 (self entry)
    c128 *nrm2;        // [1] |w|^2 after orthogonalisation
    c128 *R;           // [restart][restart+1] column-major rotated Hessenberg
    double *cs;        // [restart]
    c128 *sn;          // [restart]
    c128 *g;           // [restart+1]
    double *st;        // [4]
};

__global__ void k_givens(GState S, int j, int ldr) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c128 *col = S.R + (long long)j * ldr;
    for (int i = 0; i <= j; ++i) col[i] = S.h1[i] + S.h2[i];
    double hn = sqrt(S.nrm2[0].re);
    double w0 = sqrt(S.h1[j + 1].re);
    c128 hj1 = mk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        c128 a = col[i], b = col[i + 1];
        col[i] = S.cs[i] * a + S.sn[i] * b;
        col[i + 1] = S.cs[i] * b - conjg(S.sn[i]) * a;
    }
    c128 a = col[j];
    double c;
    c128 s, r;
    double aa = sqrt(abs2(a)), bb = hn;
    if (bb == 0.0) {
        c = 1.0;
        s = czero<double>();
        r = a;
    } else if (aa == 0.0) {
        c = 0.0;
        s = mk(1.0, 0.0);
        r = hj1;
    } else {
        double rho = hypot(aa, bb);
        c128 ph = mk(a.re / aa, a.im / aa);
        c = aa / rho;
        s = mk(ph.re * bb / rho, ph.im * bb / rho);  // phase * conj(b)/rho, b real
        r = mk(ph.re * rho, ph.im * rho);
    }
    S.cs[j] = c;
    S.sn[j] = s;
    col[j] = r;
    c128 gj = S.g[j];
    S.g[j + 1] = mk(0.0, 0.0) - conjg(s) * gj;
    S.g[j] = c * gj;
    S.st[0] = sqrt(abs2(S.g[j + 1]));
    S.st[1] = hn;
    S.st[2] = (hn <= 1e-14 * w0) ? 1.0 : 0.0;
    S.st[3] = w0;
}

// y = R^{-1} g (k x k upper triangular), single lane
__global__ void k_lsq(const c128 *R, int ldr, const c128 *g, c128 *y, int k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        c128 acc = g[i];
        for (int c = i + 1; c < k; ++c) acc = cfms(acc, R[(long long)c * ldr + i], y[c]);
        y[i] = cdiv(acc, R[(long long)i * ldr + i]);
    }
}

__global__ void k_setg(c128 *g, int n, double beta) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] = mk(i == 0 ? beta : 0.0, 0.0);
}

namespace {
struct Ctx {
    vie_op op;
    vie_pc pc;
    hipStream_t s;
    long long n;
    c128 *partial;
    double *host;  // pinned
};

vie_status dots(Ctx &C, const c128 *V, long long ldv, int nv, const c128 *w, int self, c128 *out) {
    ProfScope ps("arnoldi_dots", C.s);
    hipLaunchKernelGGL(k_dots, dim3(KR_BLOCKS), dim3(KR_THREADS), 0, C.s, V, ldv, nv, w, C.n, self, C.partial);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(nv + self), dim3(KR_THREADS), 0, C.s, C.partial, KR_BLOCKS, nv + self, out);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

vie_status norm2(Ctx &C, const c128 *w, c128 *out) { return dots(C, nullptr, 0, 0, w, 1, out); }

vie_status read_doubles(Ctx &C, const double *dev, int cnt) {
    VIE_HIP(hipMemcpyAsync(C.host, dev, sizeof(double) * cnt, hipMemcpyDeviceToHost, C.s));
    VIE_HIP(hipStreamSynchronize(C.s));
    return VIE_OK;
}

vie_status apply_A(Ctx &C, const c128 *x, c128 *y) { return launch_matvec(C.op, x, y, 1, VIE_C128, C.s); }
vie_status apply_P(Ctx &C, const c128 *x, c128 *y) {
    if (!C.pc) {
        VIE_HIP(hipMemcpyAsync(y, x, sizeof(c128) * C.n, hipMemcpyDeviceToDevice, C.s));
        return VIE_OK;
    }
    return pc_apply(C.pc, x, y, 1, VIE_C128, C.s);
}
}  // namespace

vie_status solve_gmres(vie_op op, vie_pc pc, const c128 *b_all, c128 *x_all, int nrhs, const vie_solve_opts *o,
                       vie_solve_stats *stats, hipStream_t s) {
    if (pc && pc->prec != VIE_C128) {
        vie_set_error("FP64 solve needs complex128 preconditioner factors");
        return VIE_EARG;
    }
    const int m = o->restart;
    const long long n = 3LL * op->N;
    Ctx C{op, pc, s, n, nullptr, nullptr};
    DevBuf Vb, Zb, wb, rb, part, small;
    VIE_CHECK(Vb.ensure(sizeof(c128) * n * (m + 1)));
    VIE_CHECK(Zb.ensure(sizeof(c128) * n * m));
    VIE_CHECK(wb.ensure(sizeof(c128) * n));
    VIE_CHECK(rb.ensure(sizeof(c128) * n));
    VIE_CHECK(part.ensure(sizeof(c128) * KR_BLOCKS * (m + 2)));
    // small: h1[m+2], h2[m+2], nrm2[1], R[m*(m+1)], cs[m], sn[m], g[m+1], st[4], y[m]
    size_t off_h1 = 0, off_h2 = off_h1 + (m + 2), off_n = off_h2 + (m + 2), off_R = off_n + 1,
           off_sn = off_R + (size_t)m * (m + 1), off_g = off_sn + m, off_y = off_g + m + 1, off_end = off_y + m;
    size_t bytes = sizeof(c128) * off_end + sizeof(double) * (m + 4);
    VIE_CHECK(small.ensure(bytes));
    c128 *sm = small.as<c128>();
    double *cs = reinterpret_cast<double *>(sm + off_end);
    double *st = cs + m;
    GState S{sm + off_h1, sm + off_h2, sm + off_n, sm + off_R, cs, sm + off_sn, sm + off_g, st};
    C.partial = part.as<c128>();
    double *host = nullptr;
    VIE_HIP(hipHostMalloc((void **)&host, sizeof(double) * 8, hipHostMallocDefault));
    C.host = host;
    c128 *V = Vb.as<c128>(), *Z = Zb.as<c128>(), *w = wb.as<c128>(), *r = rb.as<c128>();
    vie_status result = VIE_OK;
    for (int q = 0; q < nrhs; ++q) {
        const c128 *b = b_all + q * n;
        c128 *x = x_all + q * n;
        vie_solve_stats &sq = stats[q];
        sq.iters = 0;
        sq.restarts = 0;
        sq.relres = 0;
        sq.status = VIE_OK;
        // ||b||
        VIE_CHECK(norm2(C, b, sm + off_n));
        VIE_CHECK(read_doubles(C, reinterpret_cast<const double *>(sm + off_n), 1));
        double nb = sqrt(host[0]);
        if (!std::isfinite(nb)) {
            vie_set_error("non-finite right-hand side");
            (void)hipHostFree(host);
            return VIE_ENONFINITE;
        }
        if (nb == 0.0) {
            VIE_HIP(hipMemsetAsync(x, 0, sizeof(c128) * n, s));
            continue;
        }
        // r = b - A x0
        if (o->x0_given) {
            VIE_CHECK(apply_A(C, x, r));
            hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, n);
            VIE_HIP(hipGetLastError());
        } else {
            VIE_HIP(hipMemsetAsync(x, 0, sizeof(c128) * n, s));
            VIE_HIP(hipMemcpyAsync(r, b, sizeof(c128) * n, hipMemcpyDeviceToDevice, s));
        }
        VIE_CHECK(norm2(C, r, sm + off_n));
        VIE_CHECK(read_doubles(C, reinterpret_cast<const double *>(sm + off_n), 1));
        double beta = sqrt(host[0]);
        bool done = false;
        while (!done) {
            if (!std::isfinite(beta)) {
                vie_set_error("non-finite residual");
                (void)hipHostFree(host);
                return VIE_ENONFINITE;
            }
            if (beta / nb <= o->tol) {
                sq.relres = beta / nb;
                break;
            }
            if (sq.iters >= o->maxit) {
                sq.relres = beta / nb;
                sq.status = VIE_NOT_CONVERGED;
                result = VIE_NOT_CONVERGED;
                break;
            }
            // v0 = r / beta
            host[4] = beta;
            VIE_HIP(hipMemcpyAsync(st + 1, host + 4, sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, s, r, V, n, st + 1);
            VIE_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_setg, dim3((m + 1 + 63) / 64), dim3(64), 0, s, S.g, m + 1, beta);
            VIE_HIP(hipGetLastError());
            int j = 0;
            while (j < m && sq.iters < o->maxit) {
                c128 *vj = V + j * n, *zj = Z + j * n;
                VIE_CHECK(apply_P(C, vj, zj));
                VIE_CHECK(apply_A(C, zj, w));
                VIE_CHECK(dots(C, V, n, j + 1, w, 1, S.h1));
                {
                    ProfScope ps("arnoldi_update", s);
                    hipLaunchKernelGGL(k_update, dim3(KR_BLOCKS), dim3(KR_THREADS), 0, s, V, n, j + 1, S.h1, w, n,
                                       (c128 *)nullptr);
                }
                VIE_HIP(hipGetLastError());
                VIE_CHECK(dots(C, V, n, j + 1, w, 0, S.h2));
                {
                    ProfScope ps("arnoldi_update", s);
                    hipLaunchKernelGGL(k_update, dim3(KR_BLOCKS), dim3(KR_THREADS), 0, s, V, n, j + 1, S.h2, w, n,
                                       C.partial);
                }
                VIE_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_reduce, dim3(1), dim3(KR_THREADS), 0, s, C.partial, KR_BLOCKS, 1, S.nrm2);
                VIE_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, S, j, m + 1);
                VIE_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, s, w, V + (j + 1) * n, n, st + 1);
                VIE_HIP(hipGetLastError());
                VIE_CHECK(read_doubles(C, st, 3));
                ++j;
                ++sq.iters;
                double est = host[0] / nb;
                if (!std::isfinite(est)) {
                    vie_set_error("non-finite Arnoldi step");
                    (void)hipHostFree(host);
                    return VIE_ENONFINITE;
                }
                if (est <= o->tol || host[2] != 0.0) break;
            }
            // x += Z y
            hipLaunchKernelGGL(k_lsq, dim3(1), dim3(64), 0, s, S.R, m + 1, S.g, sm + off_y, j);
            VIE_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_combine, dim3(1024), dim3(KR_THREADS), 0, s, Z, n, j, sm + off_y, x, n, 1);
            VIE_HIP(hipGetLastError());
            ++sq.restarts;
            // true residual
            VIE_CHECK(apply_A(C, x, r));
            hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, n);
            VIE_HIP(hipGetLastError());
            VIE_CHECK(norm2(C, r, sm + off_n));
            VIE_CHECK(read_doubles(C, reinterpret_cast<const double *>(sm + off_n), 1));
            beta = sqrt(host[0]);
        }
    }
    (void)hipHostFree(host);
    return result;
}
