// Restarted right-preconditioned flexible GMRES on the device, batched over right-hand
// sides in lockstep (Sec. 1: the discrete JVIE is solved by GMRES; restart, side and
// orthogonalisation are this library's choices).
//
// Per Arnoldi step j, for every right-hand side r of the batch at once:
//   z_j = P^{-1} v_j (kept, so x += Z y at the end of a cycle: flexible GMRES),
//   w = A z_j (one batched operator product),
//   classical Gram-Schmidt applied twice with wavefront reductions (per-workgroup
//   partials, then one reduction kernel), FP64 throughout,
//   a single-lane kernel per right-hand side applies the previous complex Givens rotations
//   to the new Hessenberg column, forms the next rotation and updates |g_{j+1}|;
//   these estimates (one per right-hand side) are the only values read back per step.
// Each cycle ends with x += Z y and the FP64 true residual r = b - A x.
//
// FP64 mode: v, z, products and factors complex128.  Mixed mode: v_j is rounded to
// complex64 for the preconditioner (complex64 factors) and the complex64 operator
// product, whose result is widened back for the FP64 Arnoldi step; Z is kept in
// complex64; the true residual of every cycle uses the complex128 product, so the
// outer loop is an FP64 iterative refinement around the FP32 inner solve; the basis V is
// stored in complex64.  Mixed-preconditioner mode: only the preconditioner runs in complex64
// (or bfloat16 factors), on a complex64 copy of v_j; Z is kept in complex64, each z_j is
// widened for the complex128 product, and V stays complex128.
#include <cmath>

#include "vie_internal.h"

#define KR_THREADS 256
// The Arnoldi kernels split every vector into parts, one workgroup each: about KR_EPT_DOTS
// elements per thread for the dot products (their 16 loads in flight per element already
// cover the latency; fewer parts mean fewer partial reductions), KR_EPT_UPD for the updates,
// at most KR_PARTS_MAX parts.  The split depends on the vector length alone, so a right-hand
// side is summed in the same order whatever it is batched with.
#define KR_EPT_DOTS 12
#define KR_EPT_UPD 2
#define KR_PARTS_MAX 2048

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

// Widen a stored basis entry (complex128, or complex64 in the mixed mode) to FP64.
__device__ __forceinline__ c128 wide(c128 a) { return a; }
__device__ __forceinline__ c128 wide(c64 a) { return mk((double)a.re, (double)a.im); }

// Batched vectors: vector j of right-hand side r at base + j * ldj + r * n.  The basis V is
// complex128, or complex64 in the mixed mode; sums are accumulated in FP64.
// partial[(r * gridDim.x + blk) * stride + i] = sum_e conj(V_i[e]) w[e], stride = nv + self;
// `self` adds |w|^2 as output nv.  The outputs are formed KR_DG at a time, so w is read once
// per group of KR_DG basis vectors rather than once per vector; inside a group the KR_DG loads
// of an element are unconditional (a short last group clamps its index and drops the extra
// products), so they are all in flight together.
#define KR_DG 16
template <class VT>
__global__ void __launch_bounds__(KR_THREADS) k_dots(const VT *V, long long ldj, int nv, const c128 *w, long long n,
                                                     int self, c128 *partial) {
    __shared__ c128 sh[KR_DG + 1][KR_THREADS / 64];
    const int r = blockIdx.y;
    const c128 *wr = w + r * n;
    const VT *Vr = V + r * n;
    long long chunk = (n + gridDim.x - 1) / gridDim.x;
    long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    const int stride = nv + self;
    c128 *out = partial + ((long long)r * gridDim.x + blockIdx.x) * stride;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int ngroups = nv > 0 ? (nv + KR_DG - 1) / KR_DG : 1;
    for (int gi = 0; gi < ngroups; ++gi) {
        const int i0 = gi * KR_DG, cnt = min(KR_DG, nv - i0);
        const bool do_self = self && gi == 0;
        c128 acc[KR_DG];
        double sacc = 0.0;
#pragma unroll
        for (int u = 0; u < KR_DG; ++u) acc[u] = czero<double>();
        if (cnt == KR_DG) {
            for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) {
                const c128 we = wr[e];
                c128 v[KR_DG];
#pragma unroll
                for (int u = 0; u < KR_DG; ++u) v[u] = wide(Vr[(i0 + u) * ldj + e]);
#pragma unroll
                for (int u = 0; u < KR_DG; ++u) acc[u] = acc[u] + cmulc(v[u], we);
                if (do_self) sacc += abs2(we);
            }
        } else if (cnt > 0) {
            for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) {
                const c128 we = wr[e];
                c128 v[KR_DG];
#pragma unroll
                for (int u = 0; u < KR_DG; ++u) v[u] = wide(Vr[min(i0 + u, nv - 1) * ldj + e]);
#pragma unroll
                for (int u = 0; u < KR_DG; ++u)
                    if (u < cnt) acc[u] = acc[u] + cmulc(v[u], we);
                if (do_self) sacc += abs2(we);
            }
        } else {  // no basis vectors: the self entry alone
            for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) sacc += abs2(wr[e]);
        }
#pragma unroll
        for (int u = 0; u < KR_DG; ++u) {
            const c128 v = wave_sum(acc[u]);
            if (lane == 0) sh[u][wid] = v;
        }
        if (do_self) {
            const c128 v = wave_sum(mk(sacc, 0.0));
            if (lane == 0) sh[KR_DG][wid] = v;
        }
        __syncthreads();
        if (threadIdx.x < KR_DG && (int)threadIdx.x < cnt) {
            c128 t = czero<double>();
            for (int q = 0; q < KR_THREADS / 64; ++q) t = t + sh[threadIdx.x][q];
            out[i0 + threadIdx.x] = t;
        }
        if (do_self && threadIdx.x == KR_DG) {
            c128 t = czero<double>();
            for (int q = 0; q < KR_THREADS / 64; ++q) t = t + sh[KR_DG][q];
            out[nv] = t;
        }
        __syncthreads();
    }
}

// out[r * ostride + i] = sum_b partial[(r * nb + b) * stride + i]; grid (count, R)
__global__ void __launch_bounds__(KR_THREADS) k_reduce(const c128 *partial, int nb, int stride, c128 *out,
                                                       int ostride) {
    __shared__ c128 sh[KR_THREADS / 64];
    int i = blockIdx.x, r = blockIdx.y;
    c128 acc = czero<double>();
    for (int b = threadIdx.x; b < nb; b += KR_THREADS) acc = acc + partial[((long long)r * nb + b) * stride + i];
    c128 s = block_sum_kr(acc, sh);
    if (threadIdx.x == 0) out[(long long)r * ostride + i] = s;
}

// w_r -= sum_i V_i,r h_r[i]; optional partial |w_r|^2 into partial[r * gridDim.x + blk].
template <class VT>
__global__ void __launch_bounds__(KR_THREADS) k_update(const VT *V, long long ldj, int nv, const c128 *h, int hstride,
                                                       c128 *w, long long n, c128 *partial) {
    __shared__ c128 hs[256];
    __shared__ c128 sh[KR_THREADS / 64];
    const int r = blockIdx.y;
    for (int i = threadIdx.x; i < nv; i += KR_THREADS) hs[i] = h[(long long)r * hstride + i];
    __syncthreads();
    c128 *wr = w + r * n;
    long long chunk = (n + gridDim.x - 1) / gridDim.x;
    long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    c128 nrm = czero<double>();
    const VT *Vr = V + r * n;
    for (long long e = lo + threadIdx.x; e < hi; e += KR_THREADS) {
        c128 acc = wr[e];
        int i = 0;
        for (; i + 8 <= nv; i += 8) {  // eight loads in flight, products in order of i
            c128 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = wide(Vr[(i + u) * ldj + e]);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = cfms(acc, v[u], hs[i + u]);
        }
        for (; i < nv; ++i) acc = cfms(acc, wide(Vr[i * ldj + e]), hs[i]);
        wr[e] = acc;
        nrm.re += abs2(acc);
    }
    if (partial) {
        c128 s = block_sum_kr(nrm, sh);
        if (threadIdx.x == 0) partial[(long long)r * gridDim.x + blockIdx.x] = s;
    }
}

// x_r += sum_{i < jr[r]} Z_i,r y_r[i]   (Z in complex128 or complex64)
template <class R>
__global__ void __launch_bounds__(KR_THREADS) k_combine(const cpx<R> *Z, long long ldj, const int *jr, const c128 *y,
                                                        int ystride, c128 *x, long long n) {
    __shared__ c128 ys[256];
    const int r = blockIdx.y;
    const int nv = jr[r];
    for (int i = threadIdx.x; i < nv; i += KR_THREADS) ys[i] = y[(long long)r * ystride + i];
    __syncthreads();
    if (nv == 0) return;
    for (long long e = blockIdx.x * (long long)KR_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * KR_THREADS) {
        c128 acc = x[r * n + e];
        for (int i = 0; i < nv; ++i) {
            cpx<R> z = Z[i * ldj + r * n + e];
            acc = acc + mk((double)z.re, (double)z.im) * ys[i];
        }
        x[r * n + e] = acc;
    }
}

// v_r = w_r / scal[r * sstride]  (zero for an inactive right-hand side or a zero scale),
// stored in the basis precision
template <class VT>
__global__ void k_scale(const c128 *w, VT *v, long long n, const double *scal, int sstride, const int *active) {
    typedef decltype(v->re) T;
    const int r = blockIdx.y;
    double s = scal[(long long)r * sstride];
    double f = (active[r] && s != 0.0) ? 1.0 / s : 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        c128 a = w[r * n + e];
        v[r * n + e] = mk((T)(a.re * f), (T)(a.im * f));
    }
}

__global__ void k_residual(const c128 *b, c128 *r, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        r[e] = b[e] - r[e];
}

__global__ void k_widen(const c64 *a, c128 *b, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        b[e] = mk((double)a[e].re, (double)a[e].im);
}

// Per right-hand side Arnoldi bookkeeping arrays (device), each with R slices.
struct GState {
    c128 *h1, *h2;  // [R][m+2]: two CGS passes; h1[nv] = |w0|^2 (self entry)
    c128 *nrm2;     // [R]: |w|^2 after orthogonalisation
    c128 *Rm;       // [R][m][m+1] column-major rotated Hessenberg
    double *cs;     // [R][m]
    c128 *sn;       // [R][m]
    c128 *g;        // [R][m+1]
    c128 *y;        // [R][m]
    double *st;     // [R][4]: |g_{j+1}|, h_{j+1,j}, breakdown, |w0|
    int *active;    // [R]
    int m;
};

// Step j for every active right-hand side: one wavefront per right-hand side.  Its lanes stage
// the new column (h1 + h2) and the earlier rotations in LDS; lane 0 then applies the rotations
// in order (the serial chain reads LDS, not global memory) and forms the new one.
#define KR_MAX_RESTART VIE_MAX_RESTART
__global__ void __launch_bounds__(64) k_givens(GState S, int j, int R) {
    __shared__ c128 col[KR_MAX_RESTART + 1];
    __shared__ double csl[KR_MAX_RESTART];
    __shared__ c128 snl[KR_MAX_RESTART];
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= R) return;
    const int m = S.m;
    double *st = S.st + 4 * r;
    if (!S.active[r]) {
        if (lane == 0) {
            st[0] = 0.0;
            st[1] = 0.0;
            st[2] = 1.0;
            st[3] = 0.0;
        }
        return;
    }
    const c128 *h1 = S.h1 + (long long)r * (m + 2), *h2 = S.h2 + (long long)r * (m + 2);
    c128 *colg = S.Rm + ((long long)r * m + j) * (m + 1);
    double *cs = S.cs + (long long)r * m;
    c128 *sn = S.sn + (long long)r * m;
    c128 *g = S.g + (long long)r * (m + 1);
    for (int i = lane; i <= j; i += 64) col[i] = h1[i] + h2[i];
    for (int i = lane; i < j; i += 64) {
        csl[i] = cs[i];
        snl[i] = sn[i];
    }
    __syncthreads();
    if (lane == 0) {
        double hn = sqrt(S.nrm2[r].re);
        double w0 = sqrt(h1[j + 1].re);
        for (int i = 0; i < j; ++i) {
            c128 a = col[i], b = col[i + 1];
            col[i] = csl[i] * a + snl[i] * b;
            col[i + 1] = csl[i] * b - conjg(snl[i]) * a;
        }
        c128 a = col[j];
        double c;
        c128 s, rr;
        double aa = sqrt(abs2(a)), bb = hn;
        if (bb == 0.0) {
            c = 1.0;
            s = czero<double>();
            rr = a;
        } else if (aa == 0.0) {
            c = 0.0;
            s = mk(1.0, 0.0);
            rr = mk(hn, 0.0);
        } else {
            double rho = hypot(aa, bb);
            c128 ph = mk(a.re / aa, a.im / aa);
            c = aa / rho;
            s = mk(ph.re * bb / rho, ph.im * bb / rho);  // phase * conj(b) / rho, b real
            rr = mk(ph.re * rho, ph.im * rho);
        }
        cs[j] = c;
        sn[j] = s;
        col[j] = rr;
        c128 gj = g[j];
        g[j + 1] = mk(0.0, 0.0) - conjg(s) * gj;
        g[j] = c * gj;
        st[0] = sqrt(abs2(g[j + 1]));
        st[1] = hn;
        st[2] = (hn <= 1e-14 * w0) ? 1.0 : 0.0;
        st[3] = w0;
    }
    __syncthreads();
    for (int i = lane; i <= j; i += 64) colg[i] = col[i];
}

// y_r = R_r^{-1} g_r over the first jr[r] columns; one lane per right-hand side.
__global__ void k_lsq(GState S, const int *jr, int R) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int m = S.m, k = jr[r];
    const c128 *Rm = S.Rm + (long long)r * m * (m + 1);
    const c128 *g = S.g + (long long)r * (m + 1);
    c128 *y = S.y + (long long)r * m;
    for (int i = k - 1; i >= 0; --i) {
        c128 acc = g[i];
        for (int c = i + 1; c < k; ++c) acc = cfms(acc, Rm[(long long)c * (m + 1) + i], y[c]);
        y[i] = cdiv(acc, Rm[(long long)i * (m + 1) + i]);
    }
}

// g_r = (beta_r, 0, ...)
__global__ void k_setg(c128 *g, int m1, const double *beta, int R) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m1 * R) return;
    int r = i / m1, k = i % m1;
    g[i] = mk(k == 0 ? beta[r] : 0.0, 0.0);
}

namespace {
struct Ctx {
    vie_op op;
    hipStream_t s;
    long long n;  // 3N
    int R;
    int nbd, nbu;  // parts per vector of the dot products and of the updates
    c128 *partial;
    double *host;  // pinned scratch
};

// batched norms: out[r].re = |w_r|^2
vie_status norms(Ctx &C, const c128 *w, c128 *out) {
    hipLaunchKernelGGL(k_dots<c128>, dim3(C.nbd, C.R), dim3(KR_THREADS), 0, C.s, (const c128 *)nullptr, 0LL, 0, w,
                       C.n, 1, C.partial);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(1, C.R), dim3(KR_THREADS), 0, C.s, C.partial, C.nbd, 1, out, 1);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// Classical Gram-Schmidt twice against v_0..v_j, the Givens update of column j and
// v_{j+1} = w / h_{j+1,j} (Sec. 1: GMRES; the orthogonalisation is this library's choice).
template <class VT>
vie_status cgs2_step(Ctx &C, const VT *V, long long ldj, int j, c128 *w, GState &S, int m, dim3 grid_e,
                     VT *vnext) {
    hipStream_t s = C.s;
    const long long n = C.n;
    const int R = C.R;
    const dim3 grid_d(C.nbd, R), grid_u(C.nbu, R);
    {
        ProfScope ps("arnoldi_dots", s);
        hipLaunchKernelGGL(k_dots<VT>, grid_d, dim3(KR_THREADS), 0, s, V, ldj, j + 1, (const c128 *)w, n, 1, C.partial);
        VIE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce, dim3(j + 2, R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbd, j + 2,
                       S.h1, m + 2);
    VIE_HIP(hipGetLastError());
    {
        ProfScope ps("arnoldi_update", s);
        hipLaunchKernelGGL(k_update<VT>, grid_u, dim3(KR_THREADS), 0, s, V, ldj, j + 1, (const c128 *)S.h1, m + 2, w, n,
                           (c128 *)nullptr);
        VIE_HIP(hipGetLastError());
    }
    {
        ProfScope ps("arnoldi_dots", s);
        hipLaunchKernelGGL(k_dots<VT>, grid_d, dim3(KR_THREADS), 0, s, V, ldj, j + 1, (const c128 *)w, n, 0, C.partial);
        VIE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce, dim3(j + 1, R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbd, j + 1,
                       S.h2, m + 2);
    VIE_HIP(hipGetLastError());
    {
        ProfScope ps("arnoldi_update", s);
        hipLaunchKernelGGL(k_update<VT>, grid_u, dim3(KR_THREADS), 0, s, V, ldj, j + 1, (const c128 *)S.h2, m + 2, w, n,
                           C.partial);
        VIE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce, dim3(1, R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbu, 1, S.nrm2, 1);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_givens, dim3(R), dim3(64), 0, s, S, j, R);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scale<VT>, grid_e, dim3(256), 0, s, (const c128 *)w, vnext, n, (const double *)(S.st + 1), 4,
                       (const int *)S.active);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

vie_status read_host(Ctx &C, const void *dev, size_t bytes) {
    VIE_HIP(hipMemcpyAsync(C.host, dev, bytes, hipMemcpyDeviceToHost, C.s));
    VIE_HIP(hipStreamSynchronize(C.s));
    return VIE_OK;
}
}  // namespace

static int kr_parts(long long n, int ept) {
    return (int)std::max(1LL, std::min((long long)KR_PARTS_MAX, (n + ept * KR_THREADS - 1) / (ept * KR_THREADS)));
}

long long arnoldi_partials(long long n, int restart) {
    return std::max((long long)kr_parts(n, KR_EPT_DOTS) * (restart + 2), (long long)kr_parts(n, KR_EPT_UPD));
}

vie_status solve_gmres(vie_op op, vie_pc pc, const c128 *b, c128 *x, int R, const vie_solve_opts *o,
                       vie_solve_stats *stats, hipStream_t s, SolveHook *hook) {
    const bool mixed = o->mode == VIE_MODE_MIXED;
    const bool mixed_pc = o->mode == VIE_MODE_MIXED_PC;  // reduced-precision preconditioner only
    const bool lowpc = mixed || mixed_pc;
    if (mixed && !op->has_c64) {
        vie_set_error("mixed-precision solve needs an operator built with build_c64");
        return VIE_EARG;
    }
    if (pc && (lowpc ? (pc->prec != VIE_C64 && pc->prec != VIE_BF16C) : pc->prec != VIE_C128)) {
        vie_set_error(lowpc ? "mixed-precision solve needs complex64 or bfloat16 preconditioner factors"
                            : "FP64 solve needs complex128 preconditioner factors");
        return VIE_EARG;
    }
    const int m = o->restart;
    const long long n = 3LL * op->N;
    const long long Rn = (long long)R * n;
    Ctx C{op, s, n, R, kr_parts(n, KR_EPT_DOTS), kr_parts(n, KR_EPT_UPD), nullptr, nullptr};
    // mixed: basis V and flexible basis Z in complex64, FP64 sums and w.  mixed_pc: V in
    // complex128 with a complex64 copy of its newest vector (vlo) for the preconditioner, Z in
    // complex64, each z_j widened (zw) for the complex128 product.
    const bool v32 = mixed;
    const size_t vsz = v32 ? sizeof(c64) : sizeof(c128);
    const size_t zsz = lowpc ? sizeof(c64) : sizeof(c128);
    DevBuf Vb, Zb, wb, rb, part, small, w32, vlo, zw;
    VIE_CHECK(Vb.ensure(vsz * Rn * (m + 1)));
    VIE_CHECK(Zb.ensure(zsz * Rn * m));
    if (mixed_pc) {
        VIE_CHECK(vlo.ensure(sizeof(c64) * Rn));
        VIE_CHECK(zw.ensure(sizeof(c128) * Rn));
    }
    VIE_CHECK(wb.ensure(sizeof(c128) * Rn));
    VIE_CHECK(rb.ensure(sizeof(c128) * Rn));
    VIE_CHECK(part.ensure(sizeof(c128) * (size_t)R * arnoldi_partials(n, m)));
    if (mixed) VIE_CHECK(w32.ensure(sizeof(c64) * Rn));
    size_t nc = (size_t)R * ((size_t)(m + 2) * 2 + 1 + (size_t)m * (m + 1) + m + (m + 1) + m);
    size_t nd = (size_t)R * (m + 4 + 1);
    VIE_CHECK(small.ensure(sizeof(c128) * nc + sizeof(double) * nd + sizeof(int) * 2 * R));
    c128 *cp = small.as<c128>();
    GState S;
    S.m = m;
    S.h1 = cp;
    cp += (size_t)R * (m + 2);
    S.h2 = cp;
    cp += (size_t)R * (m + 2);
    S.nrm2 = cp;
    cp += R;
    S.Rm = cp;
    cp += (size_t)R * m * (m + 1);
    S.sn = cp;
    cp += (size_t)R * m;
    S.g = cp;
    cp += (size_t)R * (m + 1);
    S.y = cp;
    cp += (size_t)R * m;
    double *dp = reinterpret_cast<double *>(cp);
    S.cs = dp;
    dp += (size_t)R * m;
    S.st = dp;
    dp += (size_t)R * 4;
    double *beta_dev = dp;
    dp += R;
    S.active = reinterpret_cast<int *>(dp);
    int *jr_dev = S.active + R;
    C.partial = part.as<c128>();
    double *host = nullptr;
    // pinned layout: doubles [0, 4R) | ints active [R] | ints jr [R]
    VIE_HIP(hipHostMalloc((void **)&host, sizeof(double) * 4 * (size_t)R + sizeof(int) * 2 * R + 64,
                          hipHostMallocDefault));
    struct HostFree {
        double *p;
        ~HostFree() { (void)hipHostFree(p); }
    } hf{host};
    C.host = host;
    int *hact = reinterpret_cast<int *>(host + 4 * (size_t)R);
    int *hjr = hact + R;
    c128 *w = wb.as<c128>(), *r = rb.as<c128>();
    const long long ldj = Rn;  // stride between Arnoldi vectors
    dim3 grid_e(1024, R);

    std::vector<double> nb(R), beta(R);
    std::vector<int> done(R, 0), act(R, 0), jr(R, 0), told(R, 0);
    for (int q = 0; q < R; ++q) stats[q] = vie_solve_stats{0, 0, 0.0, VIE_OK};
    VIE_CHECK(norms(C, b, S.nrm2));
    VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
    for (int q = 0; q < R; ++q) nb[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
    for (int q = 0; q < R; ++q)
        if (!std::isfinite(nb[q])) {
            vie_set_error("non-finite right-hand side " + std::to_string(q));
            return VIE_ENONFINITE;
        }
    if (o->x0_given) {
        VIE_CHECK(launch_matvec(op, x, r, R, VIE_C128, s));
        hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, Rn);
        VIE_HIP(hipGetLastError());
    } else {
        VIE_HIP(hipMemsetAsync(x, 0, sizeof(c128) * Rn, s));
        VIE_HIP(hipMemcpyAsync(r, b, sizeof(c128) * Rn, hipMemcpyDeviceToDevice, s));
    }
    VIE_CHECK(norms(C, r, S.nrm2));
    VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
    for (int q = 0; q < R; ++q) beta[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
    vie_status result = VIE_OK;
    for (;;) {
        int nact = 0;
        for (int q = 0; q < R; ++q) {
            if (!std::isfinite(beta[q])) {
                vie_set_error("non-finite residual for right-hand side " + std::to_string(q));
                return VIE_ENONFINITE;
            }
            double rel = nb[q] > 0 ? beta[q] / nb[q] : 0.0;
            stats[q].relres = rel;
            if (!done[q] && (nb[q] == 0.0 || rel <= o->tol)) done[q] = 1;
            if (!done[q] && stats[q].iters >= o->maxit) {
                done[q] = 1;
                stats[q].status = VIE_NOT_CONVERGED;
                result = VIE_NOT_CONVERGED;
            }
            act[q] = !done[q];
            jr[q] = 0;
            nact += act[q];
        }
        if (hook) {  // hand out ended columns, take new right-hand sides into their slots
            std::vector<int> ended, refill;
            for (int q = 0; q < R; ++q)
                if (done[q] && !told[q]) {
                    told[q] = 1;
                    ended.push_back(q);
                }
            VIE_CHECK(hook->boundary(ended, stats, x, const_cast<c128 *>(b), s, &refill));
            if (!refill.empty()) {
                for (int q : refill) {
                    VIE_HIP(hipMemsetAsync(x + (long long)q * n, 0, sizeof(c128) * n, s));
                    VIE_HIP(hipMemcpyAsync(r + (long long)q * n, b + (long long)q * n, sizeof(c128) * n,
                                           hipMemcpyDeviceToDevice, s));
                }
                VIE_CHECK(norms(C, b, S.nrm2));
                VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
                for (int q : refill) {
                    nb[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
                    if (!std::isfinite(nb[q])) {
                        vie_set_error("non-finite right-hand side in slot " + std::to_string(q));
                        return VIE_ENONFINITE;
                    }
                    beta[q] = nb[q];
                    stats[q] = vie_solve_stats{0, 0, nb[q] > 0 ? 1.0 : 0.0, VIE_OK};
                    done[q] = told[q] = 0;
                    act[q] = 1;
                    ++nact;
                }
            }
        }
        if (nact == 0) break;
        // v0 = r / beta (zero for finished right-hand sides), g = (beta, 0, ...)
        for (int q = 0; q < R; ++q) {
            host[q] = beta[q];
            hact[q] = act[q];
        }
        VIE_HIP(hipMemcpyAsync(beta_dev, host, sizeof(double) * R, hipMemcpyHostToDevice, s));
        VIE_HIP(hipMemcpyAsync(S.active, hact, sizeof(int) * R, hipMemcpyHostToDevice, s));
        if (v32)
            hipLaunchKernelGGL(k_scale<c64>, grid_e, dim3(256), 0, s, (const c128 *)r, Vb.as<c64>(), n,
                               (const double *)beta_dev, 1, (const int *)S.active);
        else
            hipLaunchKernelGGL(k_scale<c128>, grid_e, dim3(256), 0, s, (const c128 *)r, Vb.as<c128>(), n,
                               (const double *)beta_dev, 1, (const int *)S.active);
        if (mixed_pc)
            hipLaunchKernelGGL(k_scale<c64>, grid_e, dim3(256), 0, s, (const c128 *)r, vlo.as<c64>(), n,
                               (const double *)beta_dev, 1, (const int *)S.active);
        VIE_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_setg, dim3((unsigned)(((m + 1) * R + 63) / 64)), dim3(64), 0, s, S.g, m + 1,
                           (const double *)beta_dev, R);
        VIE_HIP(hipGetLastError());
        int j = 0;
        while (j < m && nact > 0) {
            void *vj = (char *)Vb.p + vsz * Rn * j;
            void *zj = (char *)Zb.p + zsz * Rn * j;
            if (!lowpc) {
                if (pc)
                    VIE_CHECK(pc_apply(pc, vj, zj, R, VIE_C128, s));
                else
                    VIE_HIP(hipMemcpyAsync(zj, vj, sizeof(c128) * Rn, hipMemcpyDeviceToDevice, s));
                VIE_CHECK(launch_matvec(op, zj, w, R, VIE_C128, s));
            } else {
                const void *vin = mixed_pc ? vlo.p : vj;
                if (pc)
                    VIE_CHECK(pc_apply(pc, vin, zj, R, VIE_C64, s));
                else
                    VIE_HIP(hipMemcpyAsync(zj, vin, sizeof(c64) * Rn, hipMemcpyDeviceToDevice, s));
                if (mixed) {
                    VIE_CHECK(launch_matvec(op, zj, w32.p, R, VIE_C64, s));
                    hipLaunchKernelGGL(k_widen, dim3(1024), dim3(256), 0, s, w32.as<const c64>(), w, Rn);
                    VIE_HIP(hipGetLastError());
                } else {
                    hipLaunchKernelGGL(k_widen, dim3(1024), dim3(256), 0, s, (const c64 *)zj, zw.as<c128>(), Rn);
                    VIE_HIP(hipGetLastError());
                    VIE_CHECK(launch_matvec(op, zw.p, w, R, VIE_C128, s));
                }
            }
            if (v32)
                VIE_CHECK(cgs2_step<c64>(C, Vb.as<const c64>(), ldj, j, w, S, m, grid_e, Vb.as<c64>() + (j + 1) * ldj));
            else
                VIE_CHECK(cgs2_step<c128>(C, Vb.as<const c128>(), ldj, j, w, S, m, grid_e,
                                          Vb.as<c128>() + (j + 1) * ldj));
            if (mixed_pc) {  // the complex64 copy of v_{j+1} = w / h_{j+1,j}
                hipLaunchKernelGGL(k_scale<c64>, grid_e, dim3(256), 0, s, (const c128 *)w, vlo.as<c64>(), n,
                                   (const double *)(S.st + 1), 4, (const int *)S.active);
                VIE_HIP(hipGetLastError());
            }
            VIE_CHECK(read_host(C, S.st, sizeof(double) * 4 * R));
            ++j;
            bool changed = false;
            for (int q = 0; q < R; ++q) {
                if (!act[q]) continue;
                double est = host[4 * q] / nb[q];
                if (!std::isfinite(est)) {
                    vie_set_error("non-finite Arnoldi step for right-hand side " + std::to_string(q));
                    return VIE_ENONFINITE;
                }
                ++stats[q].iters;
                jr[q] = j;
                if (est <= o->tol || host[4 * q + 2] != 0.0 || stats[q].iters >= o->maxit) {
                    act[q] = 0;
                    --nact;
                    changed = true;
                }
            }
            if (changed && nact > 0 && j < m) {
                for (int q = 0; q < R; ++q) hact[q] = act[q];
                VIE_HIP(hipMemcpyAsync(S.active, hact, sizeof(int) * R, hipMemcpyHostToDevice, s));
            }
        }
        // x += Z y
        for (int q = 0; q < R; ++q) hjr[q] = jr[q];
        VIE_HIP(hipMemcpyAsync(jr_dev, hjr, sizeof(int) * R, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_lsq, dim3((R + 63) / 64), dim3(64), 0, s, S, (const int *)jr_dev, R);
        VIE_HIP(hipGetLastError());
        if (lowpc)
            hipLaunchKernelGGL(k_combine<float>, grid_e, dim3(KR_THREADS), 0, s, Zb.as<const c64>(), ldj,
                               (const int *)jr_dev, (const c128 *)S.y, m, x, n);
        else
            hipLaunchKernelGGL(k_combine<double>, grid_e, dim3(KR_THREADS), 0, s, Zb.as<const c128>(), ldj,
                               (const int *)jr_dev, (const c128 *)S.y, m, x, n);
        VIE_HIP(hipGetLastError());
        for (int q = 0; q < R; ++q)
            if (jr[q] > 0) ++stats[q].restarts;
        // FP64 true residual
        VIE_CHECK(launch_matvec(op, x, r, R, VIE_C128, s));
        hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, Rn);
        VIE_HIP(hipGetLastError());
        VIE_CHECK(norms(C, r, S.nrm2));
        VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
        for (int q = 0; q < R; ++q) beta[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
    }
    return result;
}
