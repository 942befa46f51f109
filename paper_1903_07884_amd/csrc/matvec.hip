// Operator product y = (I - M N) x (Sec. 2, eq. discrete_form) by FFT.
//
// N = I + K with K three-level block Toeplitz (Sec. 2 after eq. sys_mat).
// Each of the six unique generators is embedded in a circulant of period
// (Px, Py, Pz) >= (2nx-1, 2ny-1, 2nz-1) (offset d placed at d, -d at P-d with
// the block's parity, the rest zero) and transformed once at setup; the
// product is then crop(IFFT(Khat . FFT(zero-pad(x)))) (Sec. 1: O(n log n)).
//
// Three passes per product, each a batch of LDS-resident transforms:
//   1. forward x-FFT of every zero-padded x-line (coalesced line loads/stores),
//   2. per x-frequency: 2-D (y,z) FFT of the three components, 3x3 multiply
//      with the octant-stored, parity-signed Khat, inverse 2-D FFT, crop,
//   3. inverse x-FFT of every line, crop, and y = x - M (x + K x).
#include <cstdio>

#include <algorithm>
#include <mutex>
#include <string>

#include "fft_device.h"
#include "reg_fft.h"

// Position of x-frequency kx in its line of the x-spectra: natural order, or, for lines that
// take the four-step transform (xsplit = L2 > 1), (kx mod L2) (Px / L2) + kx / L2.
__host__ __device__ __forceinline__ int xpos(int kx, int Px, int xsplit) {
    if (xsplit <= 1) return kx;
    const int k1 = kx / xsplit;
    return (kx - k1 * xsplit) * (Px / xsplit) + k1;
}

template <class R>
__global__ void k_contrast(const c128 *chi, cpx<R> *M, long long N) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    c128 c = chi[i];
    c128 m = cdiv(c, mk(1.0 + c.re, c.im));  // M = chi / (1 + chi)
    M[i] = mk((R)m.re, (R)m.im);
}

__global__ void k_check_chi(const c128 *chi, long long N, int *bad) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    c128 c = chi[i];
    if (!isfinite(c.re) || !isfinite(c.im) || (c.re == -1.0 && c.im == 0.0)) atomicOr(bad, 1);
}

vie_status launch_check_chi(const c128 *chi, long long N, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_chi, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, chi, N, bad);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// one thread per cross-section position (z, y): does the contrast vanish along the whole x-line?
__global__ void k_line_flags(const c128 *M, int nx, int nyz, int *flags) {
    const int yz = blockIdx.x * blockDim.x + threadIdx.x;
    if (yz >= nyz) return;
    const c128 *m = M + (long long)yz * nx;
    int any = 0;
    for (int i = 0; i < nx && !any; ++i) any = m[i].re != 0.0 || m[i].im != 0.0;
    flags[yz] = any;
}

vie_status launch_line_flags(vie_op op, int *flags, hipStream_t s) {
    const int nyz = op->ny * op->nz;
    hipLaunchKernelGGL(k_line_flags, dim3((nyz + 255) / 256), dim3(256), 0, s, op->M64.as<const c128>(), op->nx, nyz,
                       flags);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

vie_status launch_contrast(vie_op op, const c128 *chi_dev, hipStream_t s) {
    long long N = op->N;
    unsigned g = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_contrast<double>, dim3(g), dim3(256), 0, s, chi_dev, op->M64.as<c128>(), N);
    hipLaunchKernelGGL(k_contrast<float>, dim3(g), dim3(256), 0, s, chi_dev, op->M32.as<c64>(), N);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

__global__ void k_rhs(const c128 *e, c128 *b, const c128 *M, long long N, long long total) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= total) return;
    b[i] = M[i % N] * e[i];
}

vie_status launch_rhs(vie_op op, const c128 *e, c128 *b, int nrhs, hipStream_t s) {
    long long total = 3LL * op->N * nrhs;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, e, b,
                       op->M64.as<c128>(), op->N, total);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// ---------------------------------------------------------------- setup
// Embedded periodic generator E[c][z][y][x] over (Pz, Py, Px).
__global__ void k_embed(const c128 *gen, c128 *E, int nx, int ny, int nz, int Px, int Py, int Pz) {
    long long P3 = (long long)Px * Py * Pz;
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= 6 * P3) return;
    int c = (int)(i / P3);
    long long r = i % P3;
    int x = (int)(r % Px), y = (int)((r / Px) % Py), z = (int)(r / ((long long)Px * Py));
    int ax = x < nx ? x : (Px - x < nx ? -(Px - x) : INT32_MAX);
    int ay = y < ny ? y : (Py - y < ny ? -(Py - y) : INT32_MAX);
    int az = z < nz ? z : (Pz - z < nz ? -(Pz - z) : INT32_MAX);
    c128 v = czero<double>();
    if (ax != INT32_MAX && ay != INT32_MAX && az != INT32_MAX) {
        int d[3] = {ax, ay, az};
        v = gen[(long long)c * nx * ny * nz + ((long long)abs(az) * ny + abs(ay)) * nx + abs(ax)];
        // components (xx, yy, zz, xy, xz, yz): odd in the two axes of an off-diagonal block
        const int oa[6] = {-1, -1, -1, 0, 0, 1}, ob[6] = {-1, -1, -1, 1, 2, 2};
        if (c >= 3) {
            double sg = 1.0;
            if (d[oa[c]] < 0) sg = -sg;
            if (d[ob[c]] < 0) sg = -sg;
            if (d[oa[c]] == 0 || d[ob[c]] == 0) sg = 0.0;  // odd: zero at zero offset
            v = mk(sg * v.re, sg * v.im);
        }
    }
    E[i] = v;
}

// In-place FFT of lines in global memory: line l starts at (l % nl1)*s1 + (l / nl1)*s2,
// element stride es.  One workgroup per line.
template <class R, int BPT>
__global__ void k_fft_lines(cpx<R> *data, long long nl1, long long s1, long long s2, long long es,
                            FftPlan plan, int inv) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    long long l = blockIdx.x;
    cpx<R> *base = data + (l % nl1) * s1 + (l / nl1) * s2;
    for (int i = threadIdx.x; i < plan.L; i += blockDim.x) a[i] = base[i * es];
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, plan, inv != 0);
    for (int i = threadIdx.x; i < plan.L; i += blockDim.x) base[i * es] = res[i];
}

// Octant extraction: khat[kx][kz][ky][c] = E[c][kz][ky][kx] / (Px Py Pz)
__global__ void k_extract(const c128 *E, c128 *k64, c64 *k32, int Px, int Py, int Pz, int Hx, int Hy,
                          int Hz, int xsplit) {
    long long total = (long long)Hx * Hy * Hz * 6;
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= total) return;
    int c = (int)(i % 6);
    long long r = i / 6;
    int ky = (int)(r % Hy);
    r /= Hy;
    int kz = (int)(r % Hz);
    int kx = (int)(r / Hz);
    double sc = 1.0 / ((double)Px * Py * Pz);
    c128 v = E[(long long)c * Px * Py * Pz + ((long long)kz * Py + ky) * Px + xpos(kx, Px, xsplit)];
    v = mk(v.re * sc, v.im * sc);
    k64[i] = v;
    if (k32) k32[i] = mk((float)v.re, (float)v.im);
}

// (x, y)-transformed generator for the direct z sum, octant in (kx, ky), real-space z offsets
// dz in [0, nz): khat[kx][ky][dz][c] = E[c][dz][ky][kx] / (Px Py)
__global__ void k_extract_xy(const c128 *E, c128 *k64, c64 *k32, int Px, int Py, int Pz, int Hx, int Hy, int nz,
                             int xsplit) {
    long long total = (long long)Hx * Hy * nz * 6;
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= total) return;
    int c = (int)(i % 6);
    long long r = i / 6;
    int dz = (int)(r % nz);
    r /= nz;
    int ky = (int)(r % Hy);
    int kx = (int)(r / Hy);
    double sc = 1.0 / ((double)Px * Py);
    c128 v = E[(long long)c * Px * Py * Pz + ((long long)dz * Py + ky) * Px + xpos(kx, Px, xsplit)];
    v = mk(v.re * sc, v.im * sc);
    k64[i] = v;
    if (k32) k32[i] = mk((float)v.re, (float)v.im);
}

// ---------------------------------------------------------------- lines longer than one workgroup's LDS
// Four-step transform of length L = L1 L2 (n = n1 + L1 n2, k = k2 + L2 k1), through the line's own
// storage in device memory:
//   columns: for every n1, the length-L2 DFT over n2, times W_L^{n1 k2}  -> [k2][n1]
//   rows:    for every k2, the length-L1 DFT over n1                     -> [k2][k1]
// so frequency k is left at position (k mod L2) L1 + k / L2 of its line (xpos).  The inverse runs
// the rows, then the columns with the conjugate twiddle, back to natural order.  A workgroup takes
// a tile of LT consecutive columns (rows of LT elements are contiguous, so loads and stores move
// LT-element segments) or one whole row.
#define LONG_LT 16

// columns forward: src line (zero beyond nx when the source is a vector of x-lines of length nx,
// src_len = nx; src_len = L for a line of the work buffer), dst = work line.
template <class R, int BPT>
__global__ void k_long_cols(const cpx<R> *src, int src_len, cpx<R> *dst, int L, int L1, FftPlan p2,
                            const cpx<R> *twL, int inv) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int L2 = p2.L, ntile = L1 / LONG_LT;
    const long long line = blockIdx.x / ntile;
    const int c0 = (blockIdx.x - (int)(line * ntile)) * LONG_LT;
    const cpx<R> *s = src + line * (long long)src_len;
    for (int i = threadIdx.x; i < L2 * LONG_LT; i += blockDim.x) {
        const int n2 = i / LONG_LT, j = i - n2 * LONG_LT;
        const int n = c0 + j + L1 * n2;
        a[i] = n < src_len ? s[n] : czero<R>();
    }
    __syncthreads();
    const LdsLines ln = {LONG_LT, 1, 0, LONG_LT, LONG_LT};
    cpx<R> *res = a;
    if (BPT > 0) fft_lds_inplace<R, (BPT > 0 ? BPT : 1)>(a, ln, p2, inv != 0);
    else res = fft_lds<R>(a, a + L2 * LONG_LT, ln, p2, inv != 0);
    cpx<R> *d = dst + line * (long long)L;
    for (int i = threadIdx.x; i < L2 * LONG_LT; i += blockDim.x) {
        const int k2 = i / LONG_LT, j = i - k2 * LONG_LT;
        const int q = (int)(((long long)(c0 + j) * k2) % L);
        cpx<R> v = res[i];
        if (q) v = v * tw_at(twL, q, inv != 0);
        d[(long long)k2 * L1 + c0 + j] = v;
    }
}

// rows, in place on the work buffer: one workgroup per (line, row)
template <class R, int BPT>
__global__ void k_long_rows(cpx<R> *work, int L, FftPlan p1, int inv) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int L1 = p1.L, L2 = L / L1;
    const long long line = blockIdx.x / L2;
    const int k2 = blockIdx.x - (int)(line * L2);
    cpx<R> *row = work + line * (long long)L + (long long)k2 * L1;
    for (int i = threadIdx.x; i < L1; i += blockDim.x) a[i] = row[i];
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, p1, inv != 0);
    for (int i = threadIdx.x; i < L1; i += blockDim.x) row[i] = res[i];
}

// columns inverse: conjugate twiddle, inverse length-L2 DFT over k2, and the line's first nx
// entries written as y = x - M (x + (K x)) (cropped product, eq. discrete_form)
template <class R, int BPT>
__global__ void k_long_cols_inv(const cpx<R> *work, int L, int L1, FftPlan p2, const cpx<R> *twL, const cpx<R> *x,
                                const cpx<R> *M, cpx<R> *y, int nx, int nyz) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int L2 = p2.L, ntile = L1 / LONG_LT;
    const long long line = blockIdx.x / ntile;
    const int c0 = (blockIdx.x - (int)(line * ntile)) * LONG_LT;
    const cpx<R> *w = work + line * (long long)L;
    for (int i = threadIdx.x; i < L2 * LONG_LT; i += blockDim.x) {
        const int k2 = i / LONG_LT, j = i - k2 * LONG_LT;
        const int q = (int)(((long long)(c0 + j) * k2) % L);
        cpx<R> v = w[(long long)k2 * L1 + c0 + j];
        a[i] = q ? v * tw_at(twL, q, true) : v;
    }
    __syncthreads();
    const LdsLines ln = {LONG_LT, 1, 0, LONG_LT, LONG_LT};
    cpx<R> *res = a;
    if (BPT > 0) fft_lds_inplace<R, (BPT > 0 ? BPT : 1)>(a, ln, p2, true);
    else res = fft_lds<R>(a, a + L2 * LONG_LT, ln, p2, true);
    const long long yz = line % nyz;
    const cpx<R> *xl = x + line * (long long)nx;
    const cpx<R> *ml = M + yz * nx;
    cpx<R> *yl = y + line * (long long)nx;
    for (int i = threadIdx.x; i < L2 * LONG_LT; i += blockDim.x) {
        const int n2 = i / LONG_LT, j = i - n2 * LONG_LT;
        const int n = c0 + j + L1 * n2;
        if (n < nx) {
            const cpx<R> xv = xl[n];
            yl[n] = xv - ml[n] * (xv + res[i]);
        }
    }
}

// Launch shape of the column kernels: LONG_LT lines of length L2 in LDS, ping-pong when both
// buffers fit in FFT_PINGPONG_LDS bytes, else in place with up to 4 butterflies per thread
// (threads enough for the radix-2 stages: (L2 / 2) LONG_LT <= 4 threads).
static void long_cols_shape(const FftPlan &p2, size_t esz, int *thr, size_t *lds, int *bpt) {
    *lds = 2 * esz * (size_t)p2.L * LONG_LT;
    *bpt = *lds > FFT_PINGPONG_LDS && fft_plan_inplace(p2) ? 4 : 0;
    if (*bpt) *lds /= 2;
    const int need = (p2.L / 2 * LONG_LT + 3) / 4;
    *thr = 256;
    while (*thr < need && *thr < 1024) *thr *= 2;
}

// Forward four-step transform of `lines` lines of length Px: columns (reading src, lines of
// src_len entries, zero beyond), then rows in place in dst.  inverse = true runs the rows only
// (the inverse columns are fused with the product's final combination, k_long_cols_inv).
template <class R>
static vie_status long_lines(vie_op op, const cpx<R> *src, int src_len, cpx<R> *dst, long long lines, bool inverse,
                             hipStream_t s) {
    const int L = op->Px, L1 = op->px1.L;
    const int ntile = L1 / LONG_LT;
    if (!inverse) {
        size_t lds;
        int thr, bpt;
        long_cols_shape(op->px2, sizeof(cpx<R>), &thr, &lds, &bpt);
#define LAUNCH_COLS(B)                                                                                         \
    vie_lds_attr((const void *)k_long_cols<R, B>, lds);                                                        \
    hipLaunchKernelGGL((k_long_cols<R, B>), dim3((unsigned)(lines * ntile)), dim3(thr), lds, s, src, src_len, dst, \
                       L, L1, op->px2, TwTable<R>::get(op->px), 0)
        if (bpt) {
            LAUNCH_COLS(4);
        } else {
            LAUNCH_COLS(0);
        }
#undef LAUNCH_COLS
        VIE_HIP(hipGetLastError());
    }
    size_t ldsr;
    int thr, bpt;
    fft_line_shape(op->px1, sizeof(cpx<R>), &thr, &ldsr, &bpt);
#define LAUNCH_ROWS(B)                                                                                        \
    vie_lds_attr((const void *)k_long_rows<R, B>, ldsr);                                                      \
    hipLaunchKernelGGL((k_long_rows<R, B>), dim3((unsigned)(lines * op->px2.L)), dim3(thr), ldsr, s, dst, L, op->px1, \
                       inverse ? 1 : 0)
    VIE_BPT_SWITCH(bpt, LAUNCH_ROWS);
#undef LAUNCH_ROWS
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

static int block_for(int L) {
    int t = 64;
    while (t < 256 && t * 4 < L) t *= 2;
    return t;
}

vie_status build_kernel_transform(vie_op op, hipStream_t s) {
    const int Px = op->Px, Py = op->Py, Pz = op->Pz;
    long long P3 = (long long)Px * Py * Pz;
    DevBuf E;
    VIE_CHECK(E.ensure(sizeof(c128) * 6 * P3));
    long long tot = 6 * P3;
    hipLaunchKernelGGL(k_embed, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, op->gen.as<c128>(),
                       E.as<c128>(), op->nx, op->ny, op->nz, Px, Py, Pz);
    VIE_HIP(hipGetLastError());
    // x lines, y lines, z lines
    struct {
        const FftPlan *p;
        long long nl1, s1, s2, es, nlines;
    } passes[3] = {
        {&op->px, 6LL * Py * Pz, Px, 0, 1, 6LL * Py * Pz},
        {&op->py, Px, 1, (long long)Px * Py, Px, 6LL * Pz * Px},
        {&op->pz, (long long)Px * Py, 1, P3, (long long)Px * Py, 6LL * Px * Py},
    };
    for (int pi = 0; pi < 3; ++pi) {
        auto &ps = passes[pi];
        if (ps.p->L == 1) continue;
        if (pi == 2 && op->direct_z) continue;  // z offsets stay in real space
        if (pi == 0 && op->xsplit > 1) {        // x lines longer than the LDS: four-step, in place
            VIE_CHECK(long_lines<double>(op, E.as<c128>(), Px, E.as<c128>(), ps.nlines, false, s));
            continue;
        }
        size_t lds;
        int thr, bpt;
        fft_line_shape(*ps.p, sizeof(c128), &thr, &lds, &bpt);
#define LAUNCH_LINES(B)                                                                                   \
    vie_lds_attr((const void *)k_fft_lines<double, B>, lds);                                              \
    hipLaunchKernelGGL((k_fft_lines<double, B>), dim3((unsigned)ps.nlines), dim3(thr), lds, s, E.as<c128>(), \
                       ps.nl1, ps.s1, ps.s2, ps.es, *ps.p, 0)
        VIE_BPT_SWITCH(bpt, LAUNCH_LINES);
#undef LAUNCH_LINES
        VIE_HIP(hipGetLastError());
    }
    long long H = op->direct_z ? (long long)op->Hx * op->Hy * op->nz * 6 : (long long)op->Hx * op->Hy * op->Hz * 6;
    VIE_CHECK(op->khat64.ensure(sizeof(c128) * H));
    if (op->has_c64) VIE_CHECK(op->khat32.ensure(sizeof(c64) * H));
    if (op->direct_z)
        hipLaunchKernelGGL(k_extract_xy, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, s, E.as<c128>(),
                           op->khat64.as<c128>(), op->has_c64 ? op->khat32.as<c64>() : nullptr, Px, Py, Pz,
                           op->Hx, op->Hy, op->nz, op->xsplit);
    else
        hipLaunchKernelGGL(k_extract, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, s, E.as<c128>(),
                           op->khat64.as<c128>(), op->has_c64 ? op->khat32.as<c64>() : nullptr, Px, Py, Pz,
                           op->Hx, op->Hy, op->Hz, op->xsplit);
    VIE_HIP(hipGetLastError());
    VIE_HIP(hipStreamSynchronize(s));
    E.release();
    return VIE_OK;
}

// MODE 0: forward, x-line (nx entries, zero beyond) -> x-spectra line; MODE 1: inverse,
// x-spectra line -> y = x - M (x + line) on the first nx entries.  With a line map, workgroup b
// takes line lmap[b mod nmap] of right-hand side b / nmap (3 nyz lines each).
template <class R, int R1, int R2, int R3, int R4, int MODE>
__global__ void __launch_bounds__((rfft::Radices<R1, R2, R3, R4>::T))
k_xline_reg(const cpx<R> *__restrict__ in, cpx<R> *__restrict__ out, const cpx<R> *__restrict__ x,
            const cpx<R> *__restrict__ M, int nx, int nyz, const cpx<R> *__restrict__ tw, const int *__restrict__ lmap,
            int nmap) {
    constexpr int L = rfft::Radices<R1, R2, R3, R4>::L;
    long long line = blockIdx.x;
    if (lmap) {
        const int rh = (int)(blockIdx.x / (unsigned)nmap);
        line = (long long)rh * 3 * nyz + lmap[blockIdx.x - (unsigned)rh * nmap];
    }
    const cpx<R> *src = MODE == 0 ? in + line * nx : in + line * L;
    const cpx<R> *xl = x + line * nx;
    const cpx<R> *ml = M + (line % nyz) * nx;
    cpx<R> *dl = MODE == 0 ? out + line * L : out + line * nx;
    rfft::reg_line<R, R1, R2, R3, R4, MODE == 1>(
        tw, [&](int i) -> cpx<R> { return MODE == 0 ? (i < nx ? src[i] : czero<R>()) : src[i]; },
        [&](int i, cpx<R> v) {
            if (MODE == 0) {
                dl[i] = v;
            } else if (i < nx) {
                const cpx<R> xv = xl[i];
                dl[i] = xv - ml[i] * (xv + v);
            }
        });
}

// y = x on the listed lines (nx entries each) of right-hand side blockIdx.y (3 nyz lines each):
// the product on a line whose contrast is zero along all of x.
template <class R>
__global__ void k_copy_lines(const cpx<R> *__restrict__ x, cpx<R> *__restrict__ y, const int *__restrict__ lines,
                             int nlines, int nx, int nyz) {
    const long long base = (long long)blockIdx.y * 3 * nyz * nx;
    const long long total = (long long)nlines * nx;
    const FastDiv fnx(nx);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int li = fnx.div((int)i);
        const long long e = base + (long long)lines[li] * nx + (i - (long long)li * nx);
        y[e] = x[e];
    }
}

// ---------------------------------------------------------------- product
// pass 1: one workgroup per x-line (rhs, a, z, y): zero-pad to Px, forward FFT.
template <class R, int BPT>
__global__ void k_xfwd(const cpx<R> *x, cpx<R> *work, int nx, FftPlan plan) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    long long line = blockIdx.x;
    const cpx<R> *src = x + line * nx;
    for (int i = threadIdx.x; i < plan.L; i += blockDim.x) a[i] = i < nx ? src[i] : czero<R>();
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, plan, false);
    cpx<R> *dst = work + line * plan.L;
    for (int i = threadIdx.x; i < plan.L; i += blockDim.x) dst[i] = res[i];
}

// Block b of a grid of 8 * ceil(count / 8) works on index (b % 8) * ceil(count / 8) + b / 8
// (>= count: nothing): workgroups are dealt to the eight XCDs round-robin, so each XCD gets
// a contiguous range and neighbouring x-frequencies share the L2 lines of their strided rows.
__device__ __forceinline__ int xcd_block(int b, int count) {
    const int per = (count + 7) / 8;
    return (b % 8) * per + b / 8;
}

// pass 2: one workgroup per (PLANE_KB consecutive x-frequencies, rhs); the planes are
// processed one after another so the cache lines of the strided gathers are reused.
#define PLANE_KB 1
template <class R>
__global__ void k_plane(cpx<R> *work, const cpx<R> *khat, int ny, int nz, int Px, int Hx, int Hy, int Hz,
                        FftPlan py, FftPlan pz, int xsplit) {
    const int Py = py.L, Pz = pz.L;
    const int plane = Py * Pz;
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    cpx<R> *b = a + 3 * plane;
    for (int kk = 0; kk < PLANE_KB; ++kk) {
    const int kx = xcd_block(blockIdx.x * PLANE_KB + kk, Px);
    if (kx >= Px) break;
    cpx<R> *base = work + (long long)blockIdx.y * 3 * ny * nz * Px + xpos(kx, Px, xsplit);
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * plane; i += blockDim.x) a[i] = czero<R>();
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * ny * nz; i += blockDim.x) {
        int y = i % ny, z = (i / ny) % nz, c = i / (ny * nz);
        a[c * plane + z * Py + y] = base[(long long)i * Px];
    }
    __syncthreads();
    cpx<R> *buf = a, *oth = b;
    // forward along y: rows z < nz of each component
    if (Py > 1) {
        LdsLines ly = {nz, Py, plane, 1, 3 * nz};
        cpx<R> *r = fft_lds<R>(buf, oth, ly, py, false);
        oth = (r == buf) ? oth : buf;
        buf = r;
    }
    // forward along z: all Py columns
    if (Pz > 1) {
        LdsLines lz = {Py, 1, plane, Py, 3 * Py};
        cpx<R> *r = fft_lds<R>(buf, oth, lz, pz, false);
        oth = (r == buf) ? oth : buf;
        buf = r;
    }
    // 3x3 multiply with the parity-signed octant transform
    {
        int kxo = kx <= Px - kx ? kx : Px - kx;
        bool fx = kx > Px - kx;
        const cpx<R> *kh = khat + (long long)kxo * Hz * Hy * 6;
        for (int i = threadIdx.x; i < plane; i += blockDim.x) {
            int ky = i % Py, kz = i / Py;
            int kyo = ky <= Py - ky ? ky : Py - ky;
            int kzo = kz <= Pz - kz ? kz : Pz - kz;
            bool fy = ky > Py - ky, fz = kz > Pz - kz;
            const cpx<R> *k6 = kh + ((long long)kzo * Hy + kyo) * 6;
            cpx<R> kxx = k6[0], kyy = k6[1], kzz = k6[2], kxy = k6[3], kxz = k6[4], kyz = k6[5];
            if (fx != fy) kxy = mk(-kxy.re, -kxy.im);
            if (fx != fz) kxz = mk(-kxz.re, -kxz.im);
            if (fy != fz) kyz = mk(-kyz.re, -kyz.im);
            cpx<R> u0 = buf[i], u1 = buf[plane + i], u2 = buf[2 * plane + i];
            buf[i] = kxx * u0 + kxy * u1 + kxz * u2;
            buf[plane + i] = kxy * u0 + kyy * u1 + kyz * u2;
            buf[2 * plane + i] = kxz * u0 + kyz * u1 + kzz * u2;
        }
        __syncthreads();
    }
    if (Pz > 1) {
        LdsLines lz = {Py, 1, plane, Py, 3 * Py};
        cpx<R> *r = fft_lds<R>(buf, oth, lz, pz, true);
        oth = (r == buf) ? oth : buf;
        buf = r;
    }
    if (Py > 1) {
        LdsLines ly = {nz, Py, plane, 1, 3 * nz};
        cpx<R> *r = fft_lds<R>(buf, oth, ly, py, true);
        oth = (r == buf) ? oth : buf;
        buf = r;
    }
    for (int i = threadIdx.x; i < 3 * ny * nz; i += blockDim.x) {
        int y = i % ny, z = (i / ny) % nz, c = i / (ny * nz);
        base[(long long)i * Px] = buf[c * plane + z * Py + y];
    }
    }
}

// pass 2 for cross-sections with few z layers: one workgroup per (x-frequency, rhs).
// Forward y-FFT of the 3 nz zero-padded rows, then for every y-frequency the z coupling as a
// direct sum over the nz z-offsets of the (x, y)-transformed generator (its z-Toeplitz
// structure kept in real space, parities applied per axis), inverse y-FFT, crop.
template <class R>
__global__ void k_plane_dz(cpx<R> *work, const cpx<R> *khat, int ny, int nz, int Px, int Hy, FftPlan py,
                           int xsplit) {
    const int Py = py.L;
    const int rows = 3 * nz;
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);  // [3][nz][Py] lines
    cpx<R> *b = a + rows * Py;                          // [3][nz][Py] second buffer
    cpx<R> *G = b + rows * Py;                          // [nz][6][Hy] (y-frequency fastest)
    const int kx = xcd_block(blockIdx.x, Px);
    if (kx >= Px) return;
    const int kxo = kx <= Px - kx ? kx : Px - kx;
    const bool fx = kx > Px - kx;
    cpx<R> *base = work + (long long)blockIdx.y * 3 * ny * nz * Px + xpos(kx, Px, xsplit);
    const cpx<R> *kh = khat + (long long)kxo * Hy * nz * 6;
    const FastDiv f6nz(6 * nz), fpy(Py), fny(ny);
    for (int i = threadIdx.x; i < Hy * nz * 6; i += blockDim.x) {
        const int kyo = f6nz.div(i), e = i - kyo * 6 * nz;  // source layout [Hy][nz][6]
        const int dz = e / 6, c = e - dz * 6;
        G[(dz * 6 + c) * Hy + kyo] = kh[i];
    }
    for (int i = threadIdx.x; i < rows * Py; i += blockDim.x) {
        const int rz = fpy.div(i), y = i - rz * Py;  // rz = c * nz + z
        a[i] = y < ny ? base[((long long)rz * ny + y) * Px] : czero<R>();
    }
    __syncthreads();
    LdsLines ln = {rows, Py, 0, 1, rows};
    cpx<R> *spec = a, *prod = b;  // spectra, then the coupled products in the other buffer
    if (Py > 1) {
        spec = fft_lds<R>(a, b, ln, py, false);
        prod = spec == a ? b : a;
    }
    // z coupling, one (z, ky) entry per thread with all three components: the 3x3 block of
    // the transformed generator at offset z - z' with its parity signs (xy odd in x and y,
    // xz in x and z, yz in y and z).
    const R sx = fx ? R(-1) : R(1);
    for (int o = threadIdx.x; o < nz * Py; o += blockDim.x) {
        const int z = fpy.div(o), ky = o - z * Py;
        const int kyo = ky <= Py - ky ? ky : Py - ky;
        const R sy = ky > Py - ky ? R(-1) : R(1);
        const R sxy = sx * sy;
        const cpx<R> *g = G + kyo;
        const cpx<R> *u = spec + ky;
        cpx<R> a0 = czero<R>(), a1 = czero<R>(), a2 = czero<R>();
        for (int zp = 0; zp < nz; ++zp) {
            const int dz = z - zp;
            const R sz = dz < 0 ? R(-1) : R(1);
            const cpx<R> *gz = g + (dz < 0 ? -dz : dz) * 6 * Hy;
            const cpx<R> gxx = gz[0], gyy = gz[Hy], gzz = gz[2 * Hy];
            const cpx<R> gxy = sxy * gz[3 * Hy], gxz = (sx * sz) * gz[4 * Hy], gyz = (sy * sz) * gz[5 * Hy];
            const cpx<R> u0 = u[zp * Py], u1 = u[(nz + zp) * Py], u2 = u[(2 * nz + zp) * Py];
            a0 = a0 + gxx * u0 + gxy * u1 + gxz * u2;
            a1 = a1 + gxy * u0 + gyy * u1 + gyz * u2;
            a2 = a2 + gxz * u0 + gyz * u1 + gzz * u2;
        }
        prod[z * Py + ky] = a0;
        prod[(nz + z) * Py + ky] = a1;
        prod[(2 * nz + z) * Py + ky] = a2;
    }
    __syncthreads();
    cpx<R> *res = prod;
    if (Py > 1) res = fft_lds<R>(prod, spec, ln, py, true);
    for (int i = threadIdx.x; i < rows * ny; i += blockDim.x) {
        const int rz = fny.div(i), y = i - rz * ny;
        base[((long long)rz * ny + y) * Px] = res[rz * Py + y];
    }
}

// pass 2 for thin cross-sections (direct z sum) with the y period and the layer count fixed at
// compile time: one workgroup per (x-frequency, group of right-hand sides), the group's planes
// processed one after another with the x-frequency's transformed generator staged in LDS once.
// The y-FFT of period PY = P1 P2 runs on registers in two steps with one LDS exchange:
// y = n2 + P2 n1, ky = k1 + P1 k2; step 1 transforms over n1 (zero-padded rows, loaded straight
// from the x-spectra), multiplies by W_PY^{n2 k1} and leaves [k1][n2] in LDS; step 2 transforms
// over n2 into natural order.  The z coupling reads every (component, layer) of a y-frequency from
// LDS; the inverse runs the two steps in reverse and stores the cropped rows.
// PL planes (consecutive right-hand sides of the group) run side by side, each on its own
// threads and LDS plane, sharing the staged generator: with PL = 2 a workgroup holds 2 x 4.5
// wavefronts of items, which the four SIMDs share more evenly than one plane's 4.5.
// TAIL: a plane takes four wavefronts (256 threads) although the 96-point phases have 288 items
// (24 lines x 12, or 3 components x 96 y-frequencies): the last 32 items of such a phase are
// split by output over all 256 threads (one DFT output, or one layer of the z sum, each), so the
// four SIMDs get equal work and two workgroups fit a compute unit.
template <int PY, int P1, int P2, int NZ, bool TAIL>
struct PlaneThreads {
    static constexpr int L = 3 * NZ, PM = P1 > P2 ? P1 : P2;
    static constexpr int value = TAIL ? 256 : 64 * ((L * PM + 63) / 64);
};
template <class R, int PY, int P1, int P2, int NZ, int PL, bool TAIL>
__global__ void __launch_bounds__((PL * PlaneThreads<PY, P1, P2, NZ, TAIL>::value))
k_plane_reg(cpx<R> *__restrict__ work, const cpx<R> *__restrict__ khat, const cpx<R> *__restrict__ twtab, int ny,
            int Px, int nrhs, int rb, int xsplit, const int *__restrict__ yzf, int zero_in) {
    static_assert(P1 * P2 == PY, "PY = P1 P2");
    constexpr int Hy = PY / 2 + 1;            // stored y-frequencies 0 .. PY/2 (octant)
    constexpr int L = 3 * NZ;                 // lines: (component, layer)
    constexpr int NTP = PlaneThreads<PY, P1, P2, NZ, TAIL>::value;  // threads per plane
    constexpr int NT = PL * NTP;
    // items past NTP in the (line, k1) and (component, y-frequency) phases, split by output
    constexpr int NTK = L * P1 > NTP ? L * P1 - NTP : 0;
    constexpr int NTC = 3 * PY > NTP ? 3 * PY - NTP : 0;
    static_assert(L * P2 <= NTP, "one (line, n2) item per thread");
    static_assert(NTK * P2 <= NTP && NTC * NZ <= NTP, "tail outputs fit the threads");
    static_assert(TAIL || (NTK == 0 && NTC == 0), "tails only in the four-wavefront form");
    // line stride: room for the padded exchange layouts [k1][P2 + 1] and [n2][P1 + 1] (odd strides,
    // so the transposed reads spread over the LDS banks) as well as the natural order [PY]
    constexpr int SP = PY + (P1 > P2 ? P1 : P2);
    const int h = PL > 1 ? (int)threadIdx.x / NTP : 0;                // plane of this thread
    const int t = (int)threadIdx.x - h * NTP;                        // thread within the plane
    cpx<R> *S = reinterpret_cast<cpx<R> *>(vie_smem) + h * L * SP;    // [L][SP] plane h
    cpx<R> *G = reinterpret_cast<cpx<R> *>(vie_smem) + PL * L * SP;   // [NZ][6][Hy] transformed generator
    cpx<R> *W = G + NZ * 6 * Hy;                                     // [PY] twiddles W_PY^q
    const int kx = xcd_block(blockIdx.x, Px);
    if (kx >= Px) return;
    const int kxo = kx <= Px - kx ? kx : Px - kx;
    const R sx = kx > Px - kx ? R(-1) : R(1);
    {
        const cpx<R> *kh = khat + (long long)kxo * Hy * NZ * 6;
        for (int i = threadIdx.x; i < Hy * NZ * 6; i += NT) {
            const int kyo = i / (6 * NZ), e = i - kyo * 6 * NZ;  // source layout [Hy][NZ][6]
            G[e * Hy + kyo] = kh[i];                              // e = dz * 6 + c
        }
        for (int i = threadIdx.x; i < PY; i += NT) W[i] = twtab[i];
    }
    const int r0 = blockIdx.y * rb, r1 = min(nrhs, r0 + rb);
    const long long xo = xpos(kx, Px, xsplit), rstride = (long long)L * ny * Px;
    // the zero-padded column of item (line, n2) of the forward step 1; the next plane's column
    // is loaded while the current plane is processed (every barrier below orders LDS only)
    // ny <= (PY + 1) / 2, so only the first NNZ entries of a column (y = n2 + P2 n1) can be
    // nonzero: the others are compile-time zeros in the step-1 DFT.  Offsets within a plane's
    // slab are 32-bit (the host keeps the slab below 2^31 entries) from a uniform base.
    constexpr int NNZ = ((PY + 1) / 2 + P2 - 1) / P2;
    const int line1 = t / P2, n21 = t - line1 * P2;
    const unsigned ystep = (unsigned)(P2 * Px);
    const unsigned off1 = (unsigned)((line1 * ny + n21) * Px);
    // bit n1: the entry y = n2 + P2 n1 of this thread's column lies on a line with contrast (with
    // yzf given, lines without contrast are not stored and, with zero_in, not loaded)
    unsigned keep = 0;
    rfft::sfor<P1>([&](auto ic) {
        constexpr int n1 = decltype(ic)::value;
        const int y = n21 + P2 * n1;
        if (t < L * P2 && y < ny && (!yzf || yzf[(line1 % NZ) * ny + y])) keep |= 1u << n1;
    });
    const unsigned keep_in = zero_in ? keep : ~0u;
    cpx<R> vn[NNZ];
    rfft::sfor<NNZ>([&](auto ic) { vn[decltype(ic)::value] = czero<R>(); });
    auto load_col = [&](int rhs) {
        const cpx<R> *src = work + rhs * rstride + xo;
        rfft::sfor<NNZ>([&](auto ic) {
            constexpr int n1 = decltype(ic)::value;
            const int y = n21 + P2 * n1;
            vn[n1] = (t < L * P2 && y < ny && ((keep_in >> n1) & 1u)) ? src[off1 + n1 * ystep] : czero<R>();
        });
    };
    if (r0 + h < r1) load_col(r0 + h);
    // every thread runs the same iterations (barriers); a plane past the group's end computes on
    // whatever its registers hold and stores nothing
    for (int rr = r0; rr < r1; rr += PL) {
        // the thread index passes through an empty asm statement once per plane, so the indices
        // and LDS addresses derived from it are recomputed in each phase instead of being kept
        // live across the whole loop (fewer registers held)
        int tq = t;
        asm volatile("" : "+v"(tq));
        const int rhs = rr + h;
        const bool live = rhs < r1;
        cpx<R> *base = work + (live ? rhs : r0) * rstride + xo;
        rfft::lds_barrier();  // G, W staged; the previous plane's last reads of S are done
        // forward step 1: item (line, n2) transforms its zero-padded column over n1
        if (tq < L * P2) {
            const int line = line1, n2 = n21;
            cpx<R> v[P1];
            rfft::sfor<P1>([&](auto ic) {
                constexpr int n1 = decltype(ic)::value;
                if constexpr (n1 < NNZ) v[n1] = vn[n1];
                else v[n1] = czero<R>();
            });
            if (rhs + PL < r1) load_col(rhs + PL);
            rfft::Dft<R, P1, false>::run(v);
            rfft::sfor<P1>([&](auto ic) {
                constexpr int k1 = decltype(ic)::value;
                S[line * SP + k1 * (P2 + 1) + n2] = k1 == 0 ? v[k1] : v[k1] * W[n2 * k1];
            });
        }
        rfft::lds_barrier();
        // forward step 2: item (line, k1) transforms over n2 -> ky = k1 + P1 k2
        {
            cpx<R> u[P2];
            const int line = tq / P1, k1 = tq - line * P1;
            const bool act = tq < L * P1;
            if (act)
                rfft::sfor<P2>([&](auto ic) { u[decltype(ic)::value] = S[line * SP + k1 * (P2 + 1) + decltype(ic)::value]; });
            // tail item NTP + ti: thread (ti, k2) forms output k2 by the definition of the DFT
            cpx<R> tv = czero<R>();
            int tdst = -1;
            if constexpr (NTK > 0) {
                const int ti = tq / P2, k2 = tq - ti * P2;
                if (ti < NTK) {
                    const int it = NTP + ti, tl = it / P1, tk = it - tl * P1;
                    const cpx<R> *col = S + tl * SP + tk * (P2 + 1);
                    rfft::sfor<P2>([&](auto ic) {
                        constexpr int n2 = decltype(ic)::value;
                        tv = cfma(tv, col[n2], W[((n2 * k2) % P2) * (PY / P2)]);
                    });
                    tdst = tl * SP + tk + P1 * k2;
                }
            }
            rfft::lds_barrier();
            if (act) {
                rfft::Dft<R, P2, false>::run(u);
                rfft::sfor<P2>([&](auto ic) { S[line * SP + k1 + P1 * decltype(ic)::value] = u[decltype(ic)::value]; });
            }
            if (NTK > 0 && tdst >= 0) S[tdst] = tv;
        }
        rfft::lds_barrier();
        // z coupling: item (c, ky) forms component c of its y-frequency at every layer z, the sum
        // over z' and c' of the (c, c') block of the transformed generator at offset z - z' with the
        // parity signs (xy odd in x and y, xz in x and z, yz in y and z).  The source components are
        // taken one at a time (NZ spectra in registers); every item reads before any writes back.
        {
            static_assert(3 * PY <= NTP + NTC, "coupling items: one per thread plus the tail");
            const bool act = tq < 3 * PY;
            const int c = tq / PY, ky = tq - c * PY;
            cpx<R> acc[NZ];
            rfft::sfor<NZ>([&](auto iz) { acc[decltype(iz)::value] = czero<R>(); });
            if (act) {
                const int kyo = ky <= PY - ky ? ky : PY - ky;
                const R sy = ky > PY - ky ? R(-1) : R(1);
#pragma unroll 1
                for (int cp = 0; cp < 3; ++cp) {
                    cpx<R> uc[NZ];
                    rfft::sfor<NZ>([&](auto iz) { uc[decltype(iz)::value] = S[(cp * NZ + decltype(iz)::value) * SP + ky]; });
                    const bool off = c != cp;
                    const int e = off ? c + cp + 2 : c;  // block index (xx yy zz xy xz yz)
                    const R pxy = (off && (c == 0 || cp == 0) ? sx : R(1)) * (off && (c == 1 || cp == 1) ? sy : R(1));
                    const bool zodd = off && (c == 2 || cp == 2);
                    const cpx<R> *ge = G + e * Hy + kyo;
                    rfft::sfor<2 * NZ - 1>([&](auto id) {
                        constexpr int dz = decltype(id)::value - (NZ - 1);
                        constexpr int adz = dz < 0 ? -dz : dz;
                        const cpx<R> g = ((zodd && dz < 0) ? -pxy : pxy) * ge[adz * 6 * Hy];
                        rfft::sfor<NZ>([&](auto iz) {
                            constexpr int z = decltype(iz)::value, zp = z - dz;
                            if constexpr (zp >= 0 && zp < NZ) acc[z] = cfma(acc[z], g, uc[zp]);
                        });
                    });
                }
            }
            // tail item NTP + ti = (component tc, y-frequency tk): thread (ti, z) forms its layer z
            cpx<R> tv = czero<R>();
            int tdst = -1;
            if constexpr (NTC > 0) {
                const int ti = tq / NZ, z = tq - ti * NZ;
                if (ti < NTC) {
                    const int it = NTP + ti, tc = it / PY, tk = it - tc * PY;
                    const int kyo = tk <= PY - tk ? tk : PY - tk;
                    const R sy = tk > PY - tk ? R(-1) : R(1);
#pragma unroll 1
                    for (int cp = 0; cp < 3; ++cp) {
                        const bool off = tc != cp;
                        const int e = off ? tc + cp + 2 : tc;
                        const R pxy = (off && (tc == 0 || cp == 0) ? sx : R(1)) * (off && (tc == 1 || cp == 1) ? sy : R(1));
                        const bool zodd = off && (tc == 2 || cp == 2);
                        const cpx<R> *ge = G + e * Hy + kyo;
                        rfft::sfor<NZ>([&](auto izp) {
                            constexpr int zp = decltype(izp)::value;
                            const int dz = z - zp, adz = dz < 0 ? -dz : dz;
                            const cpx<R> g = ((zodd && dz < 0) ? -pxy : pxy) * ge[adz * 6 * Hy];
                            tv = cfma(tv, g, S[(cp * NZ + zp) * SP + tk]);
                        });
                    }
                    tdst = (tc * NZ + z) * SP + tk;
                }
            }
            rfft::lds_barrier();
            if (act) rfft::sfor<NZ>([&](auto iz) { S[(c * NZ + decltype(iz)::value) * SP + ky] = acc[decltype(iz)::value]; });
            if (NTC > 0 && tdst >= 0) S[tdst] = tv;
        }
        rfft::lds_barrier();
        // inverse step A: item (line, k1) transforms over k2, multiplies by conj W_PY^{n2 k1}
        {
            cpx<R> u[P2];
            const int line = tq / P1, k1 = tq - line * P1;
            const bool act = tq < L * P1;
            if (act) rfft::sfor<P2>([&](auto ic) { u[decltype(ic)::value] = S[line * SP + k1 + P1 * decltype(ic)::value]; });
            // tail item NTP + ti: thread (ti, n2) forms output n2 by the definition of the inverse DFT
            cpx<R> tv = czero<R>();
            int tdst = -1;
            if constexpr (NTK > 0) {
                const int ti = tq / P2, n2 = tq - ti * P2;
                if (ti < NTK) {
                    const int it = NTP + ti, tl = it / P1, tk = it - tl * P1;
                    const cpx<R> *row = S + tl * SP + tk;
                    rfft::sfor<P2>([&](auto ic) {
                        constexpr int k2 = decltype(ic)::value;
                        tv = cfma(tv, row[P1 * k2], conjg(W[((n2 * k2) % P2) * (PY / P2)]));
                    });
                    if (n2 > 0) tv = tv * conjg(W[n2 * tk]);
                    tdst = tl * SP + n2 * (P1 + 1) + tk;
                }
            }
            rfft::lds_barrier();
            if (act) {
                rfft::Dft<R, P2, true>::run(u);
                rfft::sfor<P2>([&](auto ic) {
                    constexpr int n2 = decltype(ic)::value;
                    S[line * SP + n2 * (P1 + 1) + k1] = n2 == 0 ? u[n2] : u[n2] * conjg(W[n2 * k1]);
                });
            }
            if (NTK > 0 && tdst >= 0) S[tdst] = tv;
        }
        rfft::lds_barrier();
        // inverse step B: item (line, n2) transforms over k1 -> y = n2 + P2 n1; cropped store
        if (tq < L * P2) {
            const int line = tq / P2, n2 = tq - line * P2;
            cpx<R> v[P1];
            rfft::sfor<P1>([&](auto ic) { v[decltype(ic)::value] = S[line * SP + n2 * (P1 + 1) + decltype(ic)::value]; });
            rfft::Dft<R, P1, true>::run(v);
            const unsigned off = (unsigned)((line * ny + n2) * Px);
            rfft::sfor<P1>([&](auto ic) {
                constexpr int n1 = decltype(ic)::value;
                const int y = n2 + P2 * n1;
                if (live && y < ny && ((keep >> n1) & 1u)) base[off + n1 * ystep] = v[n1];
            });
        }
    }
}

// pass 2 split in three, for cross-sections whose (y, z) plane does not fit one workgroup's LDS
// (few z layers, direct z sum).  yb[rhs][kx][row][ky], row = c*nz + z, holds y-spectra.
// (a) forward y-FFT of `lg` zero-padded rows per workgroup (rows of one (rhs, x-frequency)).
template <class R>
__global__ void k_ysplit_fwd(const cpx<R> *work, cpx<R> *yb, int ny, int nz, int Px, int lg, FftPlan py,
                             int xsplit) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem), *b = a + lg * py.L;
    const int Py = py.L, rows = 3 * nz, ngr = (rows + lg - 1) / lg;
    const int g = blockIdx.x % ngr;
    const int kx = xcd_block(blockIdx.x / ngr, Px);
    if (kx >= Px) return;
    const long long rhs = blockIdx.y;
    const cpx<R> *base = work + rhs * 3LL * ny * nz * Px + xpos(kx, Px, xsplit);
    const int r0 = g * lg, nr = min(lg, rows - r0);
    for (int i = threadIdx.x; i < lg * Py; i += blockDim.x) {
        const int l = i / Py, y = i - l * Py;
        a[i] = (l < nr && y < ny) ? base[((long long)(r0 + l) * ny + y) * Px] : czero<R>();
    }
    __syncthreads();
    const LdsLines ln = {lg, Py, 0, 1, lg};
    cpx<R> *res = Py > 1 ? fft_lds<R>(a, b, ln, py, false) : a;
    cpx<R> *dst = yb + ((rhs * Px + kx) * rows + r0) * (long long)Py;
    for (int i = threadIdx.x; i < nr * Py; i += blockDim.x) dst[i] = res[i];
}

// (b) z coupling: one workgroup per (rhs, x-frequency, tile of KB = 256 / nz y-frequencies),
// one thread per (y-frequency, z) computing its three components as a direct sum over the z
// offsets with the 3x3 blocks of the (x, y)-transformed generator (parity signs as in the
// fused pass); yb -> yc.  The tile's y-spectra (3 nz rows) and generator blocks ([dz][c] per
// y-frequency, padded against bank conflicts) are staged in LDS with coalesced loads, and the
// results leave through LDS as coalesced rows.
template <class R>
__global__ void __launch_bounds__(256) k_ysplit_couple(const cpx<R> *__restrict__ yb, cpx<R> *__restrict__ yc,
                                                       const cpx<R> *__restrict__ khat, int nz, int Px, int Py,
                                                       int Hy) {
    cpx<R> *us = reinterpret_cast<cpx<R> *>(vie_smem);  // [3 nz][KB] y-spectra, then results
    const int KB = 256 / nz, rows = 3 * nz, gst = 6 * nz + 1;
    cpx<R> *gs = us + rows * KB;                        // [KB][gst] generator blocks
    const int ntile = (Py + KB - 1) / KB;
    const int kx = blockIdx.x / ntile, ky0 = (blockIdx.x - kx * ntile) * KB;
    const int kb = min(KB, Py - ky0);
    const long long rhs = blockIdx.y;
    const int kxo = kx <= Px - kx ? kx : Px - kx;
    const R sx = kx > Px - kx ? R(-1) : R(1);
    const cpx<R> *u = yb + (rhs * Px + kx) * rows * (long long)Py + ky0;
    cpx<R> *o = yc + (rhs * Px + kx) * rows * (long long)Py + ky0;
    for (int e = threadIdx.x; e < rows * KB; e += blockDim.x) {
        const int r = e / KB, j = e - r * KB;
        us[e] = j < kb ? u[(long long)r * Py + j] : czero<R>();
    }
    for (int e = threadIdx.x; e < KB * 6 * nz; e += blockDim.x) {
        const int j = e / (6 * nz), q = e - j * 6 * nz;
        const int ky = ky0 + j, kyo = ky <= Py - ky ? ky : Py - ky;
        gs[j * gst + q] = j < kb ? khat[((long long)kxo * Hy + kyo) * nz * 6 + q] : czero<R>();
    }
    __syncthreads();
    const int j = threadIdx.x / nz, z = threadIdx.x - j * nz;
    cpx<R> a0 = czero<R>(), a1 = czero<R>(), a2 = czero<R>();
    if (j < kb) {
        const int ky = ky0 + j;
        const R sy = ky > Py - ky ? R(-1) : R(1), sxy = sx * sy;
        const cpx<R> *g = gs + j * gst;
        for (int zp = 0; zp < nz; ++zp) {
            const int dz = z - zp;
            const R sz = dz < 0 ? R(-1) : R(1);
            const cpx<R> *gz = g + (dz < 0 ? -dz : dz) * 6;
            const cpx<R> gxx = gz[0], gyy = gz[1], gzz = gz[2];
            const cpx<R> gxy = sxy * gz[3], gxz = (sx * sz) * gz[4], gyz = (sy * sz) * gz[5];
            const cpx<R> u0 = us[zp * KB + j], u1 = us[(nz + zp) * KB + j], u2 = us[(2 * nz + zp) * KB + j];
            a0 = a0 + gxx * u0 + gxy * u1 + gxz * u2;
            a1 = a1 + gxy * u0 + gyy * u1 + gyz * u2;
            a2 = a2 + gxz * u0 + gyz * u1 + gzz * u2;
        }
    }
    __syncthreads();  // every thread is done with the staged y-spectra
    if (j < kb) {
        us[z * KB + j] = a0;
        us[(nz + z) * KB + j] = a1;
        us[(2 * nz + z) * KB + j] = a2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * KB; e += blockDim.x) {
        const int r = e / KB, jj = e - r * KB;
        if (jj < kb) o[(long long)r * Py + jj] = us[e];
    }
}

// (c) inverse y-FFT of `lg` coupled rows per workgroup, cropped back into the x-spectra.
template <class R>
__global__ void k_ysplit_inv(cpx<R> *work, const cpx<R> *yc, int ny, int nz, int Px, int lg, FftPlan py,
                             int xsplit) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem), *b = a + lg * py.L;
    const int Py = py.L, rows = 3 * nz, ngr = (rows + lg - 1) / lg;
    const int g = blockIdx.x % ngr;
    const int kx = xcd_block(blockIdx.x / ngr, Px);
    if (kx >= Px) return;
    const long long rhs = blockIdx.y;
    const int r0 = g * lg, nr = min(lg, rows - r0);
    const cpx<R> *src = yc + ((rhs * Px + kx) * rows + r0) * (long long)Py;
    for (int i = threadIdx.x; i < lg * Py; i += blockDim.x) a[i] = i < nr * Py ? src[i] : czero<R>();
    __syncthreads();
    const LdsLines ln = {lg, Py, 0, 1, lg};
    cpx<R> *res = Py > 1 ? fft_lds<R>(a, b, ln, py, true) : a;
    cpx<R> *base = work + rhs * 3LL * ny * nz * Px + xpos(kx, Px, xsplit);
    for (int i = threadIdx.x; i < nr * ny; i += blockDim.x) {
        const int l = i / ny, y = i - l * ny;
        base[((long long)(r0 + l) * ny + y) * Px] = res[l * Py + y];
    }
}

// pass 3: one workgroup per x-line; inverse FFT, crop, y = x - M (x + K x).
template <class R, int BPT>
__global__ void k_xinv(const cpx<R> *work, const cpx<R> *x, const cpx<R> *M, cpx<R> *y, int nx,
                       long long lines_per_comp_rhs_N, int nyz, FftPlan plan) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    long long line = blockIdx.x;
    const cpx<R> *src = work + line * plan.L;
    for (int i = threadIdx.x; i < plan.L; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, plan, true);
    long long yz = line % nyz;  // voxel row (z, y)
    const cpx<R> *xl = x + line * nx;
    const cpx<R> *ml = M + yz * nx;
    cpx<R> *yl = y + line * nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        cpx<R> xv = xl[i];
        yl[i] = xv - ml[i] * (xv + res[i]);
    }
    (void)lines_per_comp_rhs_N;
}

// One launch of the register-FFT plane pass: rb right-hand sides per workgroup, PL planes at a time.
template <class R, int PY, int P1, int P2, int NZ, int PL, bool TAIL>
static void plane_reg_launch_pl(vie_op op, cpx<R> *work, const cpx<R> *khat, int nrhs, int rb, const int *yzf,
                                int zero_in, hipStream_t s) {
    constexpr int L = 3 * NZ, PM = P1 > P2 ? P1 : P2;
    constexpr int NT = PL * PlaneThreads<PY, P1, P2, NZ, TAIL>::value, SP = PY + PM;
    const size_t lds = sizeof(cpx<R>) * ((size_t)PL * L * SP + (size_t)NZ * 6 * op->Hy + PY);
    const unsigned gy = (unsigned)((nrhs + rb - 1) / rb);
    vie_lds_attr((const void *)k_plane_reg<R, PY, P1, P2, NZ, PL, TAIL>, lds);
    hipLaunchKernelGGL((k_plane_reg<R, PY, P1, P2, NZ, PL, TAIL>), dim3(8 * ((op->Px + 7) / 8), gy), dim3(NT), lds, s,
                       work, khat, TwTable<R>::get(op->py), op->ny, op->Px, nrhs, rb, op->xsplit, yzf, zero_in);
}

// The register-FFT plane pass for the (y period, layer count) pairs it is instantiated for;
// false for any other shape (the generic LDS plane pass runs then).  Right-hand sides are grouped
// so that about 8192 workgroups remain (c.f. 256 CUs), each group sharing one staging of the
// x-frequency's transformed generator; groups of two or more run two planes side by side (single
// precision, or double where the pair's wavefronts fit the register file without spilling).
template <class R, int PY, int P1, int P2, int NZ>
static void plane_reg_launch(vie_op op, cpx<R> *work, const cpx<R> *khat, int nrhs, int rb_req, const int *yzf,
                             int zero_in, hipStream_t s) {
    const long long planes = (long long)op->Px * nrhs;
    const int rb = rb_req > 0 ? std::min(rb_req, nrhs)
                              : (int)std::max<long long>(1, std::min<long long>(nrhs, planes / 8192));
    // more than four wavefronts of items per plane: the four-wavefront form with split tails;
    // otherwise two planes side by side where their wavefronts still fit the register file
    constexpr int NTP = PlaneThreads<PY, P1, P2, NZ, false>::value;
    if constexpr (NTP > 256) {
        plane_reg_launch_pl<R, PY, P1, P2, NZ, 1, true>(op, work, khat, nrhs, rb, yzf, zero_in, s);
    } else {
        constexpr bool kPair = sizeof(R) == 4 || 2 * NTP <= 512;
        if constexpr (kPair) {
            if (rb >= 2) {
                plane_reg_launch_pl<R, PY, P1, P2, NZ, 2, false>(op, work, khat, nrhs, rb, yzf, zero_in, s);
                return;
            }
        }
        plane_reg_launch_pl<R, PY, P1, P2, NZ, 1, false>(op, work, khat, nrhs, rb, yzf, zero_in, s);
    }
}

// rb > 0: right-hand sides per workgroup (autotuned), 0: the default grouping.  work = nullptr
// only asks whether the shape is instantiated.  yzf: store only the lines with contrast (and with
// zero_in load only those, the others being zero).
template <class R>
static bool plane_reg(vie_op op, cpx<R> *work, const cpx<R> *khat, int nrhs, int rb, hipStream_t s,
                      const int *yzf = nullptr, int zero_in = 0) {
    const int Py = op->Py, nz = op->nz;
    if (!op->direct_z || op->split_plane) return false;
    if ((long long)3 * nz * op->ny * op->Px >= (1LL << 31)) return false;  // 32-bit offsets in a slab
#define VIE_PLANE_REG(PY, P1, P2, NZ)                                              \
    if (Py == PY && nz == NZ) {                                                    \
        if (work) plane_reg_launch<R, PY, P1, P2, NZ>(op, work, khat, nrhs, rb, yzf, zero_in, s); \
        return true;                                                               \
    }
    VIE_PLANE_REG(96, 12, 8, 8)
    VIE_PLANE_REG(64, 8, 8, 8)
    VIE_PLANE_REG(48, 8, 6, 8)
    VIE_PLANE_REG(32, 8, 4, 8)
    VIE_PLANE_REG(15, 5, 3, 8)
    VIE_PLANE_REG(32, 8, 4, 4)
    VIE_PLANE_REG(15, 5, 3, 4)
#undef VIE_PLANE_REG
    return false;
}

// The register x-line transform for the x periods it is instantiated for (false otherwise:
// the LDS Stockham kernels run).  mode 0: forward pass, 1: inverse pass with the final
// combination.
template <class R, int R1, int R2, int R3, int R4>
static void xline_launch(int mode, long long lines, const cpx<R> *in, cpx<R> *out, const cpx<R> *x, const cpx<R> *M,
                         int nx, int nyz, const cpx<R> *tw, const int *lmap, int nmap, hipStream_t s) {
    typedef rfft::Radices<R1, R2, R3, R4> RD;
    const size_t lds = sizeof(cpx<R>) * RD::L;
    const unsigned g = (unsigned)(lmap ? lines / (3LL * nyz) * nmap : lines);
    if (g == 0) return;
    if (mode == 0) {
        vie_lds_attr((const void *)k_xline_reg<R, R1, R2, R3, R4, 0>, lds);
        hipLaunchKernelGGL((k_xline_reg<R, R1, R2, R3, R4, 0>), dim3(g), dim3(RD::T), lds, s, in, out, x, M, nx, nyz,
                           tw, lmap, nmap);
    } else {
        vie_lds_attr((const void *)k_xline_reg<R, R1, R2, R3, R4, 1>, lds);
        hipLaunchKernelGGL((k_xline_reg<R, R1, R2, R3, R4, 1>), dim3(g), dim3(RD::T), lds, s, in, out, x, M, nx, nyz,
                           tw, lmap, nmap);
    }
}

// mode -1 only asks whether the length is instantiated.  lmap (nmap lines of each right-hand
// side's 3 ny nz): transform only those lines.
template <class R>
static bool xline_reg(vie_op op, int mode, long long lines, const cpx<R> *in, cpx<R> *out, const cpx<R> *x,
                      const cpx<R> *M, hipStream_t s, const int *lmap = nullptr, int nmap = 0) {
    if (op->xsplit > 1) return false;
    if (mode < 0) return op->Px == 1024 || op->Px == 2048 || op->Px == 4096 || op->Px == 8192 ||
                         (op->Px == 16384 && sizeof(R) == 4);
    const cpx<R> *tw = TwTable<R>::get(op->px);
    const int nyz = op->ny * op->nz;
    switch (op->Px) {
        case 1024: xline_launch<R, 16, 8, 8, 1>(mode, lines, in, out, x, M, op->nx, nyz, tw, lmap, nmap, s); return true;
        case 2048: xline_launch<R, 16, 16, 8, 1>(mode, lines, in, out, x, M, op->nx, nyz, tw, lmap, nmap, s); return true;
        case 4096: xline_launch<R, 16, 16, 16, 1>(mode, lines, in, out, x, M, op->nx, nyz, tw, lmap, nmap, s); return true;
        case 8192: xline_launch<R, 16, 16, 16, 2>(mode, lines, in, out, x, M, op->nx, nyz, tw, lmap, nmap, s); return true;
        case 16384:  // complex64 only (a complex128 line of this length takes the four-step path)
            if constexpr (sizeof(R) == 4) {
                xline_launch<R, 16, 16, 16, 4>(mode, lines, in, out, x, M, op->nx, nyz, tw, lmap, nmap, s);
                return true;
            }
            return false;
        default: return false;
    }
}

// Device bytes a product of nrhs vectors of element size esz works in: the x-spectra of every
// line (*work) and, for the split plane pass, the y-spectra before and after the coupling (*ysp).
static void matvec_scratch(const vie_op op, int nrhs, size_t esz, size_t *work, size_t *ysp) {
    *work = esz * 3 * (size_t)op->ny * op->nz * nrhs * op->Px;
    *ysp = op->split_plane ? 2 * esz * (size_t)nrhs * op->Px * 3 * op->nz * op->Py : 0;
}

// One product through the three passes; work and ysp hold matvec_scratch's bytes.
// cfg_plane: right-hand sides per workgroup of the register plane pass, or the threads of the
// LDS plane pass; cfg_x: threads of the LDS x-line passes (0 = defaults).
// Lines whose contrast vanishes along all of x (op->lines, when the register x-line and plane
// passes serve the shape): their product is y = x, so the inverse pass transforms only the other
// lines and copies x on these, and the plane pass does not store them.  zero_in (x zero on them,
// y not needed there): the forward pass and the plane pass skip them too and y is left as it is.
template <class R>
static vie_status matvec_run(vie_op op, const cpx<R> *x, cpx<R> *y, int nrhs, const cpx<R> *khat,
                             const cpx<R> *M, cpx<R> *work, cpx<R> *ysp, int cfg_plane, int cfg_x, hipStream_t s,
                             bool zero_in = false) {
    const int nx = op->nx, ny = op->ny, nz = op->nz, Px = op->Px;
    long long lines = 3LL * ny * nz * nrhs;
    size_t ldsx;
    int thx, bpt;
    fft_line_shape(op->px, sizeof(cpx<R>), &thx, &ldsx, &bpt, cfg_x);
    const int thp = cfg_plane ? cfg_plane : 256;
    const bool lskip = op->n_line_zero > 0 && op->direct_z && !op->split_plane &&
                       xline_reg<R>(op, -1, 0, nullptr, nullptr, nullptr, nullptr, s) &&
                       plane_reg<R>(op, nullptr, khat, nrhs, 0, s);
    const int *lact = lskip ? op->lines.as<const int>() : nullptr;
    const int *yzf = lskip ? op->yzflag.as<const int>() : nullptr;
    const int zin = lskip && zero_in ? 1 : 0;
    {
        ProfScope ps("matvec_xfwd", s);
        if (op->xsplit > 1) {
            VIE_CHECK(long_lines<R>(op, x, nx, work, lines, false, s));
        } else if (!xline_reg<R>(op, 0, lines, x, work, nullptr, nullptr, s, zin ? lact : nullptr, op->n_line_act)) {
#define LAUNCH_XFWD(B)                                      \
    vie_lds_attr((const void *)k_xfwd<R, B>, ldsx);         \
    hipLaunchKernelGGL((k_xfwd<R, B>), dim3((unsigned)lines), dim3(thx), ldsx, s, x, work, nx, op->px)
            VIE_BPT_SWITCH(bpt, LAUNCH_XFWD);
#undef LAUNCH_XFWD
        }
    }
    VIE_HIP(hipGetLastError());
    if (op->split_plane) {
        const int Py = op->Py, rows = 3 * nz;
        int lg = (int)std::min<size_t>(8, max_lds() / (2 * sizeof(cpx<R>) * Py));
        lg = std::max(1, std::min(lg, rows));
        const size_t ldsy = 2 * sizeof(cpx<R>) * lg * Py;
        cpx<R> *y1 = ysp, *y2 = y1 + (size_t)nrhs * Px * rows * Py;
        const unsigned gx = (unsigned)(8 * ((Px + 7) / 8) * ((rows + lg - 1) / lg));
        ProfScope ps("matvec_plane", s);
        vie_lds_attr((const void *)k_ysplit_fwd<R>, ldsy);
        hipLaunchKernelGGL(k_ysplit_fwd<R>, dim3(gx, nrhs), dim3(256), ldsy, s, (const cpx<R> *)work, y1, ny, nz, Px,
                           lg, op->py, op->xsplit);
        const int kb = 256 / nz;
        const size_t ldsc = sizeof(cpx<R>) * ((size_t)3 * nz * kb + (size_t)kb * (6 * nz + 1));
        vie_lds_attr((const void *)k_ysplit_couple<R>, ldsc);
        hipLaunchKernelGGL(k_ysplit_couple<R>, dim3((unsigned)(Px * ((Py + kb - 1) / kb)), nrhs), dim3(256), ldsc, s,
                           (const cpx<R> *)y1, y2, khat, nz, Px, Py, op->Hy);
        vie_lds_attr((const void *)k_ysplit_inv<R>, ldsy);
        hipLaunchKernelGGL(k_ysplit_inv<R>, dim3(gx, nrhs), dim3(256), ldsy, s, work, (const cpx<R> *)y2, ny, nz, Px,
                           lg, op->py, op->xsplit);
    } else if (op->direct_z) {
        ProfScope ps("matvec_plane", s);
        if (!plane_reg<R>(op, work, khat, nrhs, cfg_plane, s, yzf, zin)) {
            size_t ldsp = sizeof(cpx<R>) * ((size_t)6 * nz * op->Py + (size_t)6 * op->Hy * nz);
            vie_lds_attr((const void *)k_plane_dz<R>, ldsp);
            hipLaunchKernelGGL(k_plane_dz<R>, dim3(8 * ((Px + 7) / 8), nrhs), dim3(thp), ldsp, s, work, khat, ny, nz,
                               Px, op->Hy, op->py, op->xsplit);
        }
    } else {
        size_t ldsp = 6 * sizeof(cpx<R>) * op->Py * op->Pz;
        vie_lds_attr((const void *)k_plane<R>, ldsp);
        ProfScope ps("matvec_plane", s);
        hipLaunchKernelGGL(k_plane<R>, dim3(8 * ((Px + 7) / 8), nrhs), dim3(thp), ldsp, s, work, khat, ny, nz, Px,
                           op->Hx, op->Hy, op->Hz, op->py, op->pz, op->xsplit);
    }
    VIE_HIP(hipGetLastError());
    if (op->xsplit > 1) {
        ProfScope ps("matvec_xinv", s);
        VIE_CHECK(long_lines<R>(op, work, Px, work, lines, true, s));
        const int ntile = op->px1.L / LONG_LT;
        size_t lds;
        int cthr, cb;
        long_cols_shape(op->px2, sizeof(cpx<R>), &cthr, &lds, &cb);
#define LAUNCH_COLS_INV(B)                                                                                         \
    vie_lds_attr((const void *)k_long_cols_inv<R, B>, lds);                                                        \
    hipLaunchKernelGGL((k_long_cols_inv<R, B>), dim3((unsigned)(lines * ntile)), dim3(cthr), lds, s, work, Px,      \
                       op->px1.L, op->px2, TwTable<R>::get(op->px), x, M, y, nx, ny * nz)
        if (cb) {
            LAUNCH_COLS_INV(4);
        } else {
            LAUNCH_COLS_INV(0);
        }
#undef LAUNCH_COLS_INV
    } else {
        ProfScope ps("matvec_xinv", s);
        if (lskip) {
            xline_reg<R>(op, 1, lines, work, y, x, M, s, lact, op->n_line_act);
            if (!zin) {
                const long long per = (long long)op->n_line_zero * nx;
                hipLaunchKernelGGL(k_copy_lines<R>, dim3((unsigned)std::min<long long>(1024, (per + 255) / 256), nrhs),
                                   dim3(256), 0, s, x, y, op->lines.as<const int>() + op->n_line_act, op->n_line_zero,
                                   nx, ny * nz);
            }
        } else if (!xline_reg<R>(op, 1, lines, work, y, x, M, s)) {
#define LAUNCH_XINV(B)                                                                               \
    vie_lds_attr((const void *)k_xinv<R, B>, ldsx);                                                  \
    hipLaunchKernelGGL((k_xinv<R, B>), dim3((unsigned)lines), dim3(thx), ldsx, s, work, x, M, y, nx, \
                       0LL, ny * nz, op->px)
            VIE_BPT_SWITCH(bpt, LAUNCH_XINV);
#undef LAUNCH_XINV
        }
    }
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// FFT launch parameters for `nrhs` right-hand sides: defaults, or with autotuning on the
// fastest (plane-pass threads x x-line threads) for this shape, cached per process.
template <class R>
static vie_status matvec_t(vie_op op, const cpx<R> *x, cpx<R> *y, int nrhs, const cpx<R> *khat,
                           const cpx<R> *M, hipStream_t s, bool zero_in) {
    const int pi = sizeof(R) == 8 ? 0 : 1;
    OpWs *w = op->ws.get(s);
    std::lock_guard<std::mutex> lk(w->mu);
    size_t wb, yb;
    matvec_scratch(op, nrhs, sizeof(cpx<R>), &wb, &yb);
    VIE_CHECK(w->work.ensure(wb));
    if (yb) VIE_CHECK(w->ybuf.ensure(yb));
    cpx<R> *work = w->work.as<cpx<R>>(), *ysp = w->ybuf.as<cpx<R>>();
    if (tune_enabled() && w->tuned_nrhs[pi] != nrhs) {
        char key[160];
        snprintf(key, sizeof key, "matvec esz=%d P=%dx%dx%d grid=%dx%dx%d nrhs=%d direct_z=%d split=%d",
                 (int)sizeof(cpx<R>), op->Px, op->Py, op->Pz, op->nx, op->ny, op->nz, nrhs, (int)op->direct_z,
                 (int)op->split_plane);
        int t0, b0;
        size_t l0;
        fft_line_shape(op->px, sizeof(cpx<R>), &t0, &l0, &b0);
        std::vector<std::vector<int>> cands;
        {
            // plane pass: right-hand sides per workgroup (register pass) or threads (LDS pass);
            // x passes: threads of the LDS kernels (the register and four-step kernels have none)
            std::vector<int> pcand, xcand;
            if (plane_reg<R>(op, nullptr, khat, nrhs, 0, s)) {
                pcand.push_back(0);
                for (int rb = 1; rb <= nrhs && rb <= 64; rb *= 2) pcand.push_back(rb);
            } else {
                pcand = {128, 256, 512};
            }
            const bool xfixed = op->xsplit > 1 || xline_reg<R>(op, -1, 0, nullptr, nullptr, nullptr, nullptr, s);
            if (xfixed) {
                xcand.push_back(0);
            } else {
                for (int tx : {t0 / 2, t0, 2 * t0}) {
                    int t, b;
                    size_t l;
                    if (tx < 64 || tx > 1024 || !fft_line_shape(op->px, sizeof(cpx<R>), &t, &l, &b, tx)) continue;
                    xcand.push_back(tx);
                }
            }
            for (int tp : pcand)
                for (int tx : xcand) cands.push_back({tp, tx});
        }
        std::vector<int> choice;
        if (tune_lookup(key, &choice)) {
            VIE_CHECK(tune_check_choice(key, choice, cands));
        } else {
            double best = 1e300;
            for (auto &c : cands) {
                double ms = 0;
                VIE_CHECK(tune_time(s, 2, [&]() {
                    return matvec_run<R>(op, x, y, nrhs, khat, M, work, ysp, c[0], c[1], s);
                }, &ms));
                if (ms < best) {
                    best = ms;
                    choice = c;
                }
            }
            tune_store(key, choice, best, (int)cands.size());
        }
        w->cfg_plane_thr[pi] = choice[0], w->cfg_x_thr[pi] = choice[1];
        w->tuned_nrhs[pi] = nrhs;
    }
    return matvec_run<R>(op, x, y, nrhs, khat, M, work, ysp, w->cfg_plane_thr[pi], w->cfg_x_thr[pi], s, zero_in);
}

vie_status launch_matvec(vie_op op, const void *x, void *y, int nrhs, int prec, hipStream_t s, bool zero_skipped_in) {
    if (prec == VIE_C128)
        return matvec_t<double>(op, (const c128 *)x, (c128 *)y, nrhs, op->khat64.as<c128>(),
                                op->M64.as<c128>(), s, zero_skipped_in);
    return matvec_t<float>(op, (const c64 *)x, (c64 *)y, nrhs, op->khat32.as<c64>(), op->M32.as<c64>(), s,
                           zero_skipped_in);
}

// ---------------------------------------------------------------- allocation-free product
// The product's scratch (x-spectra, split-pass y-spectra) in a fixed device array instead of
// the handle's buffers.  Each device holds its own copy of the array; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[VIE_MATVEC_NOALLOC_MAX_BYTES];

#define VIE_NOALLOC_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_dev[VIE_NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
static vie_status scratch_address(void **out) {
    int dev = 0;
    VIE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= VIE_NOALLOC_MAX_DEVICES) {
        vie_set_error("vie_matvec_noalloc: device index beyond the library's table");
        return VIE_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        VIE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            vie_set_error("vie_matvec_noalloc: no device address for the scratch array");
            return VIE_EDEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return VIE_OK;
}

extern "C" vie_status vie_matvec_noalloc(vie_op op, const void *x, void *y, int32_t nrhs, vie_prec prec,
                                         void *stream) {
    NoAllocScope na;  // no profiling events either
    VIE_CHECK(matvec_check_args("vie_matvec_noalloc", op, x, y, nrhs, prec));
    const size_t esz = prec == VIE_C128 ? sizeof(c128) : sizeof(c64);
    size_t wb, yb;
    matvec_scratch(op, nrhs, esz, &wb, &yb);
    const size_t wpad = (wb + 255) & ~(size_t)255;
    if (wpad + yb > (size_t)VIE_MATVEC_NOALLOC_MAX_BYTES) {
        vie_set_error("vie_matvec_noalloc: this product needs " + std::to_string(wpad + yb) +
                      " scratch bytes, more than the fixed " + std::to_string((size_t)VIE_MATVEC_NOALLOC_MAX_BYTES) +
                      " (use vie_matvec, or fewer right-hand sides per call)");
        return VIE_EARG;
    }
    void *base = nullptr;
    VIE_CHECK(scratch_address(&base));
    unsigned char *p = static_cast<unsigned char *>(base);
    hipStream_t s = (hipStream_t)stream;
    if (prec == VIE_C128)
        return matvec_run<double>(op, (const c128 *)x, (c128 *)y, nrhs, op->khat64.as<c128>(), op->M64.as<c128>(),
                                  reinterpret_cast<c128 *>(p), reinterpret_cast<c128 *>(p + wpad), 0, 0, s);
    return matvec_run<float>(op, (const c64 *)x, (c64 *)y, nrhs, op->khat32.as<c64>(), op->M32.as<c64>(),
                             reinterpret_cast<c64 *>(p), reinterpret_cast<c64 *>(p + wpad), 0, 0, s);
}
