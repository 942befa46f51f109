// Block solves of the preconditioner apply: for every Fourier mode k of every box,
//   z_k = U^{-1} L^{-1} P rhat_k
// with the LU factors of D_k (the block-diagonal form of the one-level circulant, Sec. 4,
// eq. Di and its inverse).  The packed factors are column-major [m][m] per stored block, every
// 64x64 diagonal tile replaced by the inverses of its unit-lower part (strictly lower entries)
// and of its upper part (upper entries incl. the diagonal), so each diagonal tile is applied
// as a product.  work element (rhs, box, row i, mode k) sits at ((rhs*nboxes + box)*m + i)*n + k.
//
// A column of a stored block is one (mode, right-hand side) pair whose mode uses the block: the
// R right-hand sides of its own mode, of the reflected mode (n - k along x, and by - ky for the
// 2-level blocks: solved as S D^{-1} S, signs on the x / y rows) and, under the memory
// reduction, of every mode that shares the central block.  Three kernels share the columns:
//  * narrow: one workgroup per (stored block, chunk of <= 8 columns), rows in registers; for
//    blocks used by few columns;
//  * tiny (m <= 64): one wavefront per (stored block, 64/m columns);
//  * wide: one workgroup per (stored block, group of <= 64 columns), the products on the
//    matrix cores.
#include <algorithm>
#include <cstdio>

#include "fft_device.h"
#include "vie_internal.h"

#define TS 64

// Sign of block row `row` in a reflected mode (flags of VIE_MODE_MIRROR, mx rows per component):
// true where S = -1.
__device__ __forceinline__ bool mirror_flip(int flags, int row, int mx) {
    return ((flags & VIE_MODE_MIRROR_X) && row < mx) != ((flags & VIE_MODE_MIRROR_Y) && row >= mx && row < 2 * mx);
}

// ---------------------------------------------------------------- narrow
// Thread t owns rows t, t + 256, ... (QR of them) and keeps their RC accumulators in
// registers.  Forward and backward substitution run over 64-row tiles: the tile's owners
// publish its rows to LDS, four wavefronts apply the pre-inverted diagonal tile (each a
// quarter of its columns), and every thread then applies the tile's column panel to its
// remaining rows.  Each factor entry is read once per chunk and used RC times; the factor
// reads are coalesced along columns.
// Work item = (stored block s, first column c0, column count, box), column g of block s being the
// pair (mode mode_list[mode_ptr[s] + g / nrhs], right-hand side g % nrhs): the two modes k and
// n - k of a reflected pair share a workgroup and each factor read.  A reflected column (flag
// VIE_MODE_MIRROR) is solved as S D_k^{-1} S: its x-component rows (the first mx block rows)
// (and, for a reflected y-mode, its y-component rows) change sign on the way in and out.
template <class R, int QR, int RC, class FT>
__global__ void __launch_bounds__(256) k_block_solve(cpx<R> *work, const FT *F, const int *perm, const int4 *items,
                                                     const int *mode_ptr, const int *mode_list, int m, int n,
                                                     int nboxes, int nrhs, int mx) {
    cpx<R> *yt = reinterpret_cast<cpx<R> *>(vie_smem);  // [TS][RC]
    cpx<R> *part = yt + TS * RC;                        // [4][TS][RC]
    const int4 item = items[blockIdx.x];
    const int sblk = item.x, c0 = item.y, ncols = item.z, box = item.w;
    const FT *A = F + (long long)sblk * m * m;
    const int *pm = perm + (long long)sblk * m;
    const long long rstride = (long long)nboxes * m * n;
    long long off[RC];
    int fl[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) {
        off[c] = -1;
        fl[c] = 0;
        if (c < ncols) {
            const int g = c0 + c, me = mode_list[mode_ptr[sblk] + g / nrhs];
            off[c] = (long long)(g % nrhs) * rstride + (long long)box * m * n + (me & ~VIE_MODE_MIRROR);
            fl[c] = me & VIE_MODE_MIRROR;
        }
    }
    const int tid = threadIdx.x;
    cpx<R> acc[QR][RC];
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        int i = tid + 256 * q;
        const int src = i < m ? pm[i] : 0;
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            cpx<R> v = (i < m && off[c] >= 0) ? work[off[c] + (long long)src * n] : czero<R>();
            if (mirror_flip(fl[c], src, mx)) v = mk(-v.re, -v.im);
            acc[q][c] = v;
        }
    }
    const int g = tid >> 6, r = tid & 63;
    // forward: unit lower L (diagonal tiles hold the strictly lower part of their inverse)
    for (int t0 = 0; t0 < m; t0 += TS) {
        const int w = min(TS, m - t0);
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            int i = tid + 256 * q;
            if (i >= t0 && i < t0 + w)
#pragma unroll
                for (int c = 0; c < RC; ++c) yt[(i - t0) * RC + c] = acc[q][c];
        }
        __syncthreads();
        {
            cpx<R> p[RC];
#pragma unroll
            for (int c = 0; c < RC; ++c) p[c] = czero<R>();
            if (r < w)
                for (int cc = g; cc < r; cc += 4) {
                    cpx<R> l = ldf(A + (long long)(t0 + cc) * m + t0 + r);
#pragma unroll
                    for (int c = 0; c < RC; ++c) p[c] = p[c] + l * yt[cc * RC + c];
                }
#pragma unroll
            for (int c = 0; c < RC; ++c) part[(g * TS + r) * RC + c] = p[c];
        }
        __syncthreads();
        if (tid < w)
#pragma unroll
            for (int c = 0; c < RC; ++c)
                yt[tid * RC + c] = yt[tid * RC + c] + part[tid * RC + c] + part[(TS + tid) * RC + c] +
                                   part[(2 * TS + tid) * RC + c] + part[(3 * TS + tid) * RC + c];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            int i = tid + 256 * q;
            if (i >= t0 && i < t0 + w) {
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[q][c] = yt[(i - t0) * RC + c];
            } else if (i >= t0 + w && i < m) {
                const FT *col = A + (long long)t0 * m + i;
#pragma unroll 4
                for (int cc = 0; cc < w; ++cc) {
                    cpx<R> l = ldf(col + (long long)cc * m);
#pragma unroll
                    for (int c = 0; c < RC; ++c) acc[q][c] = cfms(acc[q][c], l, yt[cc * RC + c]);
                }
            }
        }
        __syncthreads();
    }
    // backward: upper U (diagonal tiles hold the upper part of their inverse)
    const int ntile = (m + TS - 1) / TS;
    for (int tt = ntile - 1; tt >= 0; --tt) {
        const int t0 = tt * TS;
        const int w = min(TS, m - t0);
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            int i = tid + 256 * q;
            if (i >= t0 && i < t0 + w)
#pragma unroll
                for (int c = 0; c < RC; ++c) yt[(i - t0) * RC + c] = acc[q][c];
        }
        __syncthreads();
        {
            cpx<R> p[RC];
#pragma unroll
            for (int c = 0; c < RC; ++c) p[c] = czero<R>();
            if (r < w)
                for (int cc = g; cc < w; cc += 4)
                    if (cc >= r) {
                        cpx<R> u = ldf(A + (long long)(t0 + cc) * m + t0 + r);
#pragma unroll
                        for (int c = 0; c < RC; ++c) p[c] = p[c] + u * yt[cc * RC + c];
                    }
#pragma unroll
            for (int c = 0; c < RC; ++c) part[(g * TS + r) * RC + c] = p[c];
        }
        __syncthreads();
        if (tid < w)
#pragma unroll
            for (int c = 0; c < RC; ++c)
                yt[tid * RC + c] = part[tid * RC + c] + part[(TS + tid) * RC + c] + part[(2 * TS + tid) * RC + c] +
                                   part[(3 * TS + tid) * RC + c];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            int i = tid + 256 * q;
            if (i >= t0 && i < t0 + w) {
#pragma unroll
                for (int c = 0; c < RC; ++c) acc[q][c] = yt[(i - t0) * RC + c];
            } else if (i < t0) {
                const FT *col = A + (long long)t0 * m + i;
#pragma unroll 4
                for (int cc = 0; cc < w; ++cc) {
                    cpx<R> u = ldf(col + (long long)cc * m);
#pragma unroll
                    for (int c = 0; c < RC; ++c) acc[q][c] = cfms(acc[q][c], u, yt[cc * RC + c]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        int i = tid + 256 * q;
        if (i < m)
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (off[c] >= 0) {
                    const cpx<R> v = acc[q][c];
                    work[off[c] + (long long)i * n] = mirror_flip(fl[c], i, mx) ? mk(-v.re, -v.im) : v;
                }
    }
}

// Blocks of one tile (m <= 64, e.g. the 3 nz blocks of the 2-level preconditioner): one
// wavefront per item of up to 64/m columns of one stored block (items as in the per-block solve),
// lane slot*m + i owning row i of column `slot`.  With the single diagonal tile holding
// strict(L^{-1}) below and U^{-1} on and above the diagonal,
//   y_i = (P r)_i + sum_{c < i} L^{-1}_{ic} (P r)_c,    x_i = sum_{c >= i} U^{-1}_{ic} y_c,
// each factor entry is read once per wavefront (columns coalesced across the lanes, the column
// slots reading the same addresses), the vectors go through the wavefront's LDS row.  The sums
// of the per-block kernel, accumulated in column order.
template <class R, class FT>
__global__ void __launch_bounds__(256) k_block_solve_tiny(cpx<R> *work, const FT *F, const int *perm,
                                                          const int4 *items, const int *mode_ptr,
                                                          const int *mode_list, int m, int n, int nboxes, int nrhs,
                                                          int nitems, int mx) {
    __shared__ cpx<R> vs[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int it = blockIdx.x * 4 + wv;
    if (it >= nitems) return;  // whole wavefront; no workgroup barrier below
    const int4 item = items[it];
    const int sblk = item.x, c0 = item.y, ncols = item.z, box = item.w;
    const int slot = lane / m, i = lane - slot * m;
    const bool row = slot < ncols;
    long long off = 0;
    int fl = 0;
    if (row) {
        const int g = c0 + slot, me = mode_list[mode_ptr[sblk] + g / nrhs];
        off = (long long)(g % nrhs) * nboxes * m * n + (long long)box * m * n + (me & ~VIE_MODE_MIRROR);
        fl = me & VIE_MODE_MIRROR;
    }
    const FT *A = F + (long long)sblk * m * m;
    const int *pm = perm + (long long)sblk * m;
    cpx<R> *v = vs[wv];
    const cpx<R> *vc = v + (row ? slot * m : 0);  // this column's vector
    const int src = row ? pm[i] : 0;
    cpx<R> r0 = row ? work[off + (long long)src * n] : czero<R>();
    if (mirror_flip(fl, src, mx)) r0 = mk(-r0.re, -r0.im);
    v[lane] = r0;
    __builtin_amdgcn_wave_barrier();
    cpx<R> y = r0;
    for (int c = 0; c < m; ++c)
        if (c < i && row) y = y + ldf(A + (long long)c * m + i) * vc[c];
    __builtin_amdgcn_wave_barrier();
    v[lane] = y;
    __builtin_amdgcn_wave_barrier();
    cpx<R> x = czero<R>();
    for (int c = 0; c < m; ++c)
        if (c >= i && row) x = x + ldf(A + (long long)c * m + i) * vc[c];
    if (row) work[off + (long long)i * n] = mirror_flip(fl, i, mx) ? mk(-x.re, -x.im) : x;
}

#define VIE_MAX_QR 5
// Columns per chunk: a power of two <= 8, at most the columns of a block (`cols`: right-hand
// sides times the modes sharing it), bounded by the register budget of the accumulators.
static int block_solve_rc(int m, int cols, size_t esz) {
    int qr = (m + 255) / 256;
    int budget = esz == sizeof(c128) ? 24 : 48;  // complex accumulators per thread
    int rc = 1;
    while (rc < 8 && rc < cols && qr * rc * 2 <= budget) rc *= 2;
    return rc;
}

// Most columns one stored block has for `nrhs` right-hand sides.
static int block_cols_max(vie_pc pc, int nrhs) {
    int c = 1;
    for (int sb = 0; sb < pc->nstored; ++sb) c = std::max(c, (pc->mode_ptr[sb + 1] - pc->mode_ptr[sb]) * nrhs);
    return c;
}

struct NarrowArgs {
    const int4 *items;
    const int *mode_ptr, *mode_list;
    int m, n, nboxes, nrhs, mx;
};

template <class R, int QR, int RC, class FT>
static void launch_bs(dim3 grid, size_t lds, hipStream_t s, cpx<R> *work, const FT *F, const int *perm,
                      const NarrowArgs &a) {
    hipLaunchKernelGGL((k_block_solve<R, QR, RC, FT>), grid, dim3(256), lds, s, work, F, perm, a.items, a.mode_ptr,
                       a.mode_list, a.m, a.n, a.nboxes, a.nrhs, a.mx);
}

template <class R, int QR, class FT>
static void launch_bs_rc(int rc, dim3 grid, size_t lds, hipStream_t s, cpx<R> *work, const FT *F,
                         const int *perm, const NarrowArgs &a) {
    switch (rc) {
        case 1: launch_bs<R, QR, 1>(grid, lds, s, work, F, perm, a); break;
        case 2: launch_bs<R, QR, 2>(grid, lds, s, work, F, perm, a); break;
        case 4: launch_bs<R, QR, 4>(grid, lds, s, work, F, perm, a); break;
        default: launch_bs<R, QR, 8>(grid, lds, s, work, F, perm, a); break;
    }
}

// ---------------------------------------------------------------- wide
// Complex products on the real 16x16x4 matrix-core instruction (FP32 or FP64).  A K-step
// takes two complex columns c0, c0+1 of the left operand as four real ones: lane l supplies
// row l%16 and real index q = l/16 (complex column c0 + q/2, part q%2).  With the right operand
// fed as (Re b, Im b) interleaved, the real left operand (Re a, -Im a) accumulates Re(a b) and
// (Im a, Re a) accumulates Im(a b).  The accumulator of a 16x16 tile holds, in lane l,
// register v, the entry (row acc_row(l/16, v), column l%16): row 4*(l/16) + v for FP32 and
// row 4*v + l/16 for FP64 (measured on gfx950; the operand layouts agree).
template <class R>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 fma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int acc_row(int q, int v) { return 4 * q + v; }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 fma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int acc_row(int q, int v) { return 4 * v + q; }
};

// The matrix-core products below keep one batch of K-steps in flight while the previous one
// is multiplied: loads are issued unconditionally from addresses clamped into the buffers
// (masks are applied to the loaded values), and two register sets alternate, so the waits
// only cover the older batch.

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// ---- shared right operand: the off-diagonal products of one super-tile multiply every
// wavefront's own factor rows with the same solved rows Y[kb:ke], so those rows go through LDS
// once per workgroup, in chunks, double-buffered: the next chunk's rows and factor entries are
// loaded while the current chunk is multiplied, one barrier per chunk.  Every wavefront of the
// workgroup must call these (active = false: it only helps stage).  Chunks run in rotated order
// (rot): the workgroups of one stored block take the same rotation and, dispatched together on
// one XCD, read each factor chunk at about the same time (the later reads hit L2), while
// different blocks start at different chunks.

// FP32 / FP64 solved rows, row-major [m][CT*16] complex; YC rows per chunk.  The complex
// product takes three real matrix-core products per K-step of four complex rows (Gauss):
// with a = L[row][k] and y = Y[k][col], P1 = Re a Re y, P2 = Im a Im y and
// P3 = (Re a + Im a)(Re y + Im y) give Re(a y) = P1 - P2 and Im(a y) = P3 - P1 - P2, so the
// accumulators are g1 = Re acc - sum P1, g2 = sum P2 and g3 = Re acc + Im acc - sum P3, folded
// back at the end.  Lane (r, q) of the 16x16x4 instruction supplies factor row r and solved
// column r of complex row k0 + q (four distinct complex rows per instruction, where the
// (Re, Im)-interleaved form needs two instructions for two rows).
template <class R, int CT, int NTH, class FT>
__device__ __forceinline__ void wide_gemm_chunked(typename Mfma<R>::v4 *cr, typename Mfma<R>::v4 *ci, bool active,
                                                  const FT *arow, const FT *abase, long long m, bool rv,
                                                  const cpx<R> *Y, int kb, int ke, int rot, cpx<R> *buf) {
    typedef typename Mfma<R>::v4 v4;
    constexpr int WC = CT * 16;
    constexpr int YC = 16;                            // rows per chunk (FP64: the two slots and two tiles fill 160 KB)
    constexpr int SPT = (YC * WC + NTH - 1) / NTH;    // staged complex per thread
    constexpr int KS = YC / 4;                        // K-steps per chunk
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const FT *ap = rv ? arow + r : abase;
    const int nch = (ke - kb + YC - 1) / YC;
    rot = rot % nch;
    cpx<R> st[SPT], a0[KS], a1[KS];
    v4 g2[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        g2[ct] = v4{0, 0, 0, 0};
        ci[ct] += cr[ct];  // g3; cr is g1
    }
    auto row0 = [&](int c) { int cc = c + rot; if (cc >= nch) cc -= nch; return kb + YC * cc; };
    auto load = [&](int c, cpx<R> *a) {
        const int k0 = row0(c);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = threadIdx.x + u * NTH, row = k0 + e / WC;
            st[u] = (e < YC * WC && row < ke) ? Y[(long long)row * WC + e % WC] : czero<R>();
        }
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int kc = k0 + 4 * u + q;
            a[u] = ldf(ap + (long long)(kc < ke ? kc : kb) * m);  // past ke: multiplied by zero rows
        }
    };
    auto stage = [&](int slot) {
        cpx<R> *b = buf + slot * YC * WC;
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = threadIdx.x + u * NTH;
            if (e < YC * WC) b[e] = st[u];
        }
    };
    auto compute = [&](int slot, const cpx<R> *a) {
        const cpx<R> *ys = buf + slot * YC * WC + r;
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const R n1 = -a[u].re, p2 = a[u].im, n3 = -(a[u].re + a[u].im);
            const cpx<R> *yr = ys + (4 * u + q) * WC;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const cpx<R> y = yr[ct * 16];
                cr[ct] = Mfma<R>::fma(n1, y.re, cr[ct]);
                g2[ct] = Mfma<R>::fma(p2, y.im, g2[ct]);
                ci[ct] = Mfma<R>::fma(n3, y.re + y.im, ci[ct]);
            }
        }
    };
    load(0, a0);
    stage(0);
    for (int c = 0; c < nch; c += 2) {
        if (c + 1 < nch) load(c + 1, a1);
        __syncthreads();
        if (active) compute(0, a0);
        if (c + 1 >= nch) break;
        stage(1);
        if (c + 2 < nch) load(c + 2, a0);
        __syncthreads();
        if (active) compute(1, a1);
        if (c + 2 < nch) stage(0);
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        ci[ct] = ci[ct] - cr[ct] + g2[ct];
        cr[ct] += g2[ct];
    }
}

// bfloat16 factors: solved rows split into bfloat16 hi + lo, [col][mp] per item (rows past m
// zero); a K-step is 16 complex rows on v_mfma_f32_16x16x32_bf16, whose lane l supplies row
// l%16 and reals 8 (l/16) .. +7: the four complex entries 4 (l/16) .. +3 as (re, im) pairs,
// i.e. exactly four packed factor words.  -(Re a, -Im a) is the word with the low sign bit
// flipped, -(Im a, Re a) the word with its halves swapped and both sign bits flipped.  The
// accumulator layout is that of the FP32 16x16x4 instruction.  A chunk is BF_KSTEPS K-steps:
// the products of one K-step are too short to cover the latency of the next chunk's loads, so
// a chunk carries several.  kb is a multiple of 16; rows from ke on are staged as zeros (in the
// forward pass the rows past ke are not solved yet), and rows m..mp-1 of Y are zero.
#define BF_KSTEPS 2
template <int CT, int NTH>
__device__ __forceinline__ void wide_gemm_chunked_bf16(Mfma<float>::v4 *cr, Mfma<float>::v4 *ci, bool active,
                                                       const bf16c *arow, const bf16c *abase, long long m, bool rv,
                                                       const uint32_t *Yh, const uint32_t *Yl, int mp, int kb, int ke,
                                                       int rot, uint32_t *buf) {
    constexpr int WC = CT * 16;
    constexpr int KB = BF_KSTEPS;
    constexpr int NV1 = 2 * WC * 4;                  // uint4 loads per K-step (hi and lo, 4 per column)
    constexpr int NV = NV1 * KB;
    constexpr int SPT = (NV + NTH - 1) / NTH;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const uint32_t *ap = reinterpret_cast<const uint32_t *>(rv ? arow + r : abase);
    const int nch = (ke - kb + 16 * KB - 1) / (16 * KB);
    rot = rot % nch;
    u4v st[SPT], a0[KB], a1[KB];
    auto row0 = [&](int c) { int cc = c + rot; if (cc >= nch) cc -= nch; return kb + 16 * KB * cc; };
    auto load = [&](int c, u4v *a) {
        const int k0 = row0(c);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = threadIdx.x + u * NTH;      // e = ((ks * 2 + half) * WC + col) * 4 + quad
            if (e < NV) {
                const int quad = e & 3, hc = e >> 2, col = hc % WC, hk = hc / WC, half = hk & 1;
                const int row = k0 + 16 * (hk >> 1) + 4 * quad;
                st[u] = row < ke ? *reinterpret_cast<const u4v *>((half ? Yl : Yh) + (long long)col * mp + row)
                                 : u4v{0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int ks = 0; ks < KB; ++ks) {
            const int kc0 = k0 + 16 * ks + 4 * q;
#pragma unroll
            for (int t = 0; t < 4; ++t) a[ks][t] = ap[(long long)min(kc0 + t, (int)m - 1) * m];
        }
    };
    auto stage = [&](int slot) {
        u4v *b = reinterpret_cast<u4v *>(buf) + slot * NV;
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = threadIdx.x + u * NTH;
            if (e < NV) b[e] = st[u];
        }
    };
    auto compute = [&](int slot, const u4v *a) {
#pragma unroll
        for (int ks = 0; ks < KB; ++ks) {
            const u4v *b = reinterpret_cast<const u4v *>(buf) + slot * NV + ks * NV1;
            u4v nre, nim;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                nre[t] = a[ks][t] ^ 0x00008000u;                               // -(Re a, -Im a)
                nim[t] = ((a[ks][t] >> 16) | (a[ks][t] << 16)) ^ 0x80008000u;  // -(Im a, Re a)
            }
            const v8bf vre = __builtin_bit_cast(v8bf, nre), vim = __builtin_bit_cast(v8bf, nim);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = ct * 16 + r;
                const v8bf h = __builtin_bit_cast(v8bf, b[col * 4 + q]), l = __builtin_bit_cast(v8bf, b[(WC + col) * 4 + q]);
                cr[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vre, h, cr[ct], 0, 0, 0);
                ci[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vim, h, ci[ct], 0, 0, 0);
                cr[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vre, l, cr[ct], 0, 0, 0);
                ci[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vim, l, ci[ct], 0, 0, 0);
            }
        }
    };
    load(0, a0);
    stage(0);
    for (int c = 0; c < nch; c += 2) {
        if (c + 1 < nch) load(c + 1, a1);
        __syncthreads();
        if (active) compute(0, a0);
        if (c + 1 >= nch) break;
        stage(1);
        if (c + 2 < nch) load(c + 2, a0);
        __syncthreads();
        if (active) compute(1, a1);
        if (c + 2 < nch) stage(0);
    }
}

// acc (16 rows x CT*16 columns) += T(16 x w) * Xs(w x CT*16) over K-steps [kbeg, kend) of four
// complex rows each: T entries loaded from `t_ptr(row, kc)` (always a valid address) and passed
// through `t_val(row, kc, loaded)`; Xs is an LDS tile, row-major [64][CT*16] complex.  Three real
// products per K-step as in the chunked products (here acc += T Xs: g1 = Re acc + sum P1,
// g2 = -sum P2, g3 = Re acc + Im acc + sum P3).
template <class R, int CT, class TPtr, class TVal>
__device__ __forceinline__ void wide_gemm_lds(typename Mfma<R>::v4 *cr, typename Mfma<R>::v4 *ci, const cpx<R> *xs,
                                              int kbeg, int kend, TPtr t_ptr, TVal t_val) {
    typedef typename Mfma<R>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    constexpr int WC = CT * 16;
    constexpr int KC = 2;
    if (kbeg >= kend) return;
    v4 g2[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        g2[ct] = v4{0, 0, 0, 0};
        ci[ct] += cr[ct];  // g3; cr is g1
    }
    cpx<R> a0[KC], a1[KC];
    auto load = [&](int ks0, cpx<R> *a) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int kc = 4 * (ks0 + u) + q;
            a[u] = ldf(t_ptr(r, kc < 64 ? kc : 63));
        }
    };
    auto compute = [&](int ks0, const cpx<R> *a) {
#pragma unroll
        for (int u = 0; u < KC; ++u) {
            const int ks = ks0 + u;
            const int kc = 4 * ks + q;
            const cpx<R> t = (ks < kend) ? t_val(r, kc, a[u]) : czero<R>();
            const R p1 = t.re, n2 = -t.im, p3 = t.re + t.im;
            const cpx<R> *xrow = xs + (kc < 64 ? kc : 63) * WC + r;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const cpx<R> y = xrow[ct * 16];
                cr[ct] = Mfma<R>::fma(p1, y.re, cr[ct]);
                g2[ct] = Mfma<R>::fma(n2, y.im, g2[ct]);
                ci[ct] = Mfma<R>::fma(p3, y.re + y.im, ci[ct]);
            }
        }
    };
    load(kbeg, a0);
    for (int ks0 = kbeg; ks0 < kend; ks0 += 2 * KC) {
        load(ks0 + KC, a1);
        __builtin_amdgcn_sched_barrier(0);
        compute(ks0, a0);
        __builtin_amdgcn_sched_barrier(0);
        if (ks0 + KC >= kend) break;
        load(ks0 + 2 * KC, a0);
        __builtin_amdgcn_sched_barrier(0);
        compute(ks0 + KC, a1);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        ci[ct] = ci[ct] - cr[ct] + g2[ct];
        cr[ct] += g2[ct];
    }
}

// Item = (stored block s, first column c0, column count, box).  Column g of block s is the
// pair (mode modes[mode_ptr[s] + g / nrhs], right-hand side g % nrhs).  Y is a per-item
// scratch, row-major [m][CT*16], holding y = L^{-1} P b and then x = U^{-1} y.  With bfloat16
// factors the split copy Yb alone holds y and the solved x rows, and Y receives x only when it
// is kept (out_mode 1), so a solve writes its solved rows once, not twice.
//
// NW wavefronts own 16 rows each of a super-tile of 16*NW rows (NW/4 tiles of 64 rows).
// Forward, per super-tile S:
//   acc = (P b)_S - L[S, 0:S] y[0:S]         one continuous K loop, every wavefront
//   for each tile i of S in order:
//     y_i = Linv_ii acc_i                     the tile's 4 wavefronts, through LDS
//     acc_j -= L[j, i] y_i  for tiles j > i of S   (y_i read from LDS)
// and backward the same with U from the last super-tile down.  The already solved rows are
// re-read once per super-tile (not once per tile), and with one workgroup per CU the
// per-item scratch of all resident workgroups stays in the last-level cache.
// Workgroup b of the grid takes item (b % 8) * per + b / 8 so that the eight XCDs work on
// contiguous item ranges (neighbouring modes share the cache lines of `work`).
// out_mode: 0 = write x to work; 1 = keep x in Y only; 2 = write x + Yadd to work (the
// correction step of a refined solve, Yadd holding the first solution).
// With bfloat16 factors the off-diagonal products run on the bfloat16 matrix cores against the
// solved rows split into bfloat16 hi + lo (Yb: [item][2][col][mp], mp = m rounded up to 16).
template <class R, int CT, int NW, class FT>
__global__ void __launch_bounds__(NW * 64) k_block_solve_wide(cpx<R> *work, const FT *F, const int *perm,
                                                               const int4 *items, int nitems, const int *mode_ptr,
                                                               const int *mode_list, cpx<R> *Y, int m, int n,
                                                               int nboxes, int nrhs, int out_mode,
                                                               const cpx<R> *Yadd, uint32_t *Yb, int mp, int mx) {
    typedef typename Mfma<R>::v4 v4;
    constexpr int WC = CT * 16;
    constexpr int ST = 16 * NW;  // rows per super-tile
    const int per = (nitems + 7) / 8;
    const int it = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (it >= nitems) return;  // whole workgroup, before any barrier
    const int4 item = items[it];
    const int sblk = item.x, c0 = item.y, ncols = item.z, box = item.w;
    cpx<R> *xs_c = reinterpret_cast<cpx<R> *>(vie_smem);  // [64][WC]: tile accumulators
    cpx<R> *ys_c = xs_c + TS * WC;                         // [64][WC]: solved tile
    cpx<R> *yb_c = ys_c + TS * WC;                         // staged chunks of solved rows (2 slots)
    const FT *A = F + (long long)sblk * m * m;
    const int *pm = perm + (long long)sblk * m;
    cpx<R> *Yi = Y + (long long)it * m * WC;
    const cpx<R> *Ya = Yadd ? Yadd + (long long)it * m * WC : nullptr;
    constexpr bool kBf16 = sizeof(FT) == 4;
    static_assert(!kBf16 || sizeof(R) == 4, "bfloat16 factors are solved in FP32");
    uint32_t *Yh = kBf16 ? Yb + (long long)it * 2 * WC * mp : nullptr;
    uint32_t *Yl = kBf16 ? Yh + (long long)WC * mp : nullptr;
    if (kBf16)  // zero padding rows m..mp-1 of the split copy (read by the last ragged K-step)
        for (int e = threadIdx.x; e < 2 * WC * (mp - m); e += blockDim.x) {
            const int col = e / (mp - m) % WC, row = m + e % (mp - m);
            (e < WC * (mp - m) ? Yh : Yl)[(long long)col * mp + row] = 0u;
        }
    const long long rstride = (long long)nboxes * m * n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int sub = wv >> 2;             // tile of this wavefront within the super-tile
    const int wrow = 16 * (wv & 3);      // first row of this wavefront within its tile
    long long off[CT];                   // column base offsets in work (-1: no column)
    int fl[CT];                          // reflected mode: rows where S = -1 change sign in and out
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + r;
        off[ct] = -1;
        fl[ct] = 0;
        if (col < ncols) {
            const int g = c0 + col;
            const int me = mode_list[mode_ptr[sblk] + g / nrhs];
            off[ct] = (long long)(g % nrhs) * rstride + (long long)box * m * n + (me & ~VIE_MODE_MIRROR);
            fl[ct] = me & VIE_MODE_MIRROR;
        }
    }
    const int NS = (m + ST - 1) / ST;
    v4 cr[CT], ci[CT];
    auto zero_acc = [&]() {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            cr[ct] = v4{0, 0, 0, 0};
            ci[ct] = v4{0, 0, 0, 0};
        }
    };
    // tile step of tile `tt` (rows t0..t0+w) inside a super-tile: the owners solve it, the
    // other wavefronts of the super-tile selected by `later` apply its column block.
    auto tile_step = [&](int tt, int t0, int w, bool lower, int s0) {
        const bool owner = sub == tt;
        if (owner) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    xs_c[(wrow + Mfma<R>::acc_row(q, v)) * WC + ct * 16 + r] = mk(cr[ct][v], ci[ct][v]);
        }
        __syncthreads();
        if (owner) {
            zero_acc();
            const FT *Aii = A + (long long)t0 * m + t0;
            const int wl = wv & 3;
            // addresses clamped into the tile (rows/columns >= w read entry (0, 0))
            auto tptr = [&](int rr, int kc) -> const FT * {
                const int row = wrow + rr;
                return (row < w && kc < w) ? Aii + (long long)kc * m + row : Aii;
            };
            if (lower)
                wide_gemm_lds<R, CT>(cr, ci, xs_c, 0, min((w + 3) / 4, 4 * (wl + 1)), tptr,
                                     [&](int rr, int kc, cpx<R> v) -> cpx<R> {
                                         const int row = wrow + rr;
                                         if (row >= w || kc >= w || kc > row) return czero<R>();
                                         return kc == row ? mk(R(1), R(0)) : v;
                                     });
            else
                wide_gemm_lds<R, CT>(cr, ci, xs_c, 4 * wl, (w + 3) / 4, tptr, [&](int rr, int kc, cpx<R> v) -> cpx<R> {
                    const int row = wrow + rr;
                    return (row >= w || kc >= w || kc < row) ? czero<R>() : v;
                });
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                uint32_t hv[4], lv[4];  // hi + lo bfloat16 split of the solved rows (bfloat16 factors)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = wrow + Mfma<R>::acc_row(q, v);
                    const cpx<R> x = mk(cr[ct][v], ci[ct][v]);
                    ys_c[row * WC + ct * 16 + r] = x;
                    if constexpr (kBf16) {
                        const uint32_t hr = bf16_bits((float)x.re), hi_ = bf16_bits((float)x.im);
                        const float lr = (float)x.re - __uint_as_float(hr << 16);
                        const float li = (float)x.im - __uint_as_float(hi_ << 16);
                        hv[v] = hr | (hi_ << 16);
                        lv[v] = bf16_bits(lr) | (bf16_bits(li) << 16);
                    }
                    if (row < w) {
                        const long long yo = (long long)(t0 + row) * WC + ct * 16 + r;
                        if (!kBf16 || (!lower && out_mode == 1)) Yi[yo] = x;
                        if (!lower && off[ct] >= 0 && out_mode != 1) {
                            const cpx<R> o = out_mode == 2 ? x + Ya[yo] : x;
                            work[off[ct] + (long long)(t0 + row) * n] =
                                mirror_flip(fl[ct], t0 + row, mx) ? mk(-o.re, -o.im) : o;
                        }
                    }
                }
                if constexpr (kBf16) {
                    // FP32 accumulators: register v holds row wrow + 4q + v, so a lane's four rows are
                    // consecutive in the column-major split copy: one 16-byte store each (rows
                    // t0 + wrow + 4q.. are 16-byte aligned: t0, wrow and mp are multiples of 16)
                    const int row0 = wrow + 4 * q;
                    const long long bo = (long long)(ct * 16 + r) * mp + t0 + row0;
                    if (row0 + 3 < w) {
                        *reinterpret_cast<uint4 *>(Yh + bo) = make_uint4(hv[0], hv[1], hv[2], hv[3]);
                        *reinterpret_cast<uint4 *>(Yl + bo) = make_uint4(lv[0], lv[1], lv[2], lv[3]);
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (row0 + v < w) {
                                Yh[bo + v] = hv[v];
                                Yl[bo + v] = lv[v];
                            }
                    }
                }
            }
        }
        __syncthreads();
        // the other tiles of the super-tile that still need this one
        const bool later = lower ? sub > tt : sub < tt;
        const int myt0 = s0 + TS * sub;
        if (later && myt0 < m) {
            const FT *Ab = A + (long long)t0 * m + myt0 + wrow;
            const bool rv = myt0 + wrow + r < m;
            wide_gemm_lds<R, CT>(
                cr, ci, ys_c, 0, (w + 3) / 4,
                [&](int rr, int kc) -> const FT * { return (rv && kc < w) ? Ab + (long long)kc * m + rr : A; },
                [&](int rr, int kc, cpx<R> v) -> cpx<R> { return (!rv || kc >= w) ? czero<R>() : mk(-v.re, -v.im); });
        }
    };
    // ---- forward
    for (int S = 0; S < NS; ++S) {
        const int s0 = S * ST;
        const int myt0 = s0 + TS * sub;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = myt0 + wrow + Mfma<R>::acc_row(q, v);
                const int src = row < m ? pm[row] : 0;
                cpx<R> b = (row < m && off[ct] >= 0) ? work[off[ct] + (long long)src * n] : czero<R>();
                if (mirror_flip(fl[ct], src, mx)) b = mk(-b.re, -b.im);
                cr[ct][v] = b.re;
                ci[ct][v] = b.im;
            }
        if (s0 > 0) {  // every wavefront stages; those past m only help
            const bool act = myt0 < m;
            const FT *ar = A + min(myt0 + wrow, m - 1);
            if constexpr (kBf16)
                wide_gemm_chunked_bf16<CT, NW * 64>(cr, ci, act, ar, A, m, myt0 + wrow + r < m, Yh, Yl, mp, 0, s0,
                                                    5 * sblk, reinterpret_cast<uint32_t *>(yb_c));
            else
                wide_gemm_chunked<R, CT, NW * 64>(cr, ci, act, ar, A, m, myt0 + wrow + r < m, Yi, 0, s0, 5 * sblk, yb_c);
        }
        __syncthreads();
        for (int tt = 0; tt < NW / 4; ++tt) {
            const int t0 = s0 + TS * tt;
            if (t0 >= m) break;
            tile_step(tt, t0, min(TS, m - t0), true, s0);
        }
        __syncthreads();
    }
    // ---- backward (x_i over y_i in Y)
    for (int S = NS - 1; S >= 0; --S) {
        const int s0 = S * ST;
        const int se = min(m, s0 + ST);
        const int myt0 = s0 + TS * sub;
        if constexpr (kBf16) {
            // y from its hi + lo split (about 17 significant bits, far below the error of the
            // bfloat16 factors): the lane's rows rb..rb+3 are consecutive in the column-major copy
            const int rb = myt0 + wrow + 4 * q;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                uint4 h = make_uint4(0, 0, 0, 0), l = h;
                if (rb < mp) {  // mp and rb are multiples of 16 and 4: rows rb..rb+3 exist (past m: zero)
                    const long long bo = (long long)(ct * 16 + r) * mp + rb;
                    h = *reinterpret_cast<const uint4 *>(Yh + bo);
                    l = *reinterpret_cast<const uint4 *>(Yl + bo);
                }
                const uint32_t hv[4] = {h.x, h.y, h.z, h.w}, lv[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    cr[ct][v] = __uint_as_float(hv[v] << 16) + __uint_as_float(lv[v] << 16);
                    ci[ct][v] = __uint_as_float(hv[v] & 0xffff0000u) + __uint_as_float(lv[v] & 0xffff0000u);
                }
            }
        } else {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = myt0 + wrow + Mfma<R>::acc_row(q, v);
                    cpx<R> y = row < m ? Yi[(long long)row * WC + ct * 16 + r] : czero<R>();
                    cr[ct][v] = y.re;
                    ci[ct][v] = y.im;
                }
        }
        if (se < m) {
            const bool act = myt0 < m;
            const FT *ar = A + min(myt0 + wrow, m - 1);
            if constexpr (kBf16)
                wide_gemm_chunked_bf16<CT, NW * 64>(cr, ci, act, ar, A, m, myt0 + wrow + r < m, Yh, Yl, mp, se, m,
                                                    5 * sblk, reinterpret_cast<uint32_t *>(yb_c));
            else
                wide_gemm_chunked<R, CT, NW * 64>(cr, ci, act, ar, A, m, myt0 + wrow + r < m, Yi, se, m, 5 * sblk, yb_c);
        }
        __syncthreads();
        for (int tt = NW / 4 - 1; tt >= 0; --tt) {
            const int t0 = s0 + TS * tt;
            if (t0 >= m) continue;
            tile_step(tt, t0, min(TS, m - t0), false, s0);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- refinement residual
// One refinement step of a solve with rounded (bfloat16) factors needs the residual of the
// block system itself: for an item of stored block s (factorised from D_k, k = smode[s]),
//   r^ <- r^ - D_k z0 = r^ - z0 + M~ (C^_k z0)          (over r^ in work)
// with z0 the first solve's result (the item's scratch, row-major [m][CT*16]) and
//   C^_k[(a,y,z), (b,y',z')] = C^_k^{c(a,b)}(y - y', z - z'),
// over the solve rows rows[0..m) (the cross-section rows with M~ != 0 when the identity rows
// are left out; their input enters the right-hand side before the first solve),
// the Chan/x-DFT table of the block (complex float, [6][2bz-1][2by-1] per mode, staged in
// LDS), c(a,b) the index of the unique component (xx, yy, zz, xy, xz, yz).  The product is
// a matrix-core GEMM whose left operand is generated from the table, in three real products
// per K-step of four complex columns (Gauss, as in the chunked solve products: lane (r, q)
// looks up entry (row r, column k0 + q)).  NW wavefronts take 16-row strips in turn.
template <int CT, int NW>
__global__ void __launch_bounds__(NW * 64) k_refine_residual(c64 *work, const c64 *chan, const c64 *mt,
                                                              const int *smode, const int4 *items, int nitems,
                                                              const int *mode_ptr, const int *mode_list,
                                                              const c64 *Y, const int *rows, int m, int n,
                                                              int nboxes, int nrhs, int by, int bz, int mx) {
    typedef Mfma<float>::v4 v4;
    constexpr int WC = CT * 16;
    constexpr int NTH = NW * 64;
    constexpr int YC = 16;                          // rows of z0 per staged chunk
    constexpr int SPT = (YC * WC + NTH - 1) / NTH;
    const int per = (nitems + 7) / 8;
    const int it = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (it >= nitems) return;
    const int4 item = items[it];
    const int sblk = item.x, c0 = item.y, ncols = item.z, box = item.w;
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1, plane = by * bz;
    const int tabn = 6 * ndz * ndy;
    c64 *tab = reinterpret_cast<c64 *>(vie_smem);
    c64 *buf = tab + ((tabn + 1) & ~1);             // two chunk slots of z0 rows
    // solve row j = (b, y', z'): b and the table offset z' (2by-1) + y' it subtracts, packed
    int *pk = reinterpret_cast<int *>(buf + 2 * YC * WC);
    const c64 *src = chan + (long long)smode[sblk] * tabn;
    for (int i = threadIdx.x; i < tabn; i += blockDim.x) tab[i] = src[i];
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const int pr = rows[j], b = pr / plane, yz = pr - b * plane;
        pk[j] = (b << 20) | ((yz / by) * ndy + yz % by);
    }
    const c64 *Yi = Y + (long long)it * m * WC;
    const long long rstride = (long long)nboxes * m * n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    long long off[CT];
    int fl[CT];  // reflected mode: the residual of S D_k S, i.e. rows of r - D_k z0 where S = -1 change sign
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = ct * 16 + r;
        off[ct] = -1;
        fl[ct] = 0;
        if (col < ncols) {
            const int g = c0 + col;
            const int me = mode_list[mode_ptr[sblk] + g / nrhs];
            off[ct] = (long long)(g % nrhs) * rstride + (long long)box * m * n + (me & ~VIE_MODE_MIRROR);
            fl[ct] = me & VIE_MODE_MIRROR;
        }
    }
    const int nch = (m + YC - 1) / YC;
    c64 st[SPT];
    auto load = [&](int c) {
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + u * NTH, row = c * YC + e / WC;
            st[u] = (e < YC * WC && row < m) ? Yi[(long long)row * WC + e % WC] : czero<float>();
        }
    };
    auto stage = [&](int slot) {
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + u * NTH;
            if (e < YC * WC) buf[slot * YC * WC + e] = st[u];
        }
    };
    // NW strips of 16 rows at a time; all wavefronts stage the shared z0 chunks
    for (int g0 = 0; g0 * 16 * NW < m; ++g0) {
        const int row0 = (g0 * NW + wv) * 16;
        const bool active = row0 < m;
        const int arow = rows[min(row0 + r, m - 1)];  // this lane's operand row (a, y, z)
        const int a = arow / plane, yz = arow - a * plane, z = yz / by, y = yz - z * by;
        // table index of (row, column (b, y', z')) = base[b] - (z' (2by-1) + y'), base[b] holding
        // the component c(a, b) and the row's own offsets
        const int rbase = (z + bz - 1) * ndy + (y + by - 1);
        const int base0 = (a == 0 ? 0 : a + 2) * ndz * ndy + rbase;   // c(a, 0): xx, xy, xz
        const int base1 = (a == 1 ? 1 : a + 3) * ndz * ndy + rbase;   // c(a, 1): xy, yy, yz
        const int base2 = (a == 2 ? 2 : a + 4) * ndz * ndy + rbase;   // c(a, 2): xz, yz, zz
        const int d01 = base1 - base0, d12 = base2 - base1;  // base[b] by masks (no indexed array)
        v4 g1[CT], g2[CT], g3[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            g1[ct] = v4{0, 0, 0, 0};
            g2[ct] = v4{0, 0, 0, 0};
            g3[ct] = v4{0, 0, 0, 0};
        }
        auto compute = [&](int slot, int c) {
            const c64 *ys = buf + slot * YC * WC + r;
#pragma unroll
            for (int u = 0; u < YC / 4; ++u) {
                const int kc = c * YC + 4 * u + q;
                const int pc = pk[min(kc, m - 1)];
                const int b = pc >> 20;
                const int ti = base0 + (d01 & -(b >= 1)) + (d12 & -(b >= 2)) - (pc & 0xfffff);
                const c64 t = kc < m ? tab[ti] : czero<float>();
                const float t3 = t.re + t.im;
                const c64 *yr = ys + (4 * u + q) * WC;
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const c64 v = yr[ct * 16];
                    g1[ct] = Mfma<float>::fma(t.re, v.re, g1[ct]);
                    g2[ct] = Mfma<float>::fma(t.im, v.im, g2[ct]);
                    g3[ct] = Mfma<float>::fma(t3, v.re + v.im, g3[ct]);
                }
            }
        };
        __syncthreads();  // previous group's chunk reads done (and the table staged)
        load(0);
        stage(0);
        for (int c = 0; c < nch; c += 2) {
            if (c + 1 < nch) load(c + 1);
            __syncthreads();
            if (active) compute(0, c);
            if (c + 1 >= nch) break;
            stage(1);
            if (c + 2 < nch) load(c + 2);
            __syncthreads();
            if (active) compute(1, c + 1);
            if (c + 2 < nch) stage(0);
        }
        if (active) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = row0 + Mfma<float>::acc_row(q, v);
                    if (row < m && off[ct] >= 0) {
                        const c64 mv = mt[(long long)box * plane + rows[row] % plane];  // M~ at (z, y)
                        const c64 z0 = Yi[(long long)row * WC + ct * 16 + r];
                        const long long wo = off[ct] + (long long)row * n;
                        const c64 t = mv * mk(g1[ct][v] - g2[ct][v], g3[ct][v] - g1[ct][v] - g2[ct][v]);
                        work[wo] = mirror_flip(fl[ct], row, mx) ? work[wo] + z0 - t : work[wo] - z0 + t;
                    }
                }
        }
    }
}

// ---------------------------------------------------------------- schedule + launch
#define WIDE_MIN_COLS 16
#define WIDE_MAX_COLS 64
#define WIDE_MIN_RHS 8  // below this the per-mode narrow solve keeps every CU busy

// Split the stored blocks between the two kernels for `nrhs` right-hand sides and upload the
// tables (only when nrhs changed since the last apply).
static vie_status build_schedule(vie_pc pc, PcWs *w, int nrhs, hipStream_t s) {
    if (w->sched_nrhs == nrhs) return VIE_OK;
    const int n = pc->nm;
    // bfloat16 factors are solved on the matrix cores only (every block goes wide)
    const bool all_wide = pc->prec == VIE_BF16C;
    const int min_cols = all_wide ? 1 : WIDE_MIN_COLS, min_rhs = all_wide ? 1 : w->cfg_min_rhs;
    std::vector<int> wide;    // int4 items
    std::vector<int> narrow;  // int4 items of narrow_rc columns (tiny blocks: 64/m columns)
    const bool tiny = pc->m <= TS;
    const int rc = w->cfg_rc ? w->cfg_rc : block_solve_rc(pc->m, block_cols_max(pc, nrhs),
                                                            pc->prec == VIE_C128 ? sizeof(c128) : sizeof(c64));
    int maxc = 0;
    long long wide_cols = 0;
    for (int sb = 0; sb < pc->nstored; ++sb) {
        const long long cols = (long long)(pc->mode_ptr[sb + 1] - pc->mode_ptr[sb]) * nrhs;
        if (cols >= min_cols && nrhs >= min_rhs) wide_cols += cols;
    }
    int gmax = w->cfg_gmax;
    if (gmax == 0) {
        // default: FP64 the narrowest group (16 columns: several workgroups per CU hide the
        // latency of the factor stream better than wider column tiles, whose registers allow
        // only one); bfloat16 32 columns; complex64 the widest group; each halved while it
        // gives fewer than 512 workgroups
        gmax = pc->prec == VIE_C128 ? WIDE_MIN_COLS : pc->prec == VIE_BF16C ? 32 : WIDE_MAX_COLS;
        while (gmax > WIDE_MIN_COLS && wide_cols / gmax < 512) gmax /= 2;
    }
    for (int sb = 0; sb < pc->nstored; ++sb) {
        const int cnt = pc->mode_ptr[sb + 1] - pc->mode_ptr[sb];
        const long long cols = (long long)cnt * nrhs;
        if (cols >= min_cols && nrhs >= min_rhs) {
            const long long ng = (cols + gmax - 1) / gmax;
            const long long per = (cols + ng - 1) / ng;
            for (long long c = 0; c < cols; c += per) {
                const int nc = (int)std::min(per, cols - c);
                wide.insert(wide.end(), {sb, (int)c, nc, pc->block_box[sb]});
                maxc = std::max(maxc, nc);
            }
        } else {
            const int per = tiny ? TS / pc->m : rc;  // columns per wavefront / per workgroup
            for (long long c = 0; c < cols; c += per)
                narrow.insert(narrow.end(), {sb, (int)c, (int)std::min<long long>(per, cols - c), pc->block_box[sb]});
        }
    }
    w->n_wide = (int)(wide.size() / 4);
    w->n_narrow = (int)(narrow.size() / 4);
    w->narrow_rc = rc;
    w->wide_ct = maxc <= 16 ? 1 : maxc <= 32 ? 2 : 4;
    std::vector<int> tab(wide);
    tab.insert(tab.end(), narrow.begin(), narrow.end());
    VIE_CHECK(w->sched.ensure(sizeof(int) * std::max<size_t>(tab.size(), 4)));
    VIE_HIP(hipMemcpyAsync(w->sched.p, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, s));
    VIE_HIP(hipStreamSynchronize(s));  // the host table is freed on return
    w->sched_nrhs = nrhs;
    return VIE_OK;
}

template <class R, int CT, int NW, class FT>
static void launch_wide_nw(vie_pc pc, PcWs *w, cpx<R> *work, cpx<R> *Y, int nrhs, int out_mode, const cpx<R> *Yadd,
                           hipStream_t s) {
    const int per = (w->n_wide + 7) / 8;
    // two 64-row tiles + two chunk slots of 16 solved rows (bfloat16: hi + lo of 16 BF_KSTEPS rows)
    const size_t chunk = sizeof(FT) == 4 ? 2 * 2 * (size_t)CT * 16 * 16 * BF_KSTEPS * sizeof(uint32_t)
                                         : 2 * (size_t)16 * CT * 16 * sizeof(cpx<R>);
    const size_t lds = 2 * sizeof(cpx<R>) * TS * CT * 16 + chunk;
    vie_lds_attr((const void *)k_block_solve_wide<R, CT, NW, FT>, lds);
    const int *mp = pc->modes_dev.as<const int>();
    hipLaunchKernelGGL((k_block_solve_wide<R, CT, NW, FT>), dim3(8 * per), dim3(NW * 64), lds, s, work,
                       pc->factors.as<const FT>(), pc->perm.as<const int>(), w->sched.as<const int4>(), w->n_wide,
                       mp, mp + pc->nstored + 1, Y, pc->m, pc->nm, pc->nboxes, nrhs, out_mode, Yadd,
                       w->wide_bf16.as<uint32_t>(), (pc->m + 15) / 16 * 16, pc->mirror_rows);
}

// wavefronts per workgroup (16 NW rows per super-tile): 8 or 16 for FP32, 4 or 8 for FP64
static int wide_nw(vie_pc pc, const PcWs *w, bool fp32) {
    if (w->cfg_nw) return w->cfg_nw;
    if (pc->prec == VIE_BF16C) return 8;  // the bfloat16 double buffers need > 128 VGPRs
    return fp32 ? 16 : 8;
}

template <class R, int CT, class FT>
static void launch_wide(vie_pc pc, PcWs *w, cpx<R> *work, cpx<R> *Y, int nrhs, int out_mode, const cpx<R> *Yadd,
                        hipStream_t s) {
    const int nw = wide_nw(pc, w, sizeof(R) == 4);
    if (sizeof(R) == 4) {
        if (nw == 8) launch_wide_nw<R, CT, 8, FT>(pc, w, work, Y, nrhs, out_mode, Yadd, s);
        else launch_wide_nw<R, CT, 16, FT>(pc, w, work, Y, nrhs, out_mode, Yadd, s);
    } else {
        if (nw == 4) launch_wide_nw<R, CT, 4, FT>(pc, w, work, Y, nrhs, out_mode, Yadd, s);
        else launch_wide_nw<R, CT, 8, FT>(pc, w, work, Y, nrhs, out_mode, Yadd, s);
    }
}

template <int CT, int NW>
static void launch_residual_nw(vie_pc pc, PcWs *w, c64 *work, const c64 *Y, int nrhs, size_t lds, hipStream_t s) {
    const int per = (w->n_wide + 7) / 8;
    vie_lds_attr((const void *)k_refine_residual<CT, NW>, lds);
    const int *mp = pc->modes_dev.as<const int>();
    hipLaunchKernelGGL((k_refine_residual<CT, NW>), dim3(8 * per), dim3(NW * 64), lds, s, work,
                       pc->chan32.as<const c64>(), pc->mt32.as<const c64>(), pc->smode_dev.as<const int>(),
                       w->sched.as<const int4>(), w->n_wide, mp, mp + pc->nstored + 1, Y,
                       pc->rows.as<const int>(), pc->m, pc->nm, pc->nboxes, nrhs, pc->by, pc->bz, pc->mirror_rows);
}

// 16 wavefronts in one workgroup per CU (the table fills most of the LDS), or, for 32-column
// groups whose workgroup fits in half the LDS, 8 wavefronts in two workgroups per CU, whose
// barriers then overlap (coupler, 32 columns: 3.29 -> 2.84 ms; 16 and 64 columns measured
// slower with 8: the former barely, the latter's registers allow only one such workgroup)
template <int CT>
static void launch_residual(vie_pc pc, PcWs *w, c64 *work, const c64 *Y, int nrhs, hipStream_t s) {
    const size_t tabn = 6 * (size_t)(2 * pc->bz - 1) * (2 * pc->by - 1);
    const size_t lds = sizeof(c64) * (((tabn + 1) & ~(size_t)1) + 2 * 16 * CT * 16) + sizeof(int) * pc->m;
    if constexpr (CT == 2) {
        if (lds <= 80 * 1024) {
            launch_residual_nw<CT, 8>(pc, w, work, Y, nrhs, lds, s);
            return;
        }
    }
    launch_residual_nw<CT, 16>(pc, w, work, Y, nrhs, lds, s);
}

template <class R, class FT>
static vie_status block_solve_run(vie_pc pc, PcWs *w, cpx<R> *work, int nrhs, hipStream_t s) {
    const int m = pc->m, n = pc->nm;
    const int qr = (m + 255) / 256;
    VIE_CHECK(build_schedule(pc, w, nrhs, s));
    if (w->n_wide > 0) {
        const int WC = 16 * w->wide_ct;
        const size_t ybytes = sizeof(cpx<R>) * (size_t)w->n_wide * m * WC;
        VIE_CHECK(w->wide_scratch.ensure(ybytes));
        cpx<R> *Y = w->wide_scratch.as<cpx<R>>();
        if (pc->prec == VIE_BF16C)  // hi + lo bfloat16 copies of the solved rows
            VIE_CHECK(w->wide_bf16.ensure(sizeof(uint32_t) * 2 * (size_t)w->n_wide * WC * ((m + 15) / 16 * 16)));
        // refinement comes with bfloat16 factors only; the correcting solve (out_mode 2) then
        // neither reads nor writes its Y (its solved rows live in the split copy), so it is handed
        // the first solve's Y, which it reads as Yadd
        const bool refine = pc->refine && pc->prec == VIE_BF16C;
        cpx<R> *Y2 = Y;
#define WIDE_CASES(CTV)                                                                                  \
    if (!refine) {                                                                                       \
        launch_wide<R, CTV, FT>(pc, w, work, Y, nrhs, 0, nullptr, s);                                       \
    } else {                                                                                             \
        launch_wide<R, CTV, FT>(pc, w, work, Y, nrhs, 1, nullptr, s);                                       \
        VIE_HIP(hipGetLastError());                                                                      \
        {                                                                                                \
            ProfScope pr("refine_residual", s);                                                          \
            launch_residual<CTV>(pc, w, (c64 *)work, (const c64 *)Y, nrhs, s);                              \
            VIE_HIP(hipGetLastError());                                                                  \
        }                                                                                                \
        launch_wide<R, CTV, FT>(pc, w, work, Y2, nrhs, 2, Y, s);                                            \
    }
        switch (w->wide_ct) {
            case 1: WIDE_CASES(1) break;
            case 2: WIDE_CASES(2) break;
            default: WIDE_CASES(4) break;
        }
#undef WIDE_CASES
        VIE_HIP(hipGetLastError());
    }
    if (w->n_narrow > 0 && m <= TS) {
        const int4 *items = reinterpret_cast<const int4 *>(w->sched.as<const int>() + 4 * w->n_wide);
        const int nitems = w->n_narrow;
        const int *mp = pc->modes_dev.as<const int>();
        hipLaunchKernelGGL((k_block_solve_tiny<R, FT>), dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s, work,
                           pc->factors.as<const FT>(), pc->perm.as<const int>(), items, mp, mp + pc->nstored + 1, m,
                           n, pc->nboxes, nrhs, nitems, pc->mirror_rows);
        VIE_HIP(hipGetLastError());
    } else if (w->n_narrow > 0) {
        const int rc = w->narrow_rc;
        dim3 grid((unsigned)w->n_narrow);
        size_t lds = 5 * (size_t)TS * rc * sizeof(cpx<R>);
        const int *mp = pc->modes_dev.as<const int>();
        const NarrowArgs a{reinterpret_cast<const int4 *>(w->sched.as<const int>() + 4 * w->n_wide), mp,
                           mp + pc->nstored + 1, m, n, pc->nboxes, nrhs, pc->mirror_rows};
        const FT *F = pc->factors.as<const FT>();
        const int *perm = pc->perm.as<const int>();
        switch (qr) {
            case 1: launch_bs_rc<R, 1>(rc, grid, lds, s, work, F, perm, a); break;
            case 2: launch_bs_rc<R, 2>(rc, grid, lds, s, work, F, perm, a); break;
            case 3: launch_bs_rc<R, 3>(rc, grid, lds, s, work, F, perm, a); break;
            case 4: launch_bs_rc<R, 4>(rc, grid, lds, s, work, F, perm, a); break;
            default: launch_bs_rc<R, 5>(rc, grid, lds, s, work, F, perm, a); break;
        }
        VIE_HIP(hipGetLastError());
    }
    return VIE_OK;
}

// Launch parameters of the block solves for `nrhs` right-hand sides: the defaults, or with
// autotuning on the fastest candidate for this shape (timed on a copy of `work`, since the
// solves run in place), looked up in or added to the process-wide cache.
template <class R, class FT>
static vie_status block_solve_t(vie_pc pc, PcWs *w, cpx<R> *work, int nrhs, hipStream_t s) {
    if ((pc->m + 255) / 256 > VIE_MAX_QR) {
        vie_set_error("block size above 1280 is not supported by the block solve");
        return VIE_EARG;
    }
    if (tune_enabled() && w->tuned_nrhs != nrhs) {
        const bool bf = pc->prec == VIE_BF16C, fp32 = sizeof(R) == 4;
        char key[160];
        snprintf(key, sizeof key, "block_solve prec=%d m=%d n=%d boxes=%d stored=%d nrhs=%d refine=%d", pc->prec,
                 pc->m, pc->nm, pc->nboxes, pc->nstored, nrhs, pc->refine);
        std::vector<std::vector<int>> cands;  // {gmax, nw, rc, min_rhs}
        const int rcmax = block_solve_rc(pc->m, block_cols_max(pc, nrhs), sizeof(cpx<R>));
        const int nws[2] = {fp32 ? 8 : 4, fp32 ? 16 : 8};
        if (bf || nrhs >= WIDE_MIN_RHS)
            for (int g = 16; g <= WIDE_MAX_COLS; g *= 2)
                for (int nw : nws) cands.push_back({g, nw, 0, bf ? 1 : WIDE_MIN_RHS});
        if (!bf && nrhs < 32)
            for (int rc = 1; rc <= rcmax; rc *= 2) cands.push_back({0, 0, rc, 1 << 30});
        std::vector<int> choice;
        if (tune_lookup(key, &choice)) {
            VIE_CHECK(tune_check_choice(key, choice, cands));
        } else {
            if (cands.size() > 1) {
                const size_t bytes = sizeof(cpx<R>) * (size_t)nrhs * pc->nboxes * pc->m * pc->nm;
                DevBuf copy;
                VIE_CHECK(copy.ensure(bytes));
                double best = 1e300;
                for (auto &c : cands) {
                    w->cfg_gmax = c[0], w->cfg_nw = c[1], w->cfg_rc = c[2], w->cfg_min_rhs = c[3];
                    w->sched_nrhs = 0;
                    double ms = 0;
                    VIE_CHECK(tune_time(s, 2, [&]() -> vie_status {
                        VIE_HIP(hipMemcpyAsync(copy.p, work, bytes, hipMemcpyDeviceToDevice, s));
                        return block_solve_run<R, FT>(pc, w, copy.as<cpx<R>>(), nrhs, s);
                    }, &ms));
                    if (ms < best) {
                        best = ms;
                        choice = c;
                    }
                }
                tune_store(key, choice, best, (int)cands.size());
            } else if (cands.size() == 1) {
                choice = cands[0];
                tune_store(key, choice, 0.0, 1);
            }
        }
        if (!choice.empty()) {
            w->cfg_gmax = choice[0], w->cfg_nw = choice[1], w->cfg_rc = choice[2], w->cfg_min_rhs = choice[3];
            w->sched_nrhs = 0;
        }
        w->tuned_nrhs = nrhs;
    }
    return block_solve_run<R, FT>(pc, w, work, nrhs, s);
}

vie_status launch_block_solve(vie_pc pc, PcWs *w, void *work, int nrhs, hipStream_t s) {
    if (pc->prec == VIE_C128) return block_solve_t<double, c128>(pc, w, (c128 *)work, nrhs, s);
    if (pc->prec == VIE_BF16C) return block_solve_t<float, bf16c>(pc, w, (c64 *)work, nrhs, s);
    return block_solve_t<float, c64>(pc, w, (c64 *)work, nrhs, s);
}
