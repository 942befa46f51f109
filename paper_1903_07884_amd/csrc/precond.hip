// Chan-Olkin 1-level block-circulant preconditioner (Sec. 4), its
// memory-reduced (Sec. 5.1.1), homogenised (Sec. 5.2) and blocked (Sec. 5.3)
// variants.
//
// Setup, per box of length n along x and cross-section (by, bz), m = 3 by bz:
//   * homogenised contrast M~(y, z) of the box (Sec. 5.2, three choices),
//   * for every block pair ((a,y,z),(b,y',z')) the x-level Toeplitz sequence
//     of N = I + K depends only on (ab, y-y', z-z'); T. Chan's circulant
//     c_l = ((n-l)/n) t_l + (l/n) t_{l-n} (eq. Chan) of each of these
//     6 (2by-1)(2bz-1) sequences is transformed along x by an LDS FFT
//     (C = F^{-1} diag(F c) F, Sec. 4), giving the table Chat_k,
//   * D_k[(a,y,z),(b,y',z')] = delta - M~(y,z) Chat_k^{ab}(y-y', z-z')
//     (eq. Di, with the permutation P folded into the indexing),
//   * memory reduction: v_k = Chat_k of K at (x, 0, 0 | x, column
//     ceil(by/2) ceil(bz/2)) (eq. proxy1); modes with |v_k|/max|v| <= tol
//     share the central block D_{ceil(n/2)} (eq. proxy2),
//   * LU with partial pivoting of every stored block, batched over blocks:
//     right-looking, panel of NB columns, row swaps + triangular solve for the
//     block row of U, tiled update of the trailing matrix.
// Apply z = P^{-1} r (inverse after eq. Di): per box line a forward x-FFT, one
// workgroup per (rhs, box, mode) doing the pivoted forward/backward
// substitution straight out of the FFT output (the permutation to mode-major
// order is an index map, no data copy), inverse x-FFT scaled by 1/n.
#include <algorithm>
#include <cmath>
#include <map>

#include "fft_device.h"

#define LU_NB 32
#define LU_TILE 64

// ---------------------------------------------------------------- homogenisation
// One workgroup per (box, z, y) row of a box: M~ = M(x0) (NONE, x-invariance checked),
// mean or real part of the mean along x (Sec. 5.2, items 2 and 3).
__global__ void __launch_bounds__(256) k_homog(const c128 *M, c128 *Mt, const int *boxes, int nx, int ny, int by,
                                               int bz, int kind, int *violation) {
    __shared__ c128 red[256];
    int i = blockIdx.x;
    int per = by * bz;
    int b = i / per, r = i % per;
    int y = r % by, z = r / by;
    const int *bx = boxes + 6 * b;
    const c128 *row = M + ((long long)(bx[2] + z) * ny + (bx[1] + y)) * nx + bx[0];
    int n = bx[3];
    c128 first = row[0];
    c128 acc = czero<double>();
    int bad = 0;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        c128 v = row[x];
        acc = acc + v;
        if (v.re != first.re || v.im != first.im) bad = 1;
    }
    if (kind == VIE_HOMOG_NONE) {
        if (bad) atomicOr(violation, 1);
        if (threadIdx.x == 0) Mt[i] = first;
        return;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) Mt[i] = mk(red[0].re / n, kind == VIE_HOMOG_REALMEAN ? 0.0 : red[0].im / n);
}

// ---------------------------------------------------------------- Chan table
// One workgroup per (component, dy, dz); output Ch[k][c][dz + bz - 1][dy + by - 1].
__global__ void k_chan_table(const c128 *gen, c128 *Ch, int nx, int ny, int nz, int n, int by, int bz,
                             int identity, FftPlan plan) {
    c128 *a = reinterpret_cast<c128 *>(vie_smem);
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1;
    int seq = blockIdx.x;
    int c = seq / (ndy * ndz);
    int rem = seq % (ndy * ndz);
    int iz = rem / ndy, iy = rem % ndy;
    int dy = iy - (by - 1), dz = iz - (bz - 1);
    const int oa[6] = {-1, -1, -1, 0, 0, 1}, ob[6] = {-1, -1, -1, 1, 2, 2};
    long long N = (long long)nx * ny * nz;
    const c128 *g = gen + c * N + ((long long)abs(dz) * ny + abs(dy)) * nx;
    // t_l = N^{ab}(l, dy, dz), l in (-n, n): parity sign from the octant
    auto t_at = [&](int l) -> c128 {
        c128 v = g[abs(l)];
        if (c >= 3) {
            int d[3] = {l, dy, dz};
            double s = 1.0;
            if (d[oa[c]] < 0) s = -s;
            if (d[ob[c]] < 0) s = -s;
            v = mk(s * v.re, s * v.im);
        }
        if (identity && c < 3 && l == 0 && dy == 0 && dz == 0) v.re += 1.0;
        return v;
    };
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        double w1 = (double)(n - l) / n, w2 = (double)l / n;
        c128 v = t_at(l);
        v = mk(w1 * v.re, w1 * v.im);
        if (l > 0) {
            c128 u = t_at(l - n);
            v = v + mk(w2 * u.re, w2 * u.im);
        }
        a[l] = v;
    }
    __syncthreads();
    c128 *res = fft_line<double>(a, plan, false);
    const long long stride_k = 6LL * ndz * ndy;
    for (int k = threadIdx.x; k < n; k += blockDim.x) Ch[k * stride_k + (long long)c * ndz * ndy + iz * ndy + iy] = res[k];
}

// ---------------------------------------------------------------- assembly
// D[s] column-major m x m, s-th stored block (mode ks, box bs)
template <class R>
__global__ void k_assemble(const c128 *Ch, const c128 *Mt, const int *blk_mode, const int *blk_box,
                           cpx<R> *D, int by, int bz) {
    const int m = 3 * by * bz;
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1;
    int s = blockIdx.y;
    long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)m * m) return;
    int r = (int)(e % m), col = (int)(e / m);
    int ar = r / (by * bz), yr = r % by, zr = (r / by) % bz;
    int ac = col / (by * bz), yc = col % by, zc = (col / by) % bz;
    int k = blk_mode[s], b = blk_box[s];
    const int cidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    int c = cidx[ar][ac];
    c128 ch = Ch[(long long)k * 6 * ndz * ndy + (long long)c * ndz * ndy + (zr - zc + bz - 1) * ndy + (yr - yc + by - 1)];
    c128 mt = Mt[(long long)b * by * bz + zr * by + yr];
    c128 v = mt * ch;
    v = mk(-v.re, -v.im);
    if (r == col) v.re += 1.0;
    D[(long long)s * m * m + e] = mk((R)v.re, (R)v.im);
}

// ---------------------------------------------------------------- batched LU
template <class R>
__device__ __forceinline__ R cabs2(cpx<R> a) { return a.re * a.re + a.im * a.im; }

// argmax over the workgroup of (value, index); ties -> smaller index.  Result in (sv[0], si[0]).
template <class R>
__device__ __forceinline__ void block_argmax(R v, int idx, R *sv, int *si) {
    for (int off = 32; off > 0; off >>= 1) {
        R ov = __shfl_down(v, off);
        int oi = __shfl_down(idx, off);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sv[1 + wid] = v;
        si[1 + wid] = idx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        R bv = sv[1];
        int bi = si[1];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
            if (sv[1 + k] > bv || (sv[1 + k] == bv && si[1 + k] < bi)) {
                bv = sv[1 + k];
                bi = si[1 + k];
            }
        sv[0] = bv;
        si[0] = bi;
    }
    __syncthreads();
}

// Factor the panel rows [j0, m), columns [j0, j0 + w) of every block (one workgroup per block):
// per column a wavefront-shuffle pivot search, the row interchange inside the panel, and the
// scaled rank-1 update of the remaining panel columns, which also yields the next column's
// pivot candidates.
template <class R>
__global__ void __launch_bounds__(256) k_lu_panel(cpx<R> *A, int *ipiv, int *info, int m, int j0, int w) {
    __shared__ R sv[1 + 256 / 64];
    __shared__ int si[1 + 256 / 64];
    cpx<R> *a = A + (long long)blockIdx.x * m * m;
    int *piv = ipiv + (long long)blockIdx.x * m;
    // candidates for the first column
    R best = R(-1);
    int bi = j0;
    for (int i = j0 + threadIdx.x; i < m; i += blockDim.x) {
        R v = cabs2(a[(long long)j0 * m + i]);
        if (v > best) {
            best = v;
            bi = i;
        }
    }
    for (int j = j0; j < j0 + w; ++j) {
        block_argmax<R>(best, bi, sv, si);
        int p = si[0];
        R pv = sv[0];
        if (threadIdx.x == 0) piv[j] = p;
        if (pv == R(0)) {
            if (threadIdx.x == 0 && info[blockIdx.x] == 0) info[blockIdx.x] = j + 1;
            // no elimination; next column's candidates
            best = R(-1);
            bi = j + 1;
            if (j + 1 < j0 + w)
                for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
                    R v = cabs2(a[(long long)(j + 1) * m + i]);
                    if (v > best) {
                        best = v;
                        bi = i;
                    }
                }
            continue;
        }
        if (p != j)
            for (int c = j0 + (int)threadIdx.x; c < j0 + w; c += blockDim.x) {
                cpx<R> t = a[(long long)c * m + j];
                a[(long long)c * m + j] = a[(long long)c * m + p];
                a[(long long)c * m + p] = t;
            }
        __syncthreads();
        cpx<R> piv_v = a[(long long)j * m + j];
        R d = cabs2(piv_v);
        cpx<R> inv = mk(piv_v.re / d, -piv_v.im / d);
        best = R(-1);
        bi = j + 1;
        for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
            cpx<R> l = a[(long long)j * m + i] * inv;
            a[(long long)j * m + i] = l;
            for (int c = j + 1; c < j0 + w; ++c) {
                cpx<R> v = cfms(a[(long long)c * m + i], l, a[(long long)c * m + j]);
                a[(long long)c * m + i] = v;
                if (c == j + 1) {
                    R q = cabs2(v);
                    if (q > best) {
                        best = q;
                        bi = i;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Row interchanges of the panel applied to the other columns, and for columns right of the
// panel U12 = L11^{-1} A12.  One workgroup per (64-column tile, block): rows [j0, j0 + w) of
// the tile are staged in LDS with coalesced loads; interchanges with rows below the panel are
// exchanged with global memory.
template <class R>
__global__ void __launch_bounds__(256) k_lu_swap_trsm(cpx<R> *A, const int *ipiv, int m, int j0, int w) {
    __shared__ cpx<R> T[LU_NB][65];
    __shared__ cpx<R> L11[LU_NB][LU_NB + 1];
    __shared__ int pv[LU_NB];
    const int c0 = blockIdx.x * 64;
    cpx<R> *a = A + (long long)blockIdx.y * m * m;
    if ((int)threadIdx.x < w) pv[threadIdx.x] = ipiv[(long long)blockIdx.y * m + j0 + threadIdx.x];
    for (int e = threadIdx.x; e < w * 64; e += blockDim.x) {
        int r = e % w, c = e / w, col = c0 + c;
        bool live = col < m && !(col >= j0 && col < j0 + w);
        T[r][c] = live ? a[(long long)col * m + j0 + r] : czero<R>();
    }
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        int r = e % w, c = e / w;
        L11[r][c] = a[(long long)(j0 + c) * m + j0 + r];
    }
    __syncthreads();
    const int c = threadIdx.x;
    const int col = c0 + c;
    const bool live = c < 64 && col < m && !(col >= j0 && col < j0 + w);
    if (live) {
        for (int j = 0; j < w; ++j) {
            int p = pv[j];
            if (p == j0 + j) continue;
            if (p < j0 + w) {
                cpx<R> t = T[j][c];
                T[j][c] = T[p - j0][c];
                T[p - j0][c] = t;
            } else {
                cpx<R> t = a[(long long)col * m + p];
                a[(long long)col * m + p] = T[j][c];
                T[j][c] = t;
            }
        }
        if (col >= j0 + w)
            for (int j = 0; j < w; ++j) {
                cpx<R> u = T[j][c];
                for (int i = j + 1; i < w; ++i) T[i][c] = cfms(T[i][c], L11[i][j], u);
            }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * 64; e += blockDim.x) {
        int r = e % w, cc = e / w, cl = c0 + cc;
        if (cl < m && !(cl >= j0 && cl < j0 + w)) a[(long long)cl * m + j0 + r] = T[r][cc];
    }
}

// A22 -= L21 U12 on 64x64 tiles, 4x4 complex outputs per thread.
template <class R>
__global__ void __launch_bounds__(256) k_lu_update(cpx<R> *A, int m, int j0, int w) {
    __shared__ cpx<R> Ls[LU_NB][LU_TILE];
    __shared__ cpx<R> Us[LU_NB][LU_TILE];
    const int t0 = j0 + w;
    const int nt = (m - t0 + LU_TILE - 1) / LU_TILE;
    int ti = blockIdx.x % nt, tj = blockIdx.x / nt;
    int r0 = t0 + ti * LU_TILE, c0 = t0 + tj * LU_TILE;
    cpx<R> *a = A + (long long)blockIdx.y * m * m;
    for (int e = threadIdx.x; e < LU_NB * LU_TILE; e += 256) {
        int k = e / LU_TILE, i = e % LU_TILE;
        cpx<R> lv = czero<R>(), uv = czero<R>();
        if (k < w) {
            if (r0 + i < m) lv = a[(long long)(j0 + k) * m + r0 + i];
            if (c0 + i < m) uv = a[(long long)(c0 + i) * m + j0 + k];
        }
        Ls[k][i] = lv;
        Us[k][i] = uv;
    }
    __syncthreads();
    int tr = threadIdx.x % 16, tc = threadIdx.x / 16;
    cpx<R> acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = czero<R>();
    for (int k = 0; k < w; ++k) {
        cpx<R> lv[4], uv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) lv[i] = Ls[k][tr + 16 * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) uv[j] = Us[k][tc + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j].re += lv[i].re * uv[j].re - lv[i].im * uv[j].im;
                acc[i][j].im += lv[i].re * uv[j].im + lv[i].im * uv[j].re;
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int c = c0 + tc + 16 * j;
        if (c >= m) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r = r0 + tr + 16 * i;
            if (r >= m) continue;
            cpx<R> &x = a[(long long)c * m + r];
            x = x - acc[i][j];
        }
    }
}

__global__ void k_lu_perm(const int *ipiv, int *perm, int m, int nblk) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nblk) return;
    int *p = perm + (long long)s * m;
    const int *iv = ipiv + (long long)s * m;
    for (int i = 0; i < m; ++i) p[i] = i;
    for (int j = 0; j < m; ++j) {
        int q = iv[j];
        int t = p[j];
        p[j] = p[q];
        p[q] = t;
    }
}

#define TS 64
// Setup: replace every 64x64 diagonal tile of the packed LU factors by the inverses of its
// unit-lower part (strictly lower entries) and of its upper part (upper entries incl. the
// diagonal).  The block solves then apply each diagonal tile as a parallel product.
// One workgroup (128 threads) per (tile, block): thread j < 64 inverts column j of L,
// thread 64 + j column j of U, both from an LDS copy of the tile.
template <class R>
__global__ void __launch_bounds__(128) k_invert_diag(cpx<R> *F, int m) {
    cpx<R> *T = reinterpret_cast<cpx<R> *>(vie_smem);  // [TS][TS+1], column-major: T[c*(TS+1)+r]
    cpx<R> *X = T + TS * (TS + 1);
    const int t0 = blockIdx.x * TS;
    const int w = min(TS, m - t0);
    cpx<R> *a = F + (long long)blockIdx.y * m * m;
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        int r = e % w, c = e / w;
        T[c * (TS + 1) + r] = a[(long long)(t0 + c) * m + t0 + r];
    }
    __syncthreads();
    int j = threadIdx.x & 63;
    if (j < w) {
        if (threadIdx.x < 64) {
            // column j of L^{-1} (unit lower): x_j = 1 (implicit; the diagonal slot belongs to U^{-1}),
            // x_i = -(l_ij + sum_{k=j+1}^{i-1} l_ik x_k)
            for (int i = j + 1; i < w; ++i) {
                cpx<R> acc = T[j * (TS + 1) + i];
                for (int k = j + 1; k < i; ++k) acc = acc + T[k * (TS + 1) + i] * X[j * (TS + 1) + k];
                X[j * (TS + 1) + i] = mk(-acc.re, -acc.im);
            }
        } else {
            // column j of U^{-1}: x_j = 1/u_jj, x_i = -(sum_{k=i+1}^{j} u_ik x_k) / u_ii
            X[j * (TS + 1) + j] = cdiv(mk(R(1), R(0)), T[j * (TS + 1) + j]);
            for (int i = j - 1; i >= 0; --i) {
                cpx<R> acc = czero<R>();
                for (int k = i + 1; k <= j; ++k) acc = acc + T[k * (TS + 1) + i] * X[j * (TS + 1) + k];
                X[j * (TS + 1) + i] = cdiv(mk(-acc.re, -acc.im), T[i * (TS + 1) + i]);
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        int r = e % w, c = e / w;
        a[(long long)(t0 + c) * m + t0 + r] = X[c * (TS + 1) + r];
    }
}

template <class R>
static vie_status lu_factor(vie_pc pc, hipStream_t s) {
    const int m = pc->m, nb = pc->nstored;
    cpx<R> *A = pc->factors.as<cpx<R>>();
    DevBuf ipiv;
    VIE_CHECK(ipiv.ensure(sizeof(int) * (size_t)nb * m));
    VIE_HIP(hipMemsetAsync(pc->info.p, 0, sizeof(int) * nb, s));
    for (int j0 = 0; j0 < m; j0 += LU_NB) {
        int w = std::min(LU_NB, m - j0);
        {
            ProfScope ps("lu_panel", s);
            hipLaunchKernelGGL(k_lu_panel<R>, dim3(nb), dim3(256), 0, s, A, ipiv.as<int>(), pc->info.as<int>(), m,
                               j0, w);
        }
        VIE_HIP(hipGetLastError());
        {
            ProfScope ps("lu_swap_trsm", s);
            hipLaunchKernelGGL(k_lu_swap_trsm<R>, dim3((m + 63) / 64, nb), dim3(256), 0, s, A, ipiv.as<int>(), m,
                               j0, w);
        }
        VIE_HIP(hipGetLastError());
        int rest = m - j0 - w;
        if (rest > 0) {
            int nt = (rest + LU_TILE - 1) / LU_TILE;
            ProfScope ps("lu_update", s);
            hipLaunchKernelGGL(k_lu_update<R>, dim3(nt * nt, nb), dim3(256), 0, s, A, m, j0, w);
            VIE_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_lu_perm, dim3((nb + 63) / 64), dim3(64), 0, s, ipiv.as<int>(), pc->perm.as<int>(), m,
                       nb);
    VIE_HIP(hipGetLastError());
    {
        size_t lds = 2 * sizeof(cpx<R>) * TS * (TS + 1);
        vie_lds_attr((const void *)k_invert_diag<R>, lds);
        ProfScope ps("lu_invert_diag", s);
        hipLaunchKernelGGL(k_invert_diag<R>, dim3((m + TS - 1) / TS, nb), dim3(128), lds, s, A, m);
        VIE_HIP(hipGetLastError());
    }
    VIE_HIP(hipStreamSynchronize(s));
    ipiv.release();
    return VIE_OK;
}

// ---------------------------------------------------------------- apply
// Forward x-DFT of every box line: work[rhs][box][row][k], row = a*by*bz + y + by*z.
template <class R>
__global__ void k_box_fft(const cpx<R> *r, cpx<R> *work, const int *boxes, int nx, int ny, int nz, int by,
                          int bz, int nboxes, FftPlan plan) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int n = plan.L, m = 3 * by * bz;
    long long line = blockIdx.x;  // ((rhs * nboxes + box) * m + row)
    int row = (int)(line % m);
    int box = (int)((line / m) % nboxes);
    long long rhs = line / ((long long)m * nboxes);
    int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = r + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    cpx<R> *res = fft_line<R>(a, plan, false);
    cpx<R> *dst = work + line * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = res[i];
}

// Inverse x-DFT (scaled 1/n) of every box line back into z.
template <class R>
__global__ void k_box_ifft(const cpx<R> *work, cpx<R> *zv, const int *boxes, int nx, int ny, int nz, int by,
                           int bz, int nboxes, FftPlan plan) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int n = plan.L, m = 3 * by * bz;
    long long line = blockIdx.x;
    int row = (int)(line % m);
    int box = (int)((line / m) % nboxes);
    long long rhs = line / ((long long)m * nboxes);
    int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = work + line * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    cpx<R> *res = fft_line<R>(a, plan, true);
    cpx<R> *dst = zv + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    R sc = R(1) / R(n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = sc * res[i];
}

// One workgroup per (box, mode, chunk of RC right-hand sides):
//   z_k = U^{-1} L^{-1} P rhat_k  in place in `work` for RC columns at once.
// Thread t owns rows t, t + 256, ... (QR of them) and keeps their RC accumulators in
// registers.  Forward and backward substitution run over 64-row tiles: the tile's owners
// publish its rows to LDS, four wavefronts apply the pre-inverted diagonal tile (each a
// quarter of its columns), and every thread then applies the tile's column panel to its
// remaining rows.  Each factor entry is read once per chunk and used RC times; the factor
// reads are coalesced along columns.  work element (rhs, box, row i, mode k) sits at
// ((rhs * nboxes + box) * m + i) * n + k.
template <class R, int QR, int RC>
__global__ void __launch_bounds__(256) k_block_solve(cpx<R> *work, const cpx<R> *F, const int *perm,
                                                     const int *block_of_mode, int m, int n, int nboxes, int nrhs) {
    cpx<R> *yt = reinterpret_cast<cpx<R> *>(vie_smem);  // [TS][RC]
    cpx<R> *part = yt + TS * RC;                        // [4][TS][RC]
    const int k = blockIdx.x % n, box = blockIdx.x / n;
    const int r0 = blockIdx.y * RC;
    const int nr = min(RC, nrhs - r0);
    const int sblk = block_of_mode[box * n + k];
    const cpx<R> *A = F + (long long)sblk * m * m;
    const int *pm = perm + (long long)sblk * m;
    const long long rstride = (long long)nboxes * m * n;
    cpx<R> *base = work + (long long)box * m * n + k;
    const int tid = threadIdx.x;
    cpx<R> acc[QR][RC];
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        int i = tid + 256 * q;
#pragma unroll
        for (int c = 0; c < RC; ++c)
            acc[q][c] = (i < m && c < nr) ? base[(r0 + c) * rstride + (long long)pm[i] * n] : czero<R>();
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
                    cpx<R> l = A[(long long)(t0 + cc) * m + t0 + r];
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
                const cpx<R> *col = A + (long long)t0 * m + i;
#pragma unroll 4
                for (int cc = 0; cc < w; ++cc) {
                    cpx<R> l = col[(long long)cc * m];
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
                        cpx<R> u = A[(long long)(t0 + cc) * m + t0 + r];
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
                const cpx<R> *col = A + (long long)t0 * m + i;
#pragma unroll 4
                for (int cc = 0; cc < w; ++cc) {
                    cpx<R> u = col[(long long)cc * m];
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
                if (c < nr) base[(r0 + c) * rstride + (long long)i * n] = acc[q][c];
    }
}

#define VIE_MAX_QR 5
// Columns per chunk: a power of two <= 8, bounded by the register budget of the accumulators.
static int block_solve_rc(int m, int nrhs, size_t esz) {
    int qr = (m + 255) / 256;
    int budget = esz == sizeof(c128) ? 24 : 48;  // complex accumulators per thread
    int rc = 1;
    while (rc < 8 && rc < nrhs && qr * rc * 2 <= budget) rc *= 2;
    return rc;
}

template <class R, int QR, int RC>
static void launch_bs(dim3 grid, size_t lds, hipStream_t s, cpx<R> *work, const cpx<R> *F, const int *perm,
                      const int *bom, int m, int n, int nboxes, int nrhs) {
    hipLaunchKernelGGL((k_block_solve<R, QR, RC>), grid, dim3(256), lds, s, work, F, perm, bom, m, n, nboxes, nrhs);
}

template <class R, int QR>
static void launch_bs_rc(int rc, dim3 grid, size_t lds, hipStream_t s, cpx<R> *work, const cpx<R> *F,
                         const int *perm, const int *bom, int m, int n, int nboxes, int nrhs) {
    switch (rc) {
        case 1: launch_bs<R, QR, 1>(grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        case 2: launch_bs<R, QR, 2>(grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        case 4: launch_bs<R, QR, 4>(grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        default: launch_bs<R, QR, 8>(grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
    }
}

template <class R>
static vie_status launch_block_solve(cpx<R> *work, const cpx<R> *F, const int *perm, const int *bom, int m, int n,
                                     int nboxes, int nrhs, hipStream_t s) {
    const int qr = (m + 255) / 256;
    if (qr > VIE_MAX_QR) {
        vie_set_error("block size above 1280 is not supported by the block solve");
        return VIE_EARG;
    }
    const int rc = block_solve_rc(m, nrhs, sizeof(cpx<R>));
    dim3 grid((unsigned)(nboxes * n), (unsigned)((nrhs + rc - 1) / rc));
    size_t lds = 5 * (size_t)TS * rc * sizeof(cpx<R>);
    switch (qr) {
        case 1: launch_bs_rc<R, 1>(rc, grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        case 2: launch_bs_rc<R, 2>(rc, grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        case 3: launch_bs_rc<R, 3>(rc, grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        case 4: launch_bs_rc<R, 4>(rc, grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
        default: launch_bs_rc<R, 5>(rc, grid, lds, s, work, F, perm, bom, m, n, nboxes, nrhs); break;
    }
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// ---------------------------------------------------------------- host side
template <class R>
static vie_status apply_t(vie_pc pc, const cpx<R> *r, cpx<R> *z, int nrhs, hipStream_t s) {
    vie_op op = pc->op;
    const int m = pc->m, n = pc->bx;
    long long lines = (long long)nrhs * pc->nboxes * m;
    VIE_CHECK(pc->work.ensure(sizeof(cpx<R>) * lines * n));
    if (!pc->covers_all)
        VIE_HIP(hipMemcpyAsync(z, r, sizeof(cpx<R>) * 3 * op->N * nrhs, hipMemcpyDeviceToDevice, s));
    const int *dboxes = reinterpret_cast<const int *>(pc->block_of_mode.as<int>() + pc->nboxes * n);
    int thr;
    size_t lds;
    fft_line_shape(pc->pxb, sizeof(cpx<R>), &thr, &lds);
    cpx<R> *work = pc->work.as<cpx<R>>();
    vie_lds_attr((const void *)k_box_fft<R>, lds);
    vie_lds_attr((const void *)k_box_ifft<R>, lds);
    {
        ProfScope ps("precond_xfft", s);
        hipLaunchKernelGGL(k_box_fft<R>, dim3((unsigned)lines), dim3(thr), lds, s, r, work, dboxes, op->nx, op->ny,
                           op->nz, pc->by, pc->bz, pc->nboxes, pc->pxb);
    }
    VIE_HIP(hipGetLastError());
    {
        ProfScope ps("block_solve", s);
        VIE_CHECK(launch_block_solve<R>(work, pc->factors.as<const cpx<R>>(), pc->perm.as<const int>(),
                                        pc->block_of_mode.as<const int>(), m, n, pc->nboxes, nrhs, s));
    }
    {
        ProfScope ps("precond_ixfft", s);
        hipLaunchKernelGGL(k_box_ifft<R>, dim3((unsigned)lines), dim3(thr), lds, s, work, z, dboxes, op->nx, op->ny,
                           op->nz, pc->by, pc->bz, pc->nboxes, pc->pxb);
    }
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

vie_status pc_apply(vie_pc pc, const void *r, void *z, int nrhs, int prec, hipStream_t s) {
    if (prec != pc->prec) {
        vie_set_error("precond_apply: vector precision must equal the factor precision");
        return VIE_EARG;
    }
    if (prec == VIE_C128) return apply_t<double>(pc, (const c128 *)r, (c128 *)z, nrhs, s);
    return apply_t<float>(pc, (const c64 *)r, (c64 *)z, nrhs, s);
}

// mode of complex values over one box (x fastest); ties -> earliest first occurrence
static c128 box_mode(const std::vector<c128> &M, int nx, int ny, const int *b) {
    std::map<std::pair<double, double>, std::pair<long long, long long>> cnt;  // value -> (count, first)
    long long idx = 0;
    for (int z = 0; z < b[5]; ++z)
        for (int y = 0; y < b[4]; ++y)
            for (int x = 0; x < b[3]; ++x, ++idx) {
                const c128 &v = M[((long long)(b[2] + z) * ny + b[1] + y) * nx + b[0] + x];
                auto key = std::make_pair(v.re, v.im);
                auto it = cnt.find(key);
                if (it == cnt.end())
                    cnt[key] = std::make_pair(1LL, idx);
                else
                    it->second.first++;
            }
    std::pair<double, double> best{0, 0};
    long long bc = -1, bf = 0;
    for (auto &kv : cnt)
        if (kv.second.first > bc || (kv.second.first == bc && kv.second.second < bf)) {
            bc = kv.second.first;
            bf = kv.second.second;
            best = kv.first;
        }
    return mk(best.first, best.second);
}

vie_status pc_build(vie_pc pc, const vie_pc_opts *o, hipStream_t s) {
    vie_op op = pc->op;
    const int nbx = pc->nboxes, n = pc->bx, by = pc->by, bz = pc->bz, m = pc->m;
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1;
    VIE_CHECK(op->fft.get(n, &pc->pxb));
    // boxes on the device (kept after the block map)
    DevBuf dboxes;
    VIE_CHECK(dboxes.ensure(sizeof(int) * 6 * nbx));
    VIE_HIP(hipMemcpyAsync(dboxes.p, pc->boxes.data(), sizeof(int) * 6 * nbx, hipMemcpyHostToDevice, s));
    // homogenised contrast per box
    DevBuf Mt, flag;
    VIE_CHECK(Mt.ensure(sizeof(c128) * (size_t)nbx * by * bz));
    VIE_CHECK(flag.ensure(sizeof(int)));
    VIE_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
    if (o->homog == VIE_HOMOG_MODE) {
        std::vector<c128> Mh(op->N);
        VIE_HIP(hipMemcpyAsync(Mh.data(), op->M64.p, sizeof(c128) * op->N, hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        std::vector<c128> Mth((size_t)nbx * by * bz);
        for (int b = 0; b < nbx; ++b) {
            c128 v = box_mode(Mh, op->nx, op->ny, &pc->boxes[6 * b]);
            for (int i = 0; i < by * bz; ++i) Mth[(size_t)b * by * bz + i] = v;
        }
        VIE_HIP(hipMemcpyAsync(Mt.p, Mth.data(), sizeof(c128) * Mth.size(), hipMemcpyHostToDevice, s));
    } else {
        int tot = nbx * by * bz;
        hipLaunchKernelGGL(k_homog, dim3(tot), dim3(256), 0, s, op->M64.as<const c128>(), Mt.as<c128>(),
                           dboxes.as<const int>(), op->nx, op->ny, by, bz, o->homog, flag.as<int>());
        VIE_HIP(hipGetLastError());
        int hflag = 0;
        VIE_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        if (hflag) {
            vie_set_error("homogenisation NONE needs a contrast that does not vary along x in each box");
            return VIE_EARG;
        }
    }
    // Chan + x-DFT table
    DevBuf Ch;
    VIE_CHECK(Ch.ensure(sizeof(c128) * (size_t)n * 6 * ndy * ndz));
    {
        int thr;
        size_t lds;
        fft_line_shape(pc->pxb, sizeof(c128), &thr, &lds);
        vie_lds_attr((const void *)k_chan_table, lds);
        hipLaunchKernelGGL(k_chan_table, dim3(6 * ndy * ndz), dim3(thr), lds, s, op->gen.as<const c128>(),
                           Ch.as<c128>(), op->nx, op->ny, op->nz, n, by, bz, 1, pc->pxb);
        VIE_HIP(hipGetLastError());
    }
    // memory reduction: proxy v_k of eq. proxy1 read from the table of N (minus the identity)
    std::vector<int> keep(n, 1);
    int centre = (n + 1) / 2 - 1;  // ceil(n/2) - 1
    if (o->reduce) {
        int yp, zp;
        if (o->proxy == 1) {
            yp = (by + 1) / 2 - 1;
            zp = (bz + 1) / 2 - 1;
        } else {
            int col = ((by + 1) / 2) * ((bz + 1) / 2) - 1;
            yp = col % by;
            zp = col / by;
        }
        int iy = 0 - yp + by - 1, iz = 0 - zp + bz - 1;
        std::vector<c128> v(n);
        VIE_HIP(hipMemcpy2DAsync(v.data(), sizeof(c128), Ch.as<c128>() + (long long)iz * ndy + iy,
                                 sizeof(c128) * 6 * ndy * ndz, sizeof(c128), n, hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        if (yp == 0 && zp == 0)
            for (auto &x : v) x.re -= 1.0;
        double vmax = 0;
        for (auto &x : v) vmax = std::max(vmax, std::sqrt(x.re * x.re + x.im * x.im));
        for (int k = 0; k < n; ++k) {
            double vh = vmax > 0 ? std::sqrt(v[k].re * v[k].re + v[k].im * v[k].im) / vmax : 0.0;
            keep[k] = vh > o->reduce_tol;
        }
        keep[centre] = 1;
    }
    // block map: stored blocks ordered (box, mode)
    pc->block_of_mode_host.assign((size_t)nbx * n, -1);
    std::vector<int> smode, sbox;
    for (int b = 0; b < nbx; ++b) {
        int cs = -1;
        for (int k = 0; k < n; ++k)
            if (keep[k]) {
                if (k == centre) cs = (int)smode.size();
                pc->block_of_mode_host[(size_t)b * n + k] = (int)smode.size();
                smode.push_back(k);
                sbox.push_back(b);
            }
        for (int k = 0; k < n; ++k)
            if (!keep[k]) pc->block_of_mode_host[(size_t)b * n + k] = cs;
    }
    pc->nstored = (int)smode.size();
    // device block map followed by the boxes (apply kernels read both)
    VIE_CHECK(pc->block_of_mode.ensure(sizeof(int) * ((size_t)nbx * n + 6 * nbx)));
    VIE_HIP(hipMemcpyAsync(pc->block_of_mode.p, pc->block_of_mode_host.data(), sizeof(int) * (size_t)nbx * n,
                           hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(pc->block_of_mode.as<int>() + (size_t)nbx * n, pc->boxes.data(), sizeof(int) * 6 * nbx,
                           hipMemcpyHostToDevice, s));
    DevBuf dmode, dbox;
    VIE_CHECK(dmode.ensure(sizeof(int) * pc->nstored));
    VIE_CHECK(dbox.ensure(sizeof(int) * pc->nstored));
    VIE_HIP(hipMemcpyAsync(dmode.p, smode.data(), sizeof(int) * pc->nstored, hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(dbox.p, sbox.data(), sizeof(int) * pc->nstored, hipMemcpyHostToDevice, s));
    size_t esz = pc->prec == VIE_C128 ? sizeof(c128) : sizeof(c64);
    VIE_CHECK(pc->factors.ensure(esz * (size_t)pc->nstored * m * m));
    VIE_CHECK(pc->perm.ensure(sizeof(int) * (size_t)pc->nstored * m));
    VIE_CHECK(pc->info.ensure(sizeof(int) * (size_t)pc->nstored));
    dim3 ga((unsigned)(((long long)m * m + 255) / 256), pc->nstored);
    if (pc->prec == VIE_C128)
        hipLaunchKernelGGL(k_assemble<double>, ga, dim3(256), 0, s, Ch.as<const c128>(), Mt.as<const c128>(),
                           dmode.as<const int>(), dbox.as<const int>(), pc->factors.as<c128>(), by, bz);
    else
        hipLaunchKernelGGL(k_assemble<float>, ga, dim3(256), 0, s, Ch.as<const c128>(), Mt.as<const c128>(),
                           dmode.as<const int>(), dbox.as<const int>(), pc->factors.as<c64>(), by, bz);
    VIE_HIP(hipGetLastError());
    VIE_HIP(hipStreamSynchronize(s));
    Ch.release();
    vie_status st = pc->prec == VIE_C128 ? lu_factor<double>(pc, s) : lu_factor<float>(pc, s);
    VIE_CHECK(st);
    std::vector<int> info(pc->nstored);
    VIE_HIP(hipMemcpy(info.data(), pc->info.p, sizeof(int) * pc->nstored, hipMemcpyDeviceToHost));
    for (int i = 0; i < pc->nstored; ++i)
        if (info[i]) {
            vie_set_error("preconditioner block " + std::to_string(i) + " (mode " + std::to_string(smode[i]) +
                          ", box " + std::to_string(sbox[i]) + ") has a zero pivot in column " +
                          std::to_string(info[i] - 1));
            return VIE_ESINGULAR;
        }
    dboxes.release();
    return VIE_OK;
}
