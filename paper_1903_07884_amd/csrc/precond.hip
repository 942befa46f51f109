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
#include <utility>

#include "fft_device.h"
#include "reg_fft.h"

#define LU_NB 32
#define LU_TILE 64
#define LU_MOVES (1 + 4 * LU_NB)      // ints per block of a panel's row-move list
#define SW_CT 32                      // columns per workgroup of the interchange kernel
#define SW_OUT (LU_NB * SW_CT / 256)  // U12 outputs per thread

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
template <int BPT>
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
    c128 *res = fft_line<double, BPT>(a, plan, false);
    const long long stride_k = 6LL * ndz * ndy;
    for (int k = threadIdx.x; k < n; k += blockDim.x) Ch[k * stride_k + (long long)c * ndz * ndy + iz * ndy + iy] = res[k];
}

// 2-level table (Sec. 4, the Chan approximation applied again along y): one workgroup per
// (x-mode k, component c, z offset dz) takes the y-sequence Ch[k][c][dz][dy], dy in (-by, by), of
// the x-level table, T. Chan's circulant of it (length by) and its DFT along y:
//   Ch2[ky*bx + k][c][dz + bz - 1].
__global__ void k_chan_table2(const c128 *Ch, c128 *Ch2, int bx, int by, int bz, FftPlan py) {
    c128 *a = reinterpret_cast<c128 *>(vie_smem), *b = a + py.L;
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1;
    const int iz = blockIdx.x % ndz, c = (blockIdx.x / ndz) % 6, k = blockIdx.x / (6 * ndz);
    const c128 *t = Ch + ((long long)k * 6 + c) * ndz * ndy + (long long)iz * ndy + (by - 1);  // t[dy]
    for (int l = threadIdx.x; l < by; l += blockDim.x) {
        const double w1 = (double)(by - l) / by, w2 = (double)l / by;
        c128 v = t[l];
        v = mk(w1 * v.re, w1 * v.im);
        if (l > 0) v = v + mk(w2 * t[l - by].re, w2 * t[l - by].im);
        a[l] = v;
    }
    __syncthreads();
    LdsLines ln = {1, by, 0, 1, 1};
    c128 *res = by > 1 ? fft_lds<double>(a, b, ln, py, false) : a;
    for (int ky = threadIdx.x; ky < by; ky += blockDim.x)
        Ch2[((long long)ky * bx + k) * 6 * ndz + (long long)c * ndz + iz] = res[ky];
}

// ---------------------------------------------------------------- assembly
// D[s] column-major m x m, s-th stored block (mode ks, box bs), over the cross-section rows
// rows[0..m) (entry a*by*bz + z*by + y).  One workgroup per (AS_COLS columns, block): each
// thread decodes its rows once; a column's decoding is uniform across the workgroup; every
// column is written with coalesced stores.
#define AS_COLS 16
template <class R>
__global__ void __launch_bounds__(256) k_assemble(const c128 *Ch, const c128 *Mt, const int *blk_mode,
                                                  const int *blk_box, const int *rows, cpx<R> *D, int m, int by,
                                                  int bz) {
    const int ndy = 2 * by - 1, ndz = 2 * bz - 1, byz = by * bz;
    const int s = blockIdx.y, c0 = blockIdx.x * AS_COLS;
    const c128 *chk = Ch + (long long)blk_mode[s] * 6 * ndz * ndy;
    const c128 *mtb = Mt + (long long)blk_box[s] * byz;
    cpx<R> *Ds = D + (long long)s * m * m;
    const int cidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    const int cend = min(m, c0 + AS_COLS);
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int r = rows[i];
        const int ar = r / byz, rz = r - ar * byz, zr = rz / by, yr = rz - zr * by;
        const c128 mt = mtb[zr * by + yr];
        for (int ci = c0; ci < cend; ++ci) {
            const int col = rows[ci];
            const int ac = col / byz, cz = col - ac * byz, zc = cz / by, yc = cz - zc * by;
            const c128 ch = chk[cidx[ar][ac] * ndz * ndy + (zr - zc + bz - 1) * ndy + (yr - yc + by - 1)];
            c128 v = mt * ch;
            v = mk(-v.re, -v.im);
            if (r == col) v.re += 1.0;
            Ds[(long long)ci * m + i] = mk((R)v.re, (R)v.im);
        }
    }
}

// 2-level blocks: D[s] column-major (3 bz)^2 for the stored block s of mode pair blk_mode[s]
// (= ky*bx + kx) and box blk_box[s]; row (a, z) = a*bz + z;
//   D[(a,z),(b,z')] = delta - M~(z) Ch2[k2][c(a,b)][z - z' + bz - 1],
// M~ of the box taken at y = 0 (it does not vary along y).
template <class R>
__global__ void k_assemble2(const c128 *Ch2, const c128 *Mt, const int *blk_mode, const int *blk_box, cpx<R> *D,
                            int by, int bz) {
    const int m = 3 * bz, ndz = 2 * bz - 1;
    const int s = blockIdx.y;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)m * m) return;
    const int r = (int)(e % m), col = (int)(e / m);
    const int ar = r / bz, zr = r % bz, ac = col / bz, zc = col % bz;
    const int c = ar == ac ? ar : ar + ac + 2;  // xy -> 3, xz -> 4, yz -> 5
    const c128 ch = Ch2[(long long)blk_mode[s] * 6 * ndz + c * ndz + (zr - zc + bz - 1)];
    const c128 mt = Mt[((long long)blk_box[s] * bz + zr) * by];
    c128 v = mt * ch;
    v = mk(-v.re, -v.im);
    if (r == col) v.re += 1.0;
    D[(long long)s * m * m + e] = mk((R)v.re, (R)v.im);
}

// Round complex float factors to complex bfloat16.
__global__ void k_to_bf16(const c64 *src, bf16c *dst, long long count) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const c64 v = src[i];
    dst[i].v = bf16_bits(v.re) | (bf16_bits(v.im) << 16);
}

// dst[k] = src[k * stride], k < n (one entry of every mode's table, for a contiguous read-back)
__global__ void k_gather_strided(const c128 *src, c128 *dst, int n, long long stride) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k * stride];
}

__global__ void k_narrow_c128(const c128 *src, c64 *dst, long long count) {
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    dst[i] = mk((float)src[i].re, (float)src[i].im);
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

// Register-resident panel (32 G threads, G = 32 or 16 row lanes per column): thread t holds
// column t / G of the panel for the local rows (t % G) + G q, q < QS.  Per column: pivot
// search by the G lanes that hold it (shuffles within the lane group), row interchange through
// LDS, multipliers published to LDS, and the rank-1 update of the remaining panel columns in
// registers.  No global traffic between the panel load and the panel store.  G = 16 halves
// the workgroup so that two blocks share a CU.
template <class R, int QS, int G>
__global__ void __launch_bounds__(32 * G) k_lu_panel_reg(cpx<R> *A, int *ipiv, int *info, int m, int j0, int w) {
    cpx<R> *lcol = reinterpret_cast<cpx<R> *>(vie_smem);  // [m - j0] multipliers of the current column
    __shared__ cpx<R> rj[LU_NB], rp[LU_NB];
    __shared__ int sp;
    __shared__ R spv;
    const int t = threadIdx.x, c = t / G, g = t % G;
    const int mrem = m - j0;
    cpx<R> *a = A + (long long)blockIdx.x * m * m;
    int *piv = ipiv + (long long)blockIdx.x * m;
    cpx<R> v[QS];
#pragma unroll
    for (int q = 0; q < QS; ++q) {
        int li = g + G * q;
        v[q] = (c < w && li < mrem) ? a[(long long)(j0 + c) * m + j0 + li] : czero<R>();
    }
    for (int jj = 0; jj < w; ++jj) {
        if (c == jj) {
            R best = R(-1);
            int bi = jj;
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                int li = g + G * q;
                R val = cabs2(v[q]);
                if (li >= jj && li < mrem && val > best) {
                    best = val;
                    bi = li;
                }
            }
            for (int off = G / 2; off > 0; off >>= 1) {
                R ov = __shfl_xor(best, off);
                int oi = __shfl_xor(bi, off);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            if (g == 0) {
                sp = bi;
                spv = best;
            }
        }
        __syncthreads();
        const int p = sp;
        const R pv = spv;
        if (pv == R(0)) {
            if (t == 0) {
                piv[j0 + jj] = j0 + jj;
                if (info[blockIdx.x] == 0) info[blockIdx.x] = j0 + jj + 1;
            }
            __syncthreads();
            continue;
        }
        // row interchange jj <-> p within the panel
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            int li = g + G * q;
            if (c < w && li == jj) rj[c] = v[q];
            if (c < w && li == p) rp[c] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            int li = g + G * q;
            if (c < w && li == jj) v[q] = rp[c];
            else if (c < w && li == p) v[q] = rj[c];
        }
        // new row jj is rp[]; pivot rp[jj]
        cpx<R> pivv = rp[jj];
        R d = cabs2(pivv);
        cpx<R> inv = mk(pivv.re / d, -pivv.im / d);
        if (c == jj)
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                int li = g + G * q;
                if (li > jj && li < mrem) {
                    v[q] = v[q] * inv;
                    lcol[li] = v[q];
                }
            }
        __syncthreads();
        if (c > jj && c < w) {
            cpx<R> u = rp[c];
#pragma unroll
            for (int q = 0; q < QS; ++q) {
                int li = g + G * q;
                if (li > jj && li < mrem) v[q] = cfms(v[q], lcol[li], u);
            }
        }
        if (t == 0) piv[j0 + jj] = j0 + p;
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < QS; ++q) {
        int li = g + G * q;
        if (c < w && li < mrem) a[(long long)(j0 + c) * m + j0 + li] = v[q];
    }
}

// Row-resident panel: thread t holds the physical panel rows j0 + t + s T (s < RPT, T threads)
// in registers, all LU_NB columns of each, and the logical position pos of each row; a row
// interchange swaps two positions and moves no data.  Per column jj: every row at a position
// >= jj offers |Re a| + |Im a|, a wavefront max-reduction and one LDS pass pick the pivot
// (ties to the smaller position); the pivot row publishes its entries right of jj to LDS and
// takes position jj; every row at a later position forms its multiplier and subtracts its
// multiple of the pivot row (LDS broadcast reads).  Two barriers per column.  Rows are written
// back to their final positions, which performs the panel's interchanges.

// wavefront max-reduction of the ROCm device library (every lane receives the maximum)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

template <class R, int RPT, int MAXT, int NBW, int jj>
__device__ __forceinline__ void panel_rows_column(cpx<R> (&v)[RPT][NBW], int (&pos)[RPT], const int j0, const int w,
                                                  const int mrem, const int t, const int T, const int lane,
                                                  const int wid, const int nw, cpx<R> *rowp, unsigned long long *wkey,
                                                  int *piv, int *info) {
    // pivot key: magnitude |re| + |im| rounded to FP32 in the high word, the complement of the
    // position in the low word, so the largest key is the largest magnitude at the smallest
    // position; rows already pivoted offer 0
    unsigned long long key = 0;
#pragma unroll
    for (int sidx = 0; sidx < RPT; ++sidx) {
        const float mag = (float)(fabs(v[sidx][jj].re) + fabs(v[sidx][jj].im));
        const unsigned long long k = ((unsigned long long)__float_as_uint(mag) << 32) | (0xffffffffu - (unsigned)pos[sidx]);
        if (t + sidx * T < mrem && pos[sidx] >= jj && k > key) key = k;
    }
    key = __ockl_wfred_max_u64(key);
    if (lane == 0) wkey[wid] = key;
    __syncthreads();
    key = wkey[0];
    for (int k = 1; k < nw; ++k) key = max(key, wkey[k]);
    const int pp = (int)(0xffffffffu - (unsigned)key);  // position of the pivot row
    if ((key >> 32) == 0) {  // zero column at and below the diagonal: no interchange, no elimination
        if (t == 0) {
            piv[jj] = j0 + jj;
            if (info[blockIdx.x] == 0) info[blockIdx.x] = j0 + jj + 1;
        }
        __syncthreads();
        return;
    }
#pragma unroll
    for (int sidx = 0; sidx < RPT; ++sidx) {
        if (t + sidx * T >= mrem) continue;
        if (pos[sidx] == pp) {
            // slot jj carries the reciprocal of the pivot, formed once here
            const cpx<R> pv = v[sidx][jj];
            const R rd = R(1) / cabs2(pv);
            rowp[jj] = mk(pv.re * rd, -pv.im * rd);
#pragma unroll
            for (int c = jj + 1; c < NBW; ++c) rowp[c] = v[sidx][c];
            pos[sidx] = jj;
        } else if (pos[sidx] == jj) {
            pos[sidx] = pp;
        }
    }
    __syncthreads();
    const cpx<R> inv = rowp[jj];
#pragma unroll
    for (int sidx = 0; sidx < RPT; ++sidx) {
        if (t + sidx * T < mrem && pos[sidx] > jj) {
            const cpx<R> l = v[sidx][jj] * inv;
            v[sidx][jj] = l;
            // four pivot-row entries at a time, so that the LDS reads are not all hoisted
            // into registers ahead of the products; columns >= w hold zeros and stay zero
#pragma unroll
            for (int c0 = jj + 1; c0 < NBW; c0 += 4) {
#pragma unroll
                for (int c = c0; c < c0 + 4 && c < NBW; ++c) v[sidx][c] = cfms(v[sidx][c], l, rowp[c]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (t == 0) piv[jj] = j0 + pp;
}

template <class R, int RPT, int MAXT, int NBW, int... J>
__device__ __forceinline__ void panel_rows_all(std::integer_sequence<int, J...>, cpx<R> (&v)[RPT][NBW],
                                               int (&pos)[RPT], int j0, int w, int mrem, int t, int T, int lane,
                                               int wid, int nw, cpx<R> *rowp, unsigned long long *wkey, int *piv,
                                               int *info) {
    ((J < w ? panel_rows_column<R, RPT, MAXT, NBW, J>(v, pos, j0, w, mrem, t, T, lane, wid, nw, rowp, wkey, piv, info)
            : void()),
     ...);
}

// NBW: the panel's largest width (w <= NBW columns; NBW < LU_NB for narrower sub-panels whose
// rows would not fit the registers at full width).
template <class R, int RPT, int MAXT, int NBW = LU_NB>
__global__ void __launch_bounds__(MAXT) k_lu_panel_rows(cpx<R> *A, int *ipiv, int *info, int m, int j0, int w,
                                                        int *moves) {
    __shared__ cpx<R> rowp[NBW];
    __shared__ unsigned long long wkey[MAXT / 64];
    __shared__ int nmove;
    const int T = blockDim.x, t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = T >> 6;
    const int mrem = m - j0;
    cpx<R> *a = A + (long long)blockIdx.x * m * m + (long long)j0 * m + j0;
    int *piv = ipiv + (long long)blockIdx.x * m + j0;
    cpx<R> v[RPT][NBW];
    int pos[RPT];
    // column bases are uniform, row offsets 32-bit: scalar-base addressing, no per-lane 64-bit
    // addresses kept live
#pragma unroll
    for (int sidx = 0; sidx < RPT; ++sidx) {
        const int row = t + sidx * T;
        pos[sidx] = row;
#pragma unroll
        for (int c = 0; c < NBW; ++c) {
            const cpx<R> *col = a + c * m;
            v[sidx][c] = (c < w && row < mrem) ? col[row] : czero<R>();
        }
    }
    if (t == 0) nmove = 0;
    panel_rows_all<R, RPT, MAXT, NBW>(std::make_integer_sequence<int, NBW>{}, v, pos, j0, w, mrem, t, T, lane, wid,
                                      nw, rowp, wkey, piv, info);
    // the panel's row moves for the other columns: (destination, source) of every row that
    // changed position, at most 2 NBW of them
    int *mv = moves + (long long)blockIdx.x * LU_MOVES;
#pragma unroll
    for (int sidx = 0; sidx < RPT; ++sidx) {
        const int row = t + sidx * T;
        if (row < mrem) {
#pragma unroll
            for (int c = 0; c < NBW; ++c) {
                cpx<R> *col = a + c * m;
                if (c < w) col[pos[sidx]] = v[sidx][c];
            }
            if (pos[sidx] != row) {
                const int k = atomicAdd(&nmove, 1);
                mv[1 + 2 * k] = j0 + pos[sidx];
                mv[2 + 2 * k] = j0 + row;
            }
        }
    }
    __syncthreads();
    if (t == 0) mv[0] = nmove;
}

// Row moves of the panel [j0, j0 + w) from its interchanges, for the panel kernels that do not
// emit them: one thread per block replays the interchanges on the rows they touch.
// moves[block] = {count, (destination, source) x count}.
__global__ void __launch_bounds__(64) k_lu_moves(const int *ipiv, int *moves, int m, int j0, int w, int nblk) {
    __shared__ int2 ent[64][2 * LU_NB];  // (position, source row) of the touched positions
    const int b = blockIdx.x * 64 + threadIdx.x;
    if (b >= nblk) return;
    const int *piv = ipiv + (long long)b * m;
    int2 *e = ent[threadIdx.x];
    int n = 0;
    auto find = [&](int p) {
        for (int i = 0; i < n; ++i)
            if (e[i].x == p) return i;
        e[n] = make_int2(p, p);
        return n++;
    };
    for (int j = 0; j < w; ++j) {
        const int p = piv[j0 + j];
        if (p == j0 + j) continue;
        const int ia = find(j0 + j), ib = find(p);
        const int t = e[ia].y;
        e[ia].y = e[ib].y;
        e[ib].y = t;
    }
    int *mv = moves + (long long)b * LU_MOVES;
    int k = 0;
    for (int i = 0; i < n; ++i)
        if (e[i].x != e[i].y) {
            mv[1 + 2 * k] = e[i].x;
            mv[2 + 2 * k] = e[i].y;
            ++k;
        }
    mv[0] = k;
}

// The panel [j0, j0 + w)'s row moves applied to the columns [cfirst, m) outside the panel
// (do_swap), and U12 = L11^{-1} A12 for the columns right of it (do_trsm, with L11^{-1} from
// k_lu_linv).  One workgroup per (SW_CT-column tile, block): the old values of the moved rows
// are gathered into registers, rows [j0, j0 + w) of the tile are staged in LDS with coalesced
// loads; after a barrier the moved values land in LDS (panel rows) or in place (rows below),
// the triangular product runs on the LDS rows, which are written back coalesced.
template <class R>
__global__ void __launch_bounds__(256) k_lu_swap_trsm(cpx<R> *A, const int *moves, const cpx<R> *Linv, int m, int j0,
                                                      int w, int cfirst, int do_swap, int do_trsm) {
    __shared__ cpx<R> Tp[LU_NB][SW_CT + 1];  // rows j0 + r of the tile
    __shared__ cpx<R> Li[LU_NB][LU_NB + 1];
    __shared__ int2 mvs[LU_MOVES / 2];
    __shared__ int nmv;
    const int c0 = cfirst + blockIdx.x * SW_CT;
    cpx<R> *a = A + (long long)blockIdx.y * m * m;
    if (do_swap) {
        const int *mv = moves + (long long)blockIdx.y * LU_MOVES;
        if (threadIdx.x == 0) nmv = mv[0];
        for (int k = threadIdx.x; k < LU_MOVES / 2; k += blockDim.x) mvs[k] = make_int2(mv[1 + 2 * k], mv[2 + 2 * k]);
    } else if (threadIdx.x == 0) {
        nmv = 0;
    }
    const bool right = do_trsm && c0 + SW_CT > j0 + w;
    for (int e = threadIdx.x; e < w * SW_CT; e += blockDim.x) {
        const int r = e % w, c = e / w, col = c0 + c;
        const bool live = col < m && !(col >= j0 && col < j0 + w);
        Tp[r][c] = live ? a[(long long)col * m + j0 + r] : czero<R>();
    }
    if (right) {
        const cpx<R> *li = Linv + (long long)blockIdx.y * LU_NB * LU_NB;
        for (int e = threadIdx.x; e < LU_NB * LU_NB; e += blockDim.x) Li[e / LU_NB][e % LU_NB] = li[e];
    }
    __syncthreads();
    const int nm = nmv;
    // gather: element (move k, column c) -> thread; at most LU_MOVES / 2 * SW_CT / 256 each
    constexpr int GPT = (LU_MOVES / 2) * SW_CT / 256;
    cpx<R> gv[GPT];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
        const int e = threadIdx.x + 256 * u, k = e / SW_CT, c = e % SW_CT, col = c0 + c;
        const bool live = k < nm && col < m && !(col >= j0 && col < j0 + w);
        gv[u] = live ? a[(long long)col * m + mvs[k].y] : czero<R>();
    }
    __syncthreads();  // every old value is read before any is replaced
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
        const int e = threadIdx.x + 256 * u, k = e / SW_CT, c = e % SW_CT, col = c0 + c;
        if (k < nm && col < m && !(col >= j0 && col < j0 + w)) {
            const int dst = mvs[k].x;
            if (dst < j0 + w) Tp[dst - j0][c] = gv[u];
            else a[(long long)col * m + dst] = gv[u];
        }
    }
    __syncthreads();
    if (right) {
        cpx<R> outv[SW_OUT];
        const int cc = threadIdx.x % SW_CT, rq = threadIdx.x / SW_CT;
        const int cl = c0 + cc;
#pragma unroll
        for (int k = 0; k < SW_OUT; ++k) {
            int r = rq + (256 / SW_CT) * k;
            cpx<R> acc = czero<R>();
            if (r < w) {
                acc = Tp[r][cc];
                for (int q = 0; q < r; ++q) acc = acc + Li[r][q] * Tp[q][cc];
            }
            outv[k] = acc;
        }
        __syncthreads();
        if (cl >= j0 + w && cl < m)
#pragma unroll
            for (int k = 0; k < SW_OUT; ++k) {
                int r = rq + (256 / SW_CT) * k;
                if (r < w) Tp[r][cc] = outv[k];
            }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < w * SW_CT; e += blockDim.x) {
        const int r = e % w, c = e / w, col = c0 + c;
        if (col < m && !(col >= j0 && col < j0 + w)) a[(long long)col * m + j0 + r] = Tp[r][c];
    }
}

// Marks the entries [q0, H) of a register column as computed here: the compiler then finishes
// a substitution row before starting the next, instead of interleaving rows and holding the
// factor entries of many rows in registers.  Emits no instruction.
template <class R, int H>
__device__ __forceinline__ void settle(cpx<R> (&x)[H], int q0) {
#pragma unroll
    for (int q = 0; q < H; ++q)
        if (q >= q0) asm volatile("" : "+v"(x[q].re), "+v"(x[q].im));
}

// L11^{-1} of the panel [j0, j0 + w) (unit lower, strictly lower part stored) into Linv[block]
// (row-major LU_NB x LU_NB, strictly lower part; zero diagonal and above).  One workgroup per
// block; lane jc forms column jc of the inverse in registers by forward substitution with L11
// read as LDS broadcasts, one row at a time (settled).
template <class R>
__global__ void __launch_bounds__(64) k_lu_linv(const cpx<R> *A, cpx<R> *Linv, int m, int j0, int w) {
    __shared__ cpx<R> L[LU_NB][LU_NB + 1];  // L[r][c], zero past w
    const cpx<R> *a = A + (long long)blockIdx.x * m * m;
    for (int e = threadIdx.x; e < LU_NB * LU_NB; e += blockDim.x) {
        const int r = e % LU_NB, c = e / LU_NB;
        L[r][c] = (r < w && c < w) ? a[(long long)(j0 + c) * m + j0 + r] : czero<R>();
    }
    __syncthreads();
    const int jc = threadIdx.x;
    if (jc >= LU_NB) return;
    cpx<R> x[LU_NB];
#pragma unroll
    for (int q = 0; q < LU_NB; ++q) x[q] = mk(q == jc ? R(1) : R(0), R(0));
#pragma unroll
    for (int k = 0; k < LU_NB; ++k) {
#pragma unroll
        for (int q = k + 1; q < LU_NB; ++q) x[q] = cfms(x[q], L[q][k], x[k]);
        settle(x, k + 1);
    }
    cpx<R> *out = Linv + (long long)blockIdx.x * LU_NB * LU_NB;
#pragma unroll
    for (int q = 0; q < LU_NB; ++q) out[q * LU_NB + jc] = q > jc ? x[q] : czero<R>();
}


// A[r, c] -= sum_{k in [k0, k0 + K)} A[r, k] A[k, c] for r in [r0, r1), c in [c0, c1): one
// 64x64 output tile per workgroup, K staged in LDS in chunks of LU_NB, products on the matrix
// cores.  Complex products as real ones: a K-step takes two complex columns of L as four
// real ones (lane l: row l%16, real index l/16 = 2 x complex column + part); with U fed as
// interleaved (Re, Im), the left operand (Re l, -Im l) accumulates Re(l u) and (Im l, Re l)
// accumulates Im(l u).  Each of the 4 wavefronts owns a 32x32 quarter (2x2 tiles of 16x16).
template <class R>
struct LuMfma;
template <>
struct LuMfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 fma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator register v of lane l holds row 4 v + l/16 (FP64) / 4 (l/16) + v (FP32)
    static __device__ __forceinline__ int acc_row(int q, int v) { return 4 * v + q; }
};
template <>
struct LuMfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 fma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int acc_row(int q, int v) { return 4 * q + v; }
};

// Three wavefronts per SIMD (at most 168 registers): measured 10% faster in FP64 than the two
// that the unconstrained allocation gives (four spill).  The register prefetch of the next K
// chunk pays in both precisions (FP32: 7% at 1024 blocks of 768).
template <class R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_lu_update(cpx<R> *A, int m, int r0, int r1, int c0, int c1, int k0, int K) {
    typedef typename LuMfma<R>::v4 v4;
    constexpr int KCH = sizeof(R) == 8 ? 16 : 32;  // K chunk: 32 KB of LDS either way (4 workgroups per CU)
    __shared__ cpx<R> Ls[KCH][LU_TILE];  // [k][row]
    __shared__ cpx<R> Us[KCH][LU_TILE];  // [k][col]
    const int nt = (r1 - r0 + LU_TILE - 1) / LU_TILE;
    const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;
    const int rr0 = r0 + ti * LU_TILE, cc0 = c0 + tj * LU_TILE;
    cpx<R> *a = A + (long long)blockIdx.y * m * m;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, q = lane >> 4, kh = q >> 1, p = q & 1;
    const int wrow = 32 * (wv & 1), wcol = 32 * (wv >> 1);
    // accumulators start from the output tile (loaded first, in flight during the staging)
    v4 cr[2][2], ci[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = cc0 + wcol + 16 * j + r;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rr0 + wrow + 16 * i + LuMfma<R>::acc_row(q, v);
                const cpx<R> x = (row < r1 && c < c1) ? a[(long long)c * m + row] : czero<R>();
                cr[i][j][v] = x.re;
                ci[i][j][v] = x.im;
            }
    }
    // the next K chunk of L and U is loaded into registers while the current one is multiplied
    constexpr int SPT = KCH * LU_TILE / 256;  // elements of each of L and U per thread and chunk
    cpx<R> lreg[SPT], ureg[SPT];
    auto load_chunk = [&](int kc) {
        const int kw = min(KCH, K - kc);
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + 256 * u;
            const int kl = e / LU_TILE, i = e % LU_TILE;  // L: rows contiguous
            lreg[u] = (kl < kw && rr0 + i < r1) ? a[(long long)(k0 + kc + kl) * m + rr0 + i] : czero<R>();
            const int ku = e % KCH, j = e / KCH;          // U: k contiguous within a column
            ureg[u] = (ku < kw && cc0 + j < c1) ? a[(long long)(cc0 + j) * m + k0 + kc + ku] : czero<R>();
        }
    };
    load_chunk(0);
    for (int kc = 0; kc < K; kc += KCH) {
        const int kw = min(KCH, K - kc);
        __syncthreads();  // the previous chunk's products are done with the LDS
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + 256 * u;
            Ls[e / LU_TILE][e % LU_TILE] = lreg[u];
            Us[e % KCH][e / KCH] = ureg[u];
        }
        __syncthreads();
        if (kc + KCH < K) load_chunk(kc + KCH);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
        for (int ks = 0; ks < (kw + 1) / 2; ++ks) {
            const int k = 2 * ks + kh;  // < KCH (zero-padded past kw)
            R ar[2], ai[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const cpx<R> l = Ls[k][wrow + 16 * i + r];
                ar[i] = p ? l.im : -l.re;   // negated: the accumulators subtract
                ai[i] = p ? -l.re : -l.im;
                const cpx<R> u = Us[k][wcol + 16 * i + r];
                bv[i] = p ? u.im : u.re;
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = LuMfma<R>::fma(ar[i], bv[j], cr[i][j]);
                    ci[i][j] = LuMfma<R>::fma(ai[i], bv[j], ci[i][j]);
                }
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = cc0 + wcol + 16 * j + r;
        if (c >= c1) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rr0 + wrow + 16 * i + LuMfma<R>::acc_row(q, v);
                if (row < r1) a[(long long)c * m + row] = mk(cr[i][j][v], ci[i][j][v]);
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
// One workgroup (four wavefronts) per (tile, block), the tile in LDS (column-major, padded
// to the identity past the block's order).  Lane j of a wavefront owns column j of one half
// (rows 0..31 or 32..63) of an inverse in registers and forms it by substitution, one row at
// a time, with the factor entries read as LDS broadcasts:
//   phase 1: wave 0 the L^{-1} rows 0..31 (forward), wave 3 the U^{-1} rows 32..63 (backward);
//   phase 2: wave 1 the L^{-1} rows 32..63 (the product with rows 0..31, then forward),
//            wave 2 the U^{-1} rows 0..31 (the product with rows 32..63, then backward).
// Each wavefront writes its results over the entries that it alone still reads, after its
// reads (L^{-1} over the strictly lower part, U^{-1} over the upper part).
template <class R>
__global__ void __launch_bounds__(256) k_invert_diag(cpx<R> *F, int m) {
    cpx<R> *T = reinterpret_cast<cpx<R> *>(vie_smem);  // column-major [TS][TS+1]: T[c*(TS+1)+r]
    __shared__ cpx<R> dinv[TS];
    constexpr int H = TS / 2;
    const int t0 = blockIdx.x * TS;
    const int w = min(TS, m - t0);
    cpx<R> *a = F + (long long)blockIdx.y * m * m;
    for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
        const int r = e % TS, c = e / TS;
        cpx<R> v = mk(r == c ? R(1) : R(0), R(0));
        if (r < w && c < w) v = a[(long long)(t0 + c) * m + t0 + r];
        T[c * (TS + 1) + r] = v;
    }
    __syncthreads();
    if (threadIdx.x < TS) dinv[threadIdx.x] = cdiv(mk(R(1), R(0)), T[threadIdx.x * (TS + 1) + threadIdx.x]);
    __syncthreads();
    // the role of a wavefront as a uniform value: whole wavefronts branch
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), j = threadIdx.x & 63;
    cpx<R> *Tj = T + j * (TS + 1);
    cpx<R> x[H];
    if (wv == 0) {  // L^{-1}, rows 0..31 of column j
#pragma unroll
        for (int q = 0; q < H; ++q) x[q] = mk(q == j ? R(1) : R(0), R(0));
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cpx<R> *Lk = T + k * (TS + 1);
#pragma unroll
            for (int q = k + 1; q < H; ++q) x[q] = cfms(x[q], Lk[q], x[k]);
            settle(x, k + 1);
        }
#pragma unroll
        for (int q = 0; q < H; ++q)
            if (q > j) Tj[q] = x[q];
    } else if (wv == 3) {  // U^{-1}, rows 32..63 of column j
#pragma unroll
        for (int q = 0; q < H; ++q) x[q] = mk(H + q == j ? R(1) : R(0), R(0));
#pragma unroll
        for (int k = H - 1; k >= 0; --k) {
            x[k] = x[k] * dinv[H + k];
            const cpx<R> *Uk = T + (H + k) * (TS + 1) + H;
#pragma unroll
            for (int q = 0; q < k; ++q) x[q] = cfms(x[q], Uk[q], x[k]);
            settle(x, 0);
        }
#pragma unroll
        for (int q = 0; q < H; ++q)
            if (H + q <= j) Tj[H + q] = x[q];
    }
    __syncthreads();
    if (wv == 1) {  // L^{-1}, rows 32..63 of column j
#pragma unroll
        for (int q = 0; q < H; ++q) x[q] = mk(H + q == j ? R(1) : R(0), R(0));
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cpx<R> t = Tj[k];  // L^{-1}[k][j] from phase 1: unit diagonal, zero above
            const cpx<R> xk = mk(k > j ? t.re : (k == j ? R(1) : R(0)), k > j ? t.im : R(0));
            const cpx<R> *Lk = T + k * (TS + 1) + H;
#pragma unroll
            for (int q = 0; q < H; ++q) x[q] = cfms(x[q], Lk[q], xk);
            settle(x, 0);
        }
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cpx<R> *Lk = T + (H + k) * (TS + 1) + H;
#pragma unroll
            for (int q = k + 1; q < H; ++q) x[q] = cfms(x[q], Lk[q], x[k]);
            settle(x, k + 1);
        }
#pragma unroll
        for (int q = 0; q < H; ++q)
            if (H + q > j) Tj[H + q] = x[q];
    } else if (wv == 2) {  // U^{-1}, rows 0..31 of column j
#pragma unroll
        for (int q = 0; q < H; ++q) x[q] = mk(q == j ? R(1) : R(0), R(0));
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cpx<R> t = Tj[H + k];  // U^{-1}[32 + k][j] from phase 1: zero below the diagonal
            const cpx<R> yk = mk(H + k <= j ? t.re : R(0), H + k <= j ? t.im : R(0));
            const cpx<R> *Uk = T + (H + k) * (TS + 1);
#pragma unroll
            for (int q = 0; q < H; ++q) x[q] = cfms(x[q], Uk[q], yk);
            settle(x, 0);
        }
#pragma unroll
        for (int k = H - 1; k >= 0; --k) {
            x[k] = x[k] * dinv[k];
            const cpx<R> *Uk = T + k * (TS + 1);
#pragma unroll
            for (int q = 0; q < k; ++q) x[q] = cfms(x[q], Uk[q], x[k]);
            settle(x, 0);
        }
#pragma unroll
        for (int q = 0; q < H; ++q)
            if (q <= j) Tj[q] = x[q];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        int r = e % w, c = e / w;
        a[(long long)(t0 + c) * m + t0 + r] = T[c * (TS + 1) + r];
    }
}

template <class R>
static cpx<R> *A_of(vie_pc pc) { return pc->factors.as<cpx<R>>(); }

// Width of the LU sub-panel starting with mrem rows: `pref` (LU_NB or LU_NB / 2; autotuned),
// and LU_NB / 2 for FP64 panels of 513-768 rows, which one thread per row holds in registers
// only at half width (768 threads leave 170 VGPRs each: 32 complex doubles per row spilled,
// 16 fit).
template <class R>
static int lu_sub_width(int mrem, int pref) {
    return (sizeof(R) == 8 && mrem > 512 && mrem <= 768) ? LU_NB / 2 : pref;
}

// LU with partial pivoting of nb column-major m x m blocks A (in place), all launches on
// stream `s`; ns = sub-panels of LU_NB columns per macro panel.  ipiv (nb x m), linv
// (nb x LU_NB^2) and moves (nb x LU_MOVES) are scratch; info[b] is set nonzero for a
// singular block.
template <class R>
static vie_status lu_factor_blocks(int m, int nb, cpx<R> *A, int *ipiv, cpx<R> *linv, int *moves, int *info,
                                   int ns, int wsub, hipStream_t s) {
    auto panel = [&](int j0, int w) -> vie_status {
        ProfScope ps("lu_panel", s);
        const int mrem = m - j0;
        // row-resident panel while the rows fit the registers of one workgroup
        if constexpr (sizeof(R) == 8) {
            if (mrem <= 768 && w <= LU_NB / 2) {  // half-width sub-panels (lu_sub_width)
                hipLaunchKernelGGL((k_lu_panel_rows<R, 1, 768, LU_NB / 2>), dim3(nb), dim3((mrem + 63) / 64 * 64), 0, s,
                                   A, ipiv, info, m, j0, w, moves);
                VIE_HIP(hipGetLastError());
                return VIE_OK;
            }
            if (mrem <= 512) {
                hipLaunchKernelGGL((k_lu_panel_rows<R, 1, 512>), dim3(nb), dim3((mrem + 63) / 64 * 64), 0, s, A, ipiv,
                                   info, m, j0, w, moves);
                VIE_HIP(hipGetLastError());
                return VIE_OK;
            }
        } else {
            if (mrem <= 1024 && w <= LU_NB / 2) {
                hipLaunchKernelGGL((k_lu_panel_rows<R, 1, 1024, LU_NB / 2>), dim3(nb), dim3((mrem + 63) / 64 * 64), 0,
                                   s, A, ipiv, info, m, j0, w, moves);
                VIE_HIP(hipGetLastError());
                return VIE_OK;
            }
            if (mrem <= 1024) {
                hipLaunchKernelGGL((k_lu_panel_rows<R, 1, 1024>), dim3(nb), dim3((mrem + 63) / 64 * 64), 0, s, A, ipiv,
                                   info, m, j0, w, moves);
                VIE_HIP(hipGetLastError());
                return VIE_OK;
            }
        }
        // 16 row lanes (512 threads) when the panel takes <= 32 value VGPRs per thread that
        // way (two blocks per CU), else 32 (1024 threads, one block per CU)
        const int q16 = (m - j0 + 15) / 16;
        const bool half = q16 * sizeof(cpx<R>) / 4 <= 32;
        int qs = half ? q16 : (m - j0 + 31) / 32;
        size_t lds = sizeof(cpx<R>) * (size_t)(m - j0);
        bool regs = qs * sizeof(cpx<R>) / 4 <= 96;  // accumulator VGPRs per thread
#define PANEL_CASE(QV)                                                                                     \
    if (qs <= QV) {                                                                                        \
        if (half)                                                                                          \
            hipLaunchKernelGGL((k_lu_panel_reg<R, QV, 16>), dim3(nb), dim3(512), lds, s, A, ipiv, info, m, j0, \
                               w);                                                                         \
        else                                                                                               \
            hipLaunchKernelGGL((k_lu_panel_reg<R, QV, 32>), dim3(nb), dim3(1024), lds, s, A, ipiv, info, m, j0, \
                               w);                                                                         \
    } else
        if (regs) {
            PANEL_CASE(2) PANEL_CASE(4) PANEL_CASE(8) PANEL_CASE(12) PANEL_CASE(16) PANEL_CASE(24)
            PANEL_CASE(32) PANEL_CASE(40) {
                hipLaunchKernelGGL(k_lu_panel<R>, dim3(nb), dim3(256), 0, s, A, ipiv, info, m, j0, w);
            }
        } else {
            hipLaunchKernelGGL(k_lu_panel<R>, dim3(nb), dim3(256), 0, s, A, ipiv, info, m, j0, w);
        }
#undef PANEL_CASE
        VIE_HIP(hipGetLastError());
        // these panel kernels leave the row-move list to a replay of their interchanges
        hipLaunchKernelGGL(k_lu_moves, dim3((nb + 63) / 64), dim3(64), 0, s, (const int *)ipiv, moves, m, j0, w, nb);
        VIE_HIP(hipGetLastError());
        return VIE_OK;
    };
    auto swap_trsm = [&](int j0, int w, int do_swap, int do_trsm) -> vie_status {
        ProfScope ps("lu_swap_trsm", s);
        if (do_trsm) {
            hipLaunchKernelGGL(k_lu_linv<R>, dim3(nb), dim3(64), 0, s, (const cpx<R> *)A, linv, m, j0, w);
            VIE_HIP(hipGetLastError());
        }
        // interchanges reach every column; the triangular product alone only those right of the panel
        const int cfirst = do_swap ? 0 : j0 + w;
        if (cfirst >= m) return VIE_OK;
        hipLaunchKernelGGL(k_lu_swap_trsm<R>, dim3((m - cfirst + SW_CT - 1) / SW_CT, nb), dim3(256), 0, s, A,
                           (const int *)moves, (const cpx<R> *)linv, m, j0, w, cfirst, do_swap, do_trsm);
        VIE_HIP(hipGetLastError());
        return VIE_OK;
    };
    auto update = [&](int r0, int r1, int c0, int c1, int k0, int K) -> vie_status {
        if (r1 <= r0 || c1 <= c0 || K <= 0) return VIE_OK;
        ProfScope ps("lu_update", s);
        int ntr = (r1 - r0 + LU_TILE - 1) / LU_TILE, ntc = (c1 - c0 + LU_TILE - 1) / LU_TILE;
        hipLaunchKernelGGL(k_lu_update<R>, dim3(ntr * ntc, nb), dim3(256), 0, s, A, m, r0, r1, c0, c1, k0, K);
        VIE_HIP(hipGetLastError());
        return VIE_OK;
    };
    // Two-level right-looking LU: macro panels of ns LU_NB columns, factored as sub-panels of
    // lu_sub_width columns (LU_NB, or half that for large FP64 panels).  Each
    // sub-panel first takes the updates of the earlier sub-panels of its macro panel (its
    // columns from row jr down), is factored, has its interchanges applied everywhere, and its
    // rows right of it take the same updates before the U12 solve; the trailing matrix is
    // updated once per macro panel, with K = the macro panel's width.
    for (int J0 = 0; J0 < m;) {
        const int jend = std::min(m, J0 + ns * LU_NB);
        for (int jr = J0, w = 0; jr < jend; jr += w) {
            w = std::min(lu_sub_width<R>(m - jr, wsub), jend - jr);
            if (jr == J0) {
                VIE_CHECK(panel(jr, w));
                VIE_CHECK(swap_trsm(jr, w, 1, 1));
            } else {
                VIE_CHECK(update(jr, m, jr, jr + w, J0, jr - J0));       // its columns
                VIE_CHECK(panel(jr, w));
                VIE_CHECK(swap_trsm(jr, w, 1, 0));                      // its interchanges everywhere
                VIE_CHECK(update(jr, jr + w, jr + w, m, J0, jr - J0));   // its rows, right of it
                VIE_CHECK(swap_trsm(jr, w, 0, 1));                      // its U12
            }
        }
        VIE_CHECK(update(jend, m, jend, m, J0, jend - J0));             // trailing matrix
        J0 = jend;
    }
    return VIE_OK;
}

// Macro-panel and sub-panel shape of the batched LU: the default, or with autotuning the
// fastest of {1, 2, 4, 8} sub-panels per macro panel x sub-panel width {LU_NB, LU_NB / 2},
// timed on a copy of the first min(nb, 256) blocks (one block per compute unit, the LU's own
// launch shape), cached per (precision, m, block count).  Measured default: FP32 gains from
// wider macro panels (fewer passes over the trailing matrix; 4 sub-panels: -13% update time
// at 1024 blocks of 768), FP64 does not (2: the matrix-core time dominates).
template <class R>
static vie_status lu_macro_panels(vie_pc pc, int *ipiv, cpx<R> *linv, int *moves, hipStream_t s, int *ns_out,
                                  int *w_out) {
    const int m = pc->m, nb = pc->nstored;
    int ns = sizeof(R) == 8 ? 2 : 4, wsub = LU_NB;
    if (tune_enabled() && m > LU_NB) {
        char key[128];
        snprintf(key, sizeof key, "lu_factor real=%d m=%d blocks=%d", (int)sizeof(R) * 8, m, nb);
        std::vector<std::vector<int>> cands;
        for (int c : {1, 2, 4, 8})
            if ((c - 1) * LU_NB < m)
                for (int wc : {LU_NB, LU_NB / 2}) cands.push_back({c, wc});
        std::vector<int> choice;
        if (tune_lookup(key, &choice)) {
            VIE_CHECK(tune_check_choice(key, choice, cands));
            ns = choice[0];
            wsub = choice[1];
        } else {
            const int sample = std::min(nb, 256);
            const size_t bytes = sizeof(cpx<R>) * (size_t)sample * m * m;
            DevBuf copy, info;
            VIE_CHECK(copy.ensure(bytes));
            VIE_CHECK(info.ensure(sizeof(int) * (size_t)sample));
            double best = 1e300;
            for (auto &cv : cands) {
                double ms = 0;
                VIE_CHECK(tune_time(s, 1, [&]() -> vie_status {
                    VIE_HIP(hipMemcpyAsync(copy.p, pc->factors.p, bytes, hipMemcpyDeviceToDevice, s));
                    VIE_HIP(hipMemsetAsync(info.p, 0, sizeof(int) * (size_t)sample, s));
                    return lu_factor_blocks<R>(m, sample, copy.as<cpx<R>>(), ipiv, linv, moves, info.as<int>(), cv[0],
                                               cv[1], s);
                }, &ms));
                if (ms < best) best = ms, ns = cv[0], wsub = cv[1];
            }
            tune_store(key, {ns, wsub}, best, (int)cands.size());
        }
    }
    *ns_out = ns;
    *w_out = wsub;
    return VIE_OK;
}

// Batched LU of every stored block.
template <class R>
static vie_status lu_factor(vie_pc pc, hipStream_t s) {
    const int m = pc->m, nb = pc->nstored;
    DevBuf ipiv, linv, moves;
    VIE_CHECK(ipiv.ensure(sizeof(int) * (size_t)nb * m));
    VIE_CHECK(linv.ensure(sizeof(cpx<R>) * (size_t)nb * LU_NB * LU_NB));
    VIE_CHECK(moves.ensure(sizeof(int) * (size_t)nb * LU_MOVES));
    int ns = 0, wsub = 0;
    VIE_CHECK(lu_macro_panels<R>(pc, ipiv.as<int>(), linv.as<cpx<R>>(), moves.as<int>(), s, &ns, &wsub));
    VIE_HIP(hipMemsetAsync(pc->info.p, 0, sizeof(int) * nb, s));
    VIE_CHECK(lu_factor_blocks<R>(m, nb, A_of<R>(pc), ipiv.as<int>(), linv.as<cpx<R>>(), moves.as<int>(),
                                  pc->info.as<int>(), ns, wsub, s));
    hipLaunchKernelGGL(k_lu_perm, dim3((nb + 63) / 64), dim3(64), 0, s, ipiv.as<int>(), pc->perm.as<int>(), m,
                       nb);
    VIE_HIP(hipGetLastError());
    {
        size_t lds = sizeof(cpx<R>) * TS * (TS + 1);
        vie_lds_attr((const void *)k_invert_diag<R>, lds);
        ProfScope ps("lu_invert_diag", s);
        hipLaunchKernelGGL(k_invert_diag<R>, dim3((m + TS - 1) / TS, nb), dim3(256), lds, s, A_of<R>(pc), m);
        VIE_HIP(hipGetLastError());
    }
    VIE_HIP(hipStreamSynchronize(s));
    ipiv.release();
    return VIE_OK;
}

// ---------------------------------------------------------------- apply
// Forward x-DFT of the box lines of `mr` cross-section rows rows[0..mr):
// work[rhs][box][i][k] holds line rows[i].  With a gate, the whole launch is skipped unless
// *gate == epoch (the identity rows of this apply held input).
template <class R, int BPT>
__global__ void k_box_fft(const cpx<R> *r, cpx<R> *work, const int *boxes, const int *rows, int mr, int nx,
                          int ny, int nz, int by, int bz, int nboxes, FftPlan plan, const uint32_t *gate,
                          uint32_t epoch) {
    if (gate && *gate != epoch) return;
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int n = plan.L;
    long long line = blockIdx.x;  // ((rhs * nboxes + box) * mr + i)
    int row = rows[(int)(line % mr)];
    int box = (int)((line / mr) % nboxes);
    long long rhs = line / ((long long)mr * nboxes);
    int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = r + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, plan, false);
    cpx<R> *dst = work + line * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = res[i];
}

// Inverse x-DFT (scaled 1/n) of the solved lines back into z.
template <class R, int BPT>
__global__ void k_box_ifft(const cpx<R> *work, cpx<R> *zv, const int *boxes, const int *rows, int mr, int nx,
                           int ny, int nz, int by, int bz, int nboxes, FftPlan plan) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem);
    const int n = plan.L;
    long long line = blockIdx.x;
    int row = rows[(int)(line % mr)];
    int box = (int)((line / mr) % nboxes);
    long long rhs = line / ((long long)mr * nboxes);
    int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = work + line * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = src[i];
    __syncthreads();
    cpx<R> *res = fft_line<R, BPT>(a, plan, true);
    cpx<R> *dst = zv + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    R sc = R(1) / R(n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = sc * res[i];
}

// The box line transforms above on registers for the box lengths they are instantiated for:
// the same lines, maps and scaling, one line per workgroup of L / 16 threads.
template <class R, int R1, int R2, int R3, int R4>
__global__ void __launch_bounds__((rfft::Radices<R1, R2, R3, R4>::T))
k_box_fft_reg(const cpx<R> *r, cpx<R> *work, const int *boxes, const int *rows, int mr, int nx, int ny, int nz, int by,
              int bz, int nboxes, const cpx<R> *tw, const uint32_t *gate, uint32_t epoch) {
    if (gate && *gate != epoch) return;
    constexpr int n = rfft::Radices<R1, R2, R3, R4>::L;
    const long long line = blockIdx.x;  // ((rhs * nboxes + box) * mr + i)
    const int row = rows[(int)(line % mr)];
    const int box = (int)((line / mr) % nboxes);
    const long long rhs = line / ((long long)mr * nboxes);
    const int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = r + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    cpx<R> *dst = work + line * n;
    rfft::reg_line<R, R1, R2, R3, R4, false>(tw, [&](int i) { return src[i]; }, [&](int i, cpx<R> v) { dst[i] = v; });
}

template <class R, int R1, int R2, int R3, int R4>
__global__ void __launch_bounds__((rfft::Radices<R1, R2, R3, R4>::T))
k_box_ifft_reg(const cpx<R> *work, cpx<R> *zv, const int *boxes, const int *rows, int mr, int nx, int ny, int nz,
               int by, int bz, int nboxes, const cpx<R> *tw) {
    constexpr int n = rfft::Radices<R1, R2, R3, R4>::L;
    const long long line = blockIdx.x;
    const int row = rows[(int)(line % mr)];
    const int box = (int)((line / mr) % nboxes);
    const long long rhs = line / ((long long)mr * nboxes);
    const int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const cpx<R> *src = work + line * n;
    cpx<R> *dst = zv + rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    const R sc = R(1) / R(n);
    rfft::reg_line<R, R1, R2, R3, R4, true>(tw, [&](int i) { return src[i]; },
                                            [&](int i, cpx<R> v) { dst[i] = sc * v; });
}

// Launch the register box transform for lengths 1024 .. 8192 (16384 in complex64); false for
// any other length (the LDS Stockham kernels run).  inverse: k_box_ifft_reg (gate unused).
template <class R>
static bool box_fft_reg(bool inverse, const FftPlan &p, long long lines, const cpx<R> *in, cpx<R> *out,
                        const int *boxes, const int *rows, int mr, int nx, int ny, int nz, int by, int bz, int nboxes,
                        const uint32_t *gate, uint32_t epoch, hipStream_t s) {
    const cpx<R> *tw = TwTable<R>::get(p);
#define VIE_BOX_REG(R1, R2, R3, R4)                                                                                    \
    {                                                                                                                  \
        typedef rfft::Radices<R1, R2, R3, R4> RD;                                                                      \
        const size_t lds = sizeof(cpx<R>) * RD::L;                                                                     \
        if (inverse) {                                                                                                 \
            vie_lds_attr((const void *)k_box_ifft_reg<R, R1, R2, R3, R4>, lds);                                        \
            hipLaunchKernelGGL((k_box_ifft_reg<R, R1, R2, R3, R4>), dim3((unsigned)lines), dim3(RD::T), lds, s, in,    \
                               out, boxes, rows, mr, nx, ny, nz, by, bz, nboxes, tw);                                  \
        } else {                                                                                                       \
            vie_lds_attr((const void *)k_box_fft_reg<R, R1, R2, R3, R4>, lds);                                         \
            hipLaunchKernelGGL((k_box_fft_reg<R, R1, R2, R3, R4>), dim3((unsigned)lines), dim3(RD::T), lds, s, in,     \
                               out, boxes, rows, mr, nx, ny, nz, by, bz, nboxes, tw, gate, epoch);                     \
        }                                                                                                              \
        return true;                                                                                                   \
    }
    switch (p.L) {
        case 1024: VIE_BOX_REG(16, 8, 8, 1)
        case 2048: VIE_BOX_REG(16, 16, 8, 1)
        case 4096: VIE_BOX_REG(16, 16, 16, 1)
        case 8192: VIE_BOX_REG(16, 16, 16, 2)
        case 16384:
            if constexpr (sizeof(R) == 4) VIE_BOX_REG(16, 16, 16, 4)
            return false;
        default: return false;
    }
#undef VIE_BOX_REG
}

// 2-level apply, y stage.  Forward: from the x-DFT lines x1[rb][(a, y, z)][kx] (rb = rhs*nboxes
// + box, cross-section row a*by*bz + z*by + y) to x2[rb][(a, z)][ky*bx + kx], transforming along
// y; inverse: back, scaled by 1/by.  One workgroup per (rb, (a, z), group of YC x-modes); the
// YC lines of length by are staged in LDS with coalesced loads and stores along kx.
#define YC 8
template <class R>
__global__ void k_box_yfft(cpx<R> *x1, cpx<R> *x2, int bx, int by, int bz, FftPlan py, int inverse) {
    cpx<R> *a = reinterpret_cast<cpx<R> *>(vie_smem), *b = a + YC * by;
    const int ngx = (bx + YC - 1) / YC;
    const int kg = blockIdx.x % ngx;
    const long long row2 = blockIdx.x / ngx;  // rb * 3 bz + (a*bz + z)
    const int r2 = (int)(row2 % (3 * bz));
    const long long rb = row2 / (3 * bz);
    const int comp = r2 / bz, z = r2 % bz;
    const int kx0 = kg * YC;
    const long long m1 = 3LL * by * bz, nm = (long long)bx * by;
    cpx<R> *l1 = x1 + (rb * m1 + (long long)comp * by * bz + (long long)z * by) * bx;  // + y*bx + kx
    cpx<R> *l2 = x2 + row2 * nm;                                                       // + ky*bx + kx
    for (int e = threadIdx.x; e < YC * by; e += blockDim.x) {
        const int y = e / YC, j = e % YC;
        const int kx = kx0 + j;
        cpx<R> v = czero<R>();
        if (kx < bx) v = inverse ? l2[(long long)y * bx + kx] : l1[(long long)y * bx + kx];
        a[j * by + y] = v;
    }
    __syncthreads();
    LdsLines ln = {YC, by, 0, 1, YC};
    cpx<R> *res = by > 1 ? fft_lds<R>(a, b, ln, py, inverse != 0) : a;
    const R sc = inverse ? R(1) / R(by) : R(1);
    for (int e = threadIdx.x; e < YC * by; e += blockDim.x) {
        const int y = e / YC, j = e % YC;
        const int kx = kx0 + j;
        if (kx >= bx) continue;
        const cpx<R> v = sc * res[j * by + y];
        if (inverse)
            l1[(long long)y * bx + kx] = v;
        else
            l2[(long long)y * bx + kx] = v;
    }
}

// Clear one flag word (a kernel rather than a memset, so a captured apply replays it).
__global__ void k_zero_u32(uint32_t *p) {
    if (threadIdx.x == 0) *p = 0u;
}

// Identity rows of every D_k (M~ = 0 on the row): z = r on their box lines, and *flag = epoch
// when any of that input is nonzero (it then couples into the solved rows).
template <class R>
__global__ void __launch_bounds__(256) k_identity_rows(const cpx<R> *r, cpx<R> *zv, const int *boxes,
                                                       const int *rows, int mc, int nx, int ny, int nz, int by,
                                                       int bz, int nboxes, uint32_t *flag, uint32_t epoch) {
    const long long line = blockIdx.x;  // ((rhs * nboxes + box) * mc + j)
    const int row = rows[(int)(line % mc)];
    const int box = (int)((line / mc) % nboxes);
    const long long rhs = line / ((long long)mc * nboxes);
    const int comp = row / (by * bz), y = row % by, z = (row / by) % bz;
    const int *bx = boxes + 6 * box;
    const long long o = rhs * 3LL * nx * ny * nz + (((long long)comp * nz + bx[2] + z) * ny + bx[1] + y) * nx + bx[0];
    bool nz_ = false;
    for (int i = threadIdx.x; i < bx[3]; i += blockDim.x) {
        const cpx<R> v = r[o + i];
        zv[o + i] = v;
        nz_ |= v.re != R(0) || v.im != R(0) || v.re != v.re || v.im != v.im;
    }
    if (nz_) *flag = epoch;
}

// Coupling of the identity rows C into the solved rows S of D_k = I - M~ C^_k:
// with z^_C = r^_C, the solved rows satisfy D_SS z^_S = r^_S + M~_S (C^_k)_SC r^_C, so
//   work[S] += M~(y, z) sum_j C^_k[(a,y,z), row_j] r^_C[j]
// (one workgroup per (rhs, box, mode k); C^_k read from the Chan/x-DFT table).  Skipped
// unless *gate == epoch.
template <class R>
__global__ void __launch_bounds__(256) k_couple(cpx<R> *work, const cpx<R> *workc, const cpx<R> *chan,
                                                const cpx<R> *mt, const int *rows, int m, int mc, int n,
                                                int nboxes, int by, int bz, const uint32_t *gate,
                                                uint32_t epoch) {
    if (*gate != epoch) return;
    cpx<R> *rc = reinterpret_cast<cpx<R> *>(vie_smem);  // r^_C at mode k
    int *pk = reinterpret_cast<int *>(rc + mc);          // (b, z', y') of row j, packed
    const long long item = blockIdx.x;                   // (rhs * nboxes + box) * n + k
    const int k = (int)(item % n);
    const long long rb = item / n;
    const int box = (int)(rb % nboxes);
    const int plane = by * bz, ndy = 2 * by - 1, ndz = 2 * bz - 1;
    for (int j = threadIdx.x; j < mc; j += blockDim.x) {
        rc[j] = workc[(rb * mc + j) * n + k];
        const int p = rows[m + j], b = p / plane, yz = p - b * plane;
        pk[j] = (b << 20) | ((yz / by) << 10) | (yz % by);
    }
    __syncthreads();
    const cpx<R> *tab = chan + (long long)k * 6 * ndz * ndy;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int p = rows[i], a = p / plane, yz = p - a * plane, z = yz / by, y = yz % by;
        cpx<R> acc = czero<R>();
        for (int j = 0; j < mc; ++j) {
            const int b = pk[j] >> 20, zc = (pk[j] >> 10) & 1023, yc = pk[j] & 1023;
            const int cc = a == b ? a : a + b + 2;  // xy -> 3, xz -> 4, yz -> 5
            acc = acc + tab[(cc * ndz + z - zc + bz - 1) * ndy + y - yc + by - 1] * rc[j];
        }
        cpx<R> *w = work + (rb * m + i) * n + k;
        *w = *w + mt[(long long)box * plane + yz] * acc;
    }
}

// ---------------------------------------------------------------- host side
// 2-level apply: x-DFT of every box line, y-DFT to the (x-mode, y-mode) spectra, one block solve
// per mode pair, inverse y-DFT, inverse x-DFT (Sec. 4: C_B2^{-1}).
template <class R>
static vie_status apply2_t(vie_pc pc, PcWs *ws, const cpx<R> *r, cpx<R> *z, int nrhs, hipStream_t s) {
    vie_op op = pc->op;
    const int bx = pc->bx, by = pc->by, bz = pc->bz, m1 = 3 * by * bz;
    const long long lines1 = (long long)nrhs * pc->nboxes * m1;
    VIE_CHECK(ws->work1.ensure(sizeof(cpx<R>) * lines1 * bx));
    VIE_CHECK(ws->work.ensure(sizeof(cpx<R>) * (size_t)nrhs * pc->nboxes * pc->m * pc->nm));
    if (!pc->covers_all)
        VIE_HIP(hipMemcpyAsync(z, r, sizeof(cpx<R>) * 3 * op->N * nrhs, hipMemcpyDeviceToDevice, s));
    const int *dboxes = reinterpret_cast<const int *>(pc->block_of_mode.as<int>() + pc->nboxes * pc->nm);
    const int *rows1 = pc->rows1.as<const int>();
    int thr, bpt;
    size_t lds;
    fft_line_shape(pc->pxb, sizeof(cpx<R>), &thr, &lds, &bpt);
    cpx<R> *w1 = ws->work1.as<cpx<R>>(), *w2 = ws->work.as<cpx<R>>();
    const unsigned ygrid = (unsigned)((long long)nrhs * pc->nboxes * pc->m * ((bx + YC - 1) / YC));
    const size_t ylds = 2 * sizeof(cpx<R>) * YC * by;
    vie_lds_attr((const void *)k_box_yfft<R>, ylds);
    {
        ProfScope ps("precond_xfft", s);
#define LAUNCH_BOX_FFT(B)                                                                                        \
    vie_lds_attr((const void *)k_box_fft<R, B>, lds);                                                            \
    hipLaunchKernelGGL((k_box_fft<R, B>), dim3((unsigned)lines1), dim3(thr), lds, s, r, w1, dboxes, rows1, m1, op->nx, \
                       op->ny, op->nz, by, bz, pc->nboxes, pc->pxb, nullptr, 0u)
        if (!box_fft_reg<R>(false, pc->pxb, lines1, r, w1, dboxes, rows1, m1, op->nx, op->ny, op->nz, by, bz,
                            pc->nboxes, nullptr, 0u, s))
            VIE_BPT_SWITCH(bpt, LAUNCH_BOX_FFT);
#undef LAUNCH_BOX_FFT
        VIE_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_box_yfft<R>, dim3(ygrid), dim3(256), ylds, s, w1, w2, bx, by, bz, pc->pyb2, 0);
        VIE_HIP(hipGetLastError());
    }
    {
        ProfScope ps("block_solve", s);
        VIE_CHECK(launch_block_solve(pc, ws, w2, nrhs, s));
    }
    {
        ProfScope ps("precond_ixfft", s);
        hipLaunchKernelGGL(k_box_yfft<R>, dim3(ygrid), dim3(256), ylds, s, w1, w2, bx, by, bz, pc->pyb2, 1);
        VIE_HIP(hipGetLastError());
#define LAUNCH_BOX_IFFT(B)                                                                                       \
    vie_lds_attr((const void *)k_box_ifft<R, B>, lds);                                                           \
    hipLaunchKernelGGL((k_box_ifft<R, B>), dim3((unsigned)lines1), dim3(thr), lds, s, w1, z, dboxes, rows1, m1,     \
                       op->nx, op->ny, op->nz, by, bz, pc->nboxes, pc->pxb)
        if (!box_fft_reg<R>(true, pc->pxb, lines1, w1, z, dboxes, rows1, m1, op->nx, op->ny, op->nz, by, bz,
                            pc->nboxes, nullptr, 0u, s))
            VIE_BPT_SWITCH(bpt, LAUNCH_BOX_IFFT);
#undef LAUNCH_BOX_IFFT
    }
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

template <class R>
static vie_status apply_t(vie_pc pc, const cpx<R> *r, cpx<R> *z, int nrhs, hipStream_t s) {
    vie_op op = pc->op;
    PcWs *ws = pc->ws.get(s);
    std::lock_guard<std::mutex> lk(ws->mu);
    if (pc->levels == 2) return apply2_t<R>(pc, ws, r, z, nrhs, s);
    const int m = pc->m, mc = pc->m_full - pc->m, n = pc->bx;
    long long lines = (long long)nrhs * pc->nboxes * m;
    VIE_CHECK(ws->work.ensure(sizeof(cpx<R>) * lines * n));
    if (mc > 0) {
        VIE_CHECK(ws->workc.ensure(sizeof(cpx<R>) * (size_t)nrhs * pc->nboxes * mc * n));
        if (!ws->cflag.p) {  // this stream's first apply: no epoch has matched yet
            VIE_CHECK(ws->cflag.ensure(sizeof(uint32_t)));
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws->cflag.as<uint32_t>());
            VIE_HIP(hipGetLastError());
            ws->epoch = 0;
        }
    }
    if (!pc->covers_all)
        VIE_HIP(hipMemcpyAsync(z, r, sizeof(cpx<R>) * 3 * op->N * nrhs, hipMemcpyDeviceToDevice, s));
    const int *dboxes = reinterpret_cast<const int *>(pc->block_of_mode.as<int>() + pc->nboxes * pc->nm);
    const int *rows = pc->rows.as<const int>();
    int thr, bpt;
    size_t lds;
    fft_line_shape(pc->pxb, sizeof(cpx<R>), &thr, &lds, &bpt);
    cpx<R> *work = ws->work.as<cpx<R>>();
    uint32_t *flag = ws->cflag.as<uint32_t>();
    if (mc > 0) {
        if (++ws->epoch == 0) {  // wrapped: no earlier apply may match the new epochs
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, flag);
            VIE_HIP(hipGetLastError());
            ws->epoch = 1;
        }
        ProfScope ps("precond_identity_rows", s);
        hipLaunchKernelGGL(k_identity_rows<R>, dim3((unsigned)((long long)nrhs * pc->nboxes * mc)), dim3(256), 0, s,
                           r, z, dboxes, rows + m, mc, op->nx, op->ny, op->nz, pc->by, pc->bz, pc->nboxes, flag,
                           ws->epoch);
        VIE_HIP(hipGetLastError());
    }
    {
        ProfScope ps("precond_xfft", s);
#define LAUNCH_BOX_FFT(B)                                                                                   \
    vie_lds_attr((const void *)k_box_fft<R, B>, lds);                                                       \
    hipLaunchKernelGGL((k_box_fft<R, B>), dim3((unsigned)lines), dim3(thr), lds, s, r, work, dboxes, rows, m, \
                       op->nx, op->ny, op->nz, pc->by, pc->bz, pc->nboxes, pc->pxb, nullptr, 0u)
        if (!box_fft_reg<R>(false, pc->pxb, lines, r, work, dboxes, rows, m, op->nx, op->ny, op->nz, pc->by, pc->bz,
                            pc->nboxes, nullptr, 0u, s))
            VIE_BPT_SWITCH(bpt, LAUNCH_BOX_FFT);
#undef LAUNCH_BOX_FFT
    }
    VIE_HIP(hipGetLastError());
    if (mc > 0) {  // both launches return at once unless the identity rows held input
        ProfScope ps("precond_identity_rows", s);
        cpx<R> *workc = ws->workc.as<cpx<R>>();
        const long long clines = (long long)nrhs * pc->nboxes * mc;
#define LAUNCH_BOX_FFT_C(B)                                                                                       \
    vie_lds_attr((const void *)k_box_fft<R, B>, lds);                                                             \
    hipLaunchKernelGGL((k_box_fft<R, B>), dim3((unsigned)clines), dim3(thr), lds, s, r, workc, dboxes, rows + m, \
                       mc, op->nx, op->ny, op->nz, pc->by, pc->bz, pc->nboxes, pc->pxb, flag, ws->epoch)
        if (!box_fft_reg<R>(false, pc->pxb, clines, r, workc, dboxes, rows + m, mc, op->nx, op->ny, op->nz, pc->by,
                            pc->bz, pc->nboxes, flag, ws->epoch, s))
            VIE_BPT_SWITCH(bpt, LAUNCH_BOX_FFT_C);
#undef LAUNCH_BOX_FFT_C
        VIE_HIP(hipGetLastError());
        const cpx<R> *chan = sizeof(R) == 8 ? (const cpx<R> *)pc->chan64.p : (const cpx<R> *)pc->chan32.p;
        const cpx<R> *mt = sizeof(R) == 8 ? (const cpx<R> *)pc->mt64.p : (const cpx<R> *)pc->mt32.p;
        const size_t clds = (sizeof(cpx<R>) + sizeof(int)) * mc;
        vie_lds_attr((const void *)k_couple<R>, clds);
        hipLaunchKernelGGL(k_couple<R>, dim3((unsigned)((long long)nrhs * pc->nboxes * n)), dim3(256), clds, s, work,
                           workc, chan, mt, rows, m, mc, n, pc->nboxes, pc->by, pc->bz, flag, ws->epoch);
        VIE_HIP(hipGetLastError());
    }
    {
        ProfScope ps("block_solve", s);
        VIE_CHECK(launch_block_solve(pc, ws, work, nrhs, s));
    }
    {
        ProfScope ps("precond_ixfft", s);
#define LAUNCH_BOX_IFFT(B)                                                                                  \
    vie_lds_attr((const void *)k_box_ifft<R, B>, lds);                                                      \
    hipLaunchKernelGGL((k_box_ifft<R, B>), dim3((unsigned)lines), dim3(thr), lds, s, work, z, dboxes, rows, m, \
                       op->nx, op->ny, op->nz, pc->by, pc->bz, pc->nboxes, pc->pxb)
        if (!box_fft_reg<R>(true, pc->pxb, lines, work, z, dboxes, rows, m, op->nx, op->ny, op->nz, pc->by, pc->bz,
                            pc->nboxes, nullptr, 0u, s))
            VIE_BPT_SWITCH(bpt, LAUNCH_BOX_IFFT);
#undef LAUNCH_BOX_IFFT
    }
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

vie_status pc_apply(vie_pc pc, const void *r, void *z, int nrhs, int prec, hipStream_t s) {
    if (prec != (pc->prec == VIE_BF16C ? (int)VIE_C64 : pc->prec)) {
        vie_set_error("precond_apply: vector precision must be the factor precision (complex64 for BF16 factors)");
        return VIE_EARG;
    }
    if (!pc->children.empty()) {  // groups of boxes: copy r to z once, then each group writes its boxes
        if (!pc->covers_all) {
            const size_t esz = prec == VIE_C128 ? sizeof(c128) : sizeof(c64);
            VIE_HIP(hipMemcpyAsync(z, r, esz * 3 * pc->op->N * nrhs, hipMemcpyDeviceToDevice, s));
        }
        for (vie_pc c : pc->children) VIE_CHECK(pc_apply(c, r, z, nrhs, prec, s));
        return VIE_OK;
    }
    if (prec == VIE_C128) return apply_t<double>(pc, (const c128 *)r, (c128 *)z, nrhs, s);
    return apply_t<float>(pc, (const c64 *)r, (c64 *)z, nrhs, s);
}

// The central mode is always kept under the memory reduction (the discarded modes use its block).
static bool levels_one_centre(const std::vector<int> &keep, int centre) {
    return centre >= 0 && centre < (int)keep.size() && keep[centre];
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
    const int nbx = pc->nboxes, n = pc->bx, by = pc->by, bz = pc->bz;
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
    if (pc->levels == 2) {
        // the 2-level blocks need M~ independent of y; rows (a, z) in natural order, and the
        // identity map of the full cross-section lines for the x stage of the apply
        std::vector<c128> Mth((size_t)nbx * by * bz);
        VIE_HIP(hipMemcpyAsync(Mth.data(), Mt.p, sizeof(c128) * Mth.size(), hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < Mth.size(); ++i) {
            const c128 &v = Mth[i], &v0 = Mth[i - i % by];
            if (v.re != v0.re || v.im != v0.im) {
                vie_set_error("the 2-level circulant needs a homogenised contrast that does not vary along y "
                              "(homog MODE, or a contrast uniform in x and y per z layer)");
                return VIE_EARG;
            }
        }
        pc->rows_host.resize(pc->m_full);
        for (int i = 0; i < pc->m_full; ++i) pc->rows_host[i] = i;
        VIE_CHECK(pc->rows.ensure(sizeof(int) * pc->m_full));
        VIE_HIP(hipMemcpyAsync(pc->rows.p, pc->rows_host.data(), sizeof(int) * pc->m_full, hipMemcpyHostToDevice, s));
        std::vector<int> id1(3 * by * bz);
        for (int i = 0; i < 3 * by * bz; ++i) id1[i] = i;
        VIE_CHECK(pc->rows1.ensure(sizeof(int) * id1.size()));
        VIE_HIP(hipMemcpyAsync(pc->rows1.p, id1.data(), sizeof(int) * id1.size(), hipMemcpyHostToDevice, s));
        VIE_HIP(hipStreamSynchronize(s));
        VIE_CHECK(op->fft.get(by, &pc->pyb2));
    } else {
    // Row order: cross-section positions (y, z) with M~ != 0 in some box first (all three
    // components); the others are identity rows of every D_k and are not factorised.
        const int plane = by * bz;
        std::vector<char> act(plane, 1);
        if (!o->keep_zero_rows) {
            std::vector<c128> Mth((size_t)nbx * plane);
            VIE_HIP(hipMemcpyAsync(Mth.data(), Mt.p, sizeof(c128) * Mth.size(), hipMemcpyDeviceToHost, s));
            VIE_HIP(hipStreamSynchronize(s));
            int cnt = 0;
            for (int yz = 0; yz < plane; ++yz) {
                bool any = false;
                for (int b = 0; b < nbx; ++b) {
                    const c128 v = Mth[(size_t)b * plane + yz];
                    any |= v.re != 0.0 || v.im != 0.0;
                }
                act[yz] = any;
                cnt += any;
            }
            if (cnt == 0) std::fill(act.begin(), act.end(), 1);  // M~ = 0: keep the (identity) blocks
        }
        pc->rows_host.clear();
        for (int pass = 1; pass >= 0; --pass)
            for (int a = 0; a < 3; ++a)
                for (int yz = 0; yz < plane; ++yz)
                    if (act[yz] == pass) pc->rows_host.push_back(a * plane + yz);
        pc->m = 0;
        for (int yz = 0; yz < plane; ++yz) pc->m += 3 * act[yz];
        // the operator's lines without contrast: identity rows here too when the boxes span the
        // cross-section (position z*by + y in both), so the apply copies its input there
        pc->zero_lines_kept = false;
        if (op->n_line_zero > 0 && by == op->ny && bz == op->nz) {
            std::vector<int> hf(plane);
            VIE_HIP(hipMemcpyAsync(hf.data(), op->yzflag.p, sizeof(int) * plane, hipMemcpyDeviceToHost, s));
            VIE_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int yz = 0; yz < plane; ++yz) all &= hf[yz] != 0 || !act[yz];
            pc->zero_lines_kept = all;
        }
        VIE_CHECK(pc->rows.ensure(sizeof(int) * pc->m_full));
        VIE_HIP(hipMemcpyAsync(pc->rows.p, pc->rows_host.data(), sizeof(int) * pc->m_full, hipMemcpyHostToDevice, s));
    }
    const int m = pc->m, nm = pc->nm;
    const bool shortcut = pc->m < pc->m_full;
    // Chan + x-DFT table
    DevBuf Ch;
    VIE_CHECK(Ch.ensure(sizeof(c128) * (size_t)n * 6 * ndy * ndz));
    {
        int thr, bpt;
        size_t lds;
        fft_line_shape(pc->pxb, sizeof(c128), &thr, &lds, &bpt);
#define LAUNCH_CHAN(B)                                                                                     \
    vie_lds_attr((const void *)k_chan_table<B>, lds);                                                      \
    hipLaunchKernelGGL(k_chan_table<B>, dim3(6 * ndy * ndz), dim3(thr), lds, s, op->gen.as<const c128>(),  \
                       Ch.as<c128>(), op->nx, op->ny, op->nz, n, by, bz, 1, pc->pxb)
        VIE_BPT_SWITCH(bpt, LAUNCH_CHAN);
#undef LAUNCH_CHAN
        VIE_HIP(hipGetLastError());
    }
    // memory reduction: proxy v_k of eq. proxy1 read from the table of N (minus the identity)
    std::vector<int> keep(nm, 1), rep(nm);
    for (int k = 0; k < nm; ++k) rep[k] = k;
    int centre = (n + 1) / 2 - 1;  // ceil(n/2) - 1 (the 1-level memory reduction only)
    if (o->reduce || o->share_tol > 0) {
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
        DevBuf vd;  // gathered on the device: a strided copy of n 16-byte rows to the host is slow
        VIE_CHECK(vd.ensure(sizeof(c128) * n));
        hipLaunchKernelGGL(k_gather_strided, dim3((n + 255) / 256), dim3(256), 0, s,
                           Ch.as<const c128>() + (long long)iz * ndy + iy, vd.as<c128>(), n, 6LL * ndy * ndz);
        VIE_HIP(hipGetLastError());
        VIE_HIP(hipMemcpyAsync(v.data(), vd.p, sizeof(c128) * n, hipMemcpyDeviceToHost, s));
        VIE_HIP(hipStreamSynchronize(s));
        if (yp == 0 && zp == 0)
            for (auto &x : v) x.re -= 1.0;
        double vmax = 0;
        for (auto &x : v) vmax = std::max(vmax, std::sqrt(x.re * x.re + x.im * x.im));
        if (o->reduce) {
            for (int k = 0; k < n; ++k) {
                double vh = vmax > 0 ? std::sqrt(v[k].re * v[k].re + v[k].im * v[k].im) / vmax : 0.0;
                keep[k] = vh > o->reduce_tol;
            }
            // With the reflection pairing (below) the decision of mode k > n/2 is taken at n - k: the
            // proxy is an xx entry, even in x, so |v_{n-k}| = |v_k| up to the DFT's rounding.  The
            // kept set is then symmetric and kept modes pair; discarded ones take the central block
            // unsigned.  (Taken before the central mode is forced in, which its partner is not.)
            if (!o->no_mirror && !(o->share_tol > 0))
                for (int k = 1; k < n; ++k)
                    if (n - k < k) keep[k] = keep[n - k];
            keep[centre] = 1;
        }
        // runs of kept modes whose proxy stays within share_tol of the run's first mode share its block
        if (o->share_tol > 0) {
            int cur = -1;
            for (int k = 0; k < n; ++k) {
                if (!keep[k]) continue;
                const double dre = v[k].re - (cur >= 0 ? v[cur].re : 0.0), dim = v[k].im - (cur >= 0 ? v[cur].im : 0.0);
                const bool own = o->reduce && k == centre;  // the discarded modes' block stays its own
                if (cur >= 0 && !own &&
                    std::sqrt(dre * dre + dim * dim) <=
                        o->share_tol * std::sqrt(v[cur].re * v[cur].re + v[cur].im * v[cur].im))
                    rep[k] = cur;
                else
                    cur = k;
            }
        }
    }
    // reflections: C^_{n-kx} = S_x C^_kx S_x (the x parities of the Chan sequences, exact before
    // the x-DFT), so D_{n-kx} = S_x D_kx S_x and modes kx > n/2 take the factors of mode n - kx;
    // the 2-level table keeps the y parities through its Chan circulant along y, so y-modes
    // ky > by/2 take those of by - ky (S_y on the y rows).
    const bool mirror = !o->no_mirror && (pc->levels == 2 || !(o->share_tol > 0));
    pc->mirror_rows = m / 3;
    std::vector<int> mir(nm, 0), canon(nm);
    for (int k = 0; k < nm; ++k) {
        const int kx = k % n, ky = k / n;
        const bool fx = mirror && n - kx < kx, fy = mirror && pc->levels == 2 && by - ky < ky;
        canon[k] = (fy ? by - ky : ky) * n + (fx ? n - kx : kx);
        mir[k] = (fx ? VIE_MODE_MIRROR_X : 0) | (fy ? VIE_MODE_MIRROR_Y : 0);
    }

    // block map: stored blocks ordered (box, mode)
    pc->block_of_mode_host.assign((size_t)nbx * nm, -1);
    std::vector<int> smode, sbox;
    for (int b = 0; b < nbx; ++b) {
        int *bom = &pc->block_of_mode_host[(size_t)b * nm];
        for (int k = 0; k < nm; ++k)
            if (keep[k] && rep[k] == k && !mir[k]) {  // a stored block
                bom[k] = (int)smode.size();
                smode.push_back(k);
                sbox.push_back(b);
            }
        for (int k = 0; k < nm; ++k)
            if (mir[k]) bom[k] = bom[canon[k]] | mir[k];
        for (int k = 0; k < nm; ++k)
            if (keep[k] && rep[k] != k) bom[k] = bom[rep[k]];  // shares its run's block
        const int cs = levels_one_centre(keep, centre) ? bom[centre] : -1;
        for (int k = 0; k < nm; ++k)
            if (!keep[k]) bom[k] = cs;  // discarded: the central block
    }
    pc->nstored = (int)smode.size();
    // per stored block: the modes that use it (block-solve columns) and its box
    pc->mode_ptr.assign(pc->nstored + 1, 0);
    pc->mode_list.clear();
    pc->block_box = sbox;
    for (int b = 0; b < nbx; ++b)
        for (int k = 0; k < nm; ++k) pc->mode_ptr[(pc->block_of_mode_host[(size_t)b * nm + k] & ~VIE_MODE_MIRROR) + 1]++;
    for (int sb = 0; sb < pc->nstored; ++sb) pc->mode_ptr[sb + 1] += pc->mode_ptr[sb];
    pc->mode_list.assign(pc->mode_ptr[pc->nstored], 0);
    {
        std::vector<int> fill(pc->mode_ptr.begin(), pc->mode_ptr.end() - 1);
        for (int b = 0; b < nbx; ++b)
            for (int k = 0; k < nm; ++k) {
                const int e = pc->block_of_mode_host[(size_t)b * nm + k];
                pc->mode_list[fill[e & ~VIE_MODE_MIRROR]++] = k | (e & VIE_MODE_MIRROR);
            }
    }
    VIE_CHECK(pc->modes_dev.ensure(sizeof(int) * (pc->mode_ptr.size() + pc->mode_list.size())));
    VIE_HIP(hipMemcpyAsync(pc->modes_dev.p, pc->mode_ptr.data(), sizeof(int) * pc->mode_ptr.size(),
                           hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(pc->modes_dev.as<int>() + pc->mode_ptr.size(), pc->mode_list.data(),
                           sizeof(int) * pc->mode_list.size(), hipMemcpyHostToDevice, s));
    // device block map followed by the boxes (apply kernels read both)
    VIE_CHECK(pc->block_of_mode.ensure(sizeof(int) * ((size_t)nbx * nm + 6 * nbx)));
    VIE_HIP(hipMemcpyAsync(pc->block_of_mode.p, pc->block_of_mode_host.data(), sizeof(int) * (size_t)nbx * nm,
                           hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(pc->block_of_mode.as<int>() + (size_t)nbx * nm, pc->boxes.data(), sizeof(int) * 6 * nbx,
                           hipMemcpyHostToDevice, s));
    DevBuf dmode, dbox;
    VIE_CHECK(dmode.ensure(sizeof(int) * pc->nstored));
    VIE_CHECK(dbox.ensure(sizeof(int) * pc->nstored));
    VIE_HIP(hipMemcpyAsync(dmode.p, smode.data(), sizeof(int) * pc->nstored, hipMemcpyHostToDevice, s));
    VIE_HIP(hipMemcpyAsync(dbox.p, sbox.data(), sizeof(int) * pc->nstored, hipMemcpyHostToDevice, s));
    // BF16 factors: assembled and factorised in complex float, rounded afterwards
    size_t esz = pc->prec == VIE_C128 ? sizeof(c128) : sizeof(c64);
    VIE_CHECK(pc->factors.ensure(esz * (size_t)pc->nstored * m * m));
    VIE_CHECK(pc->perm.ensure(sizeof(int) * (size_t)pc->nstored * m));
    VIE_CHECK(pc->info.ensure(sizeof(int) * (size_t)pc->nstored));
    dim3 ga((unsigned)(((long long)m * m + 255) / 256), pc->nstored);
    dim3 gc((unsigned)((m + AS_COLS - 1) / AS_COLS), pc->nstored);
    if (pc->levels == 2) {  // second level: Chan along y + y-DFT of the x-level table, then the blocks
        DevBuf Ch2;
        VIE_CHECK(Ch2.ensure(sizeof(c128) * (size_t)nm * 6 * ndz));
        const size_t lds = 2 * sizeof(c128) * by;
        vie_lds_attr((const void *)k_chan_table2, lds);
        hipLaunchKernelGGL(k_chan_table2, dim3((unsigned)(n * 6 * ndz)), dim3(64), lds, s, Ch.as<const c128>(),
                           Ch2.as<c128>(), n, by, bz, pc->pyb2);
        VIE_HIP(hipGetLastError());
        if (pc->prec == VIE_C128)
            hipLaunchKernelGGL(k_assemble2<double>, ga, dim3(256), 0, s, Ch2.as<const c128>(), Mt.as<const c128>(),
                               dmode.as<const int>(), dbox.as<const int>(), pc->factors.as<c128>(), by, bz);
        else
            hipLaunchKernelGGL(k_assemble2<float>, ga, dim3(256), 0, s, Ch2.as<const c128>(), Mt.as<const c128>(),
                               dmode.as<const int>(), dbox.as<const int>(), pc->factors.as<c64>(), by, bz);
        VIE_HIP(hipGetLastError());
        VIE_HIP(hipStreamSynchronize(s));
    } else if (pc->prec == VIE_C128)
        hipLaunchKernelGGL(k_assemble<double>, gc, dim3(256), 0, s, Ch.as<const c128>(), Mt.as<const c128>(),
                           dmode.as<const int>(), dbox.as<const int>(), pc->rows.as<const int>(),
                           pc->factors.as<c128>(), m, by, bz);
    else
        hipLaunchKernelGGL(k_assemble<float>, gc, dim3(256), 0, s, Ch.as<const c128>(), Mt.as<const c128>(),
                           dmode.as<const int>(), dbox.as<const int>(), pc->rows.as<const int>(),
                           pc->factors.as<c64>(), m, by, bz);
    VIE_HIP(hipGetLastError());
    VIE_HIP(hipStreamSynchronize(s));
    if (pc->refine || (shortcut && pc->prec != VIE_C128)) {
        // FP32 copies of the C^_k tables and of M~ (refinement residual, identity-row coupling)
        const long long nch = (long long)n * 6 * ndy * ndz, nmt = (long long)nbx * by * bz;
        VIE_CHECK(pc->chan32.ensure(sizeof(c64) * nch));
        VIE_CHECK(pc->mt32.ensure(sizeof(c64) * nmt));
        hipLaunchKernelGGL(k_narrow_c128, dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, s, Ch.as<const c128>(),
                           pc->chan32.as<c64>(), nch);
        hipLaunchKernelGGL(k_narrow_c128, dim3((unsigned)((nmt + 255) / 256)), dim3(256), 0, s, Mt.as<const c128>(),
                           pc->mt32.as<c64>(), nmt);
        VIE_HIP(hipGetLastError());
    }
    VIE_CHECK(pc->smode_dev.ensure(sizeof(int) * pc->nstored));
    VIE_HIP(hipMemcpyAsync(pc->smode_dev.p, smode.data(), sizeof(int) * pc->nstored, hipMemcpyHostToDevice, s));
    VIE_HIP(hipStreamSynchronize(s));
    if (shortcut && pc->prec == VIE_C128) {  // FP64 table and M~ kept for the identity-row coupling
        std::swap(pc->chan64.p, Ch.p);
        std::swap(pc->chan64.bytes, Ch.bytes);
        std::swap(pc->mt64.p, Mt.p);
        std::swap(pc->mt64.bytes, Mt.bytes);
    }
    Ch.release();
    vie_status st = pc->prec == VIE_C128 ? lu_factor<double>(pc, s) : lu_factor<float>(pc, s);
    VIE_CHECK(st);
    if (pc->prec == VIE_BF16C) {
        const long long cnt = (long long)pc->nstored * m * m;
        DevBuf b16;
        VIE_CHECK(b16.ensure(sizeof(bf16c) * cnt));
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, pc->factors.as<const c64>(),
                           b16.as<bf16c>(), cnt);
        VIE_HIP(hipGetLastError());
        VIE_HIP(hipStreamSynchronize(s));
        std::swap(pc->factors.p, b16.p);
        std::swap(pc->factors.bytes, b16.bytes);
    }
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
