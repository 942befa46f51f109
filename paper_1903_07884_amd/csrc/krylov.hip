// Restarted right-preconditioned flexible GMRES on the device, batched over right-hand
// sides in lockstep (Sec. 1: the discrete JVIE is solved by GMRES; restart, side and
// orthogonalisation are this library's choices).
//
// Arnoldi by classical Gram-Schmidt applied twice, with the second pass of each vector
// delayed to the next step, so that a step makes one reduction pass and one update pass over
// the basis instead of two of each.  Slot j of the basis first holds u_j: orthogonalised once
// against q_0..q_{j-1}, not normalised (u_0 = r).  Step j, for every right-hand side at once:
//   z_j = P^{-1} u_j (kept, so x += Z y at the end of a cycle: flexible GMRES),
//   w = A z_j (one batched operator product),
//   reduction pass:  s = Q^H u_j, a = |u_j|^2, c = Q^H w, d = u_j^H w, e = |w|^2,
//   alpha = sqrt(a - |s|^2), so q_j = (u_j - Q s) / alpha is u_j's second pass, normalised,
//   h = q_j^H w = (d - s^H c) / alpha,
//   update pass:  q_j over u_j in slot j, and in slot j + 1
//                 u_{j+1} = (w - Q c - q_j h) / sigma = (w - Q (c - s h / alpha) - u_j h / alpha) / sigma,
//                 sigma = |w|, so that no stored vector grows or shrinks from step to step
//                 (u_0 = r / |r| likewise).
// As u_{j+1} = Q' s' + alpha' q_{j+1} (Q' = [Q, q_j]; s', alpha' from the next reduction),
// A z_j = Q' ([c; h] + sigma s') + sigma alpha' q_{j+1}: column j of the Hessenberg matrix is
// [c; h] + sigma s' with subdiagonal sigma alpha'.  So step j completes column j - 1 and forms its complex Givens
// rotation, and a cycle's last column is completed by one more reduction pass.  Convergence
// and breakdown are judged at step j on the provisional column [c; h] with subdiagonal
// sigma |u_{j+1}|, which differs from the completed one only by the second-pass terms.  Z holds the
// preconditioned u_j, for which A Z = Q H holds, so x += Z y is the flexible GMRES update; with
// a fixed preconditioner span{P^{-1} u_i} = P^{-1} span{q_i}, and the iterates are GMRES's.
// All sums are FP64; one residual estimate and breakdown flag per right-hand side are read
// back per step.  Each cycle ends with x += Z y and the FP64 true residual r = b - A x.
// Every right-hand side runs its own restart cycles in a ring of basis slots (ring_slot), so
// a column can end a cycle, restart or enter (a queued request taking a free slot) at any step
// while the others go on; a column's arithmetic never depends on the others'.
//
// FP64 mode: basis, z, products and factors complex128.  Mixed mode: the basis (u_j, then q_j)
// is stored in complex64 and u_j feeds the complex64 preconditioner and operator product, whose
// result the reduction and update passes read as is and widen on load (their sums are FP64); Z is
// kept in complex64; the true residual of every cycle uses the complex128 product, so the outer
// loop is an FP64 iterative refinement around the FP32 inner solve.  Mixed-preconditioner mode: only the preconditioner
// runs in complex64 (or bfloat16 factors), on a complex64 copy of u_j; Z is kept in complex64,
// each z_j is widened for the complex128 product, and the basis stays complex128.
#include <cmath>

#include "vie_internal.h"

#define KR_THREADS 256
#define KR_MAX_RESTART VIE_MAX_RESTART
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

// Basis slots form a ring of m + 1 per right-hand side: basis vector i of column r's current
// cycle lives in slot (s0_r + i) mod (m + 1), s0_r being the slot its cycle started in.  Columns
// that started together share the slot of every step; a column that (re)starts later keeps its
// own offset, and at any step the vector every active column needs next sits in one common
// slot (the step index mod m + 1), so the batched preconditioner and product read one slot.
__device__ __forceinline__ long long ring_slot(int s0, int i, int m1) {
    const int k = s0 + i;
    return k >= m1 ? k - m1 : k;
}

// The elements of a vector one part of the Arnoldi passes covers.  Without a line list: a
// contiguous chunk of [0, n).  With one (the x-lines of the grid where the contrast is not zero
// everywhere; every basis vector is zero on the others, see solve_gmres): the part's share of the
// listed lines, element i of the share at lines[l0 + i / nx] * nx + i mod nx.
struct ActiveLines {
    const int *lines = nullptr;  // nullptr: every element
    int nlines = 0, nx = 0;
};
struct PartRange {
    long long lo, hi;  // local indices [lo, hi) of this part
    int l0, nx;
    const int *lines;
    __device__ __forceinline__ PartRange(const ActiveLines &A, long long n, int part, int parts) : nx(A.nx), lines(A.lines) {
        if (lines) {
            const int per = (A.nlines + parts - 1) / parts;
            l0 = min(A.nlines, part * per);
            const int l1 = min(A.nlines, l0 + per);
            lo = 0;
            hi = (long long)(l1 - l0) * nx;
        } else {
            const long long chunk = (n + parts - 1) / parts;
            lo = part * chunk;
            hi = min(n, lo + chunk);
            l0 = 0;
        }
    }
    // vector index of local index i (i < hi; (l1 - l0) nx is far below 2^24, so FastDiv is exact)
    __device__ __forceinline__ long long at(long long i, const FastDiv &fnx) const {
        if (!lines) return i;
        const int li = fnx.div((int)i);
        return (long long)lines[l0 + li] * nx + (i - (long long)li * nx);
    }
};

// Reduction pass of an Arnoldi step, per right-hand side r with mask[r] set (no mask: all), and
// with nq = nq_r[r] basis vectors q_i, u in the ring slot after them, and w (optional):
//   partial[(r * gridDim.x + blk) * stride + k] = the part's share of
//     k < nq: conj(q_k) . u;  with w: nq + k: conj(q_k) . w, then 2nq: |u|^2, 2nq+1: conj(u) . w,
//     2nq+2: |w|^2;  without w: nq: |u|^2.
// need_nq skips columns with nq = 0 (the finishing reduction of a cycle).  The outputs are
// formed KR_DG2 basis vectors at a time (u and w read once per group); inside a group the
// loads of an element are unconditional (a short last group clamps its index and drops the
// extra products), so they are in flight together.  w is complex128 or, in mixed mode, the
// complex64 product itself (widened on load: the sums stay FP64).
#define KR_DG2 8
template <class VT, class WT>
__global__ void __launch_bounds__(KR_THREADS) k_dots2(const VT *V, long long ldj, int m1, const int *nq_r,
                                                      const int *s0_r, const WT *w, long long n, const int *mask,
                                                      int need_nq, int stride, c128 *partial, ActiveLines act) {
    __shared__ c128 sh[2 * KR_DG2 + 3][KR_THREADS / 64];
    const int r = blockIdx.y;
    if (mask && !mask[r]) return;
    const int nqr = nq_r[r], s0 = s0_r[r];
    if (need_nq && nqr == 0) return;
    const VT *Vr = V + r * n;
    const VT *ur = Vr + ring_slot(s0, nqr, m1) * ldj;
    const WT *wr = w ? w + r * n : nullptr;
    const PartRange pr(act, n, blockIdx.x, gridDim.x);
    const FastDiv fnx(act.lines ? act.nx : 1);
    c128 *out = partial + ((long long)r * gridDim.x + blockIdx.x) * stride;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int ngroups = nqr > 0 ? (nqr + KR_DG2 - 1) / KR_DG2 : 1;
    const int self0 = wr ? 2 * nqr : nqr;  // index of |u|^2
    const int last = max(nqr - 1, 0);
    for (int gi = 0; gi < ngroups; ++gi) {
        const int i0 = gi * KR_DG2, cnt = max(0, min(KR_DG2, nqr - i0));
        const bool self = gi == 0;
        const VT *vp[KR_DG2];
#pragma unroll
        for (int u = 0; u < KR_DG2; ++u) vp[u] = Vr + ring_slot(s0, min(i0 + u, last), m1) * ldj;
        c128 as[KR_DG2], ac[KR_DG2], sd = czero<double>();
        double sa = 0.0, se = 0.0;
#pragma unroll
        for (int u = 0; u < KR_DG2; ++u) as[u] = ac[u] = czero<double>();
        for (long long i = pr.lo + threadIdx.x; i < pr.hi; i += KR_THREADS) {
            const long long e = pr.at(i, fnx);
            const c128 ue = wide(ur[e]);
            const c128 we = wr ? wide(wr[e]) : czero<double>();
            c128 v[KR_DG2];
#pragma unroll
            for (int u = 0; u < KR_DG2; ++u) v[u] = wide(vp[u][e]);
#pragma unroll
            for (int u = 0; u < KR_DG2; ++u)
                if (u < cnt) {
                    as[u] = as[u] + cmulc(v[u], ue);
                    if (wr) ac[u] = ac[u] + cmulc(v[u], we);
                }
            if (self) {
                sa += abs2(ue);
                if (wr) {
                    sd = sd + cmulc(ue, we);
                    se += abs2(we);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KR_DG2; ++u) {
            if (u >= cnt) break;
            const c128 t1 = wave_sum(as[u]);
            if (lane == 0) sh[u][wid] = t1;
            if (wr) {
                const c128 t2 = wave_sum(ac[u]);
                if (lane == 0) sh[KR_DG2 + u][wid] = t2;
            }
        }
        if (self) {
            const c128 t0 = wave_sum(mk(sa, 0.0));
            if (lane == 0) sh[2 * KR_DG2][wid] = t0;
            if (wr) {
                const c128 t1 = wave_sum(sd), t2 = wave_sum(mk(se, 0.0));
                if (lane == 0) {
                    sh[2 * KR_DG2 + 1][wid] = t1;
                    sh[2 * KR_DG2 + 2][wid] = t2;
                }
            }
        }
        __syncthreads();
        // thread t < 2 KR_DG2 + 3 writes one output of the group
        const int t = threadIdx.x;
        int slot = -1, dst = 0;
        if (t < cnt) slot = t, dst = i0 + t;
        else if (wr && t >= KR_DG2 && t < KR_DG2 + cnt) slot = t, dst = nqr + i0 + (t - KR_DG2);
        else if (self && t == 2 * KR_DG2) slot = t, dst = self0;
        else if (self && wr && t > 2 * KR_DG2 && t < 2 * KR_DG2 + 3) slot = t, dst = self0 + (t - 2 * KR_DG2);
        if (slot >= 0) {
            c128 acc = czero<double>();
            for (int q = 0; q < KR_THREADS / 64; ++q) acc = acc + sh[slot][q];
            out[dst] = acc;
        }
        __syncthreads();
    }
}

// Update pass of an Arnoldi step, per active right-hand side r with nq = nq_r[r] basis vectors
// in its ring (above) and co = coef + r * cstride = [s_i (nq) | c_i - s_i h/alpha (nq) | 1/alpha |
// h/alpha | 1/sigma]:
//   slot of u_j:  q_j = (u_j - sum_i q_i s_i) / alpha                                  (over u_j)
//   next slot:    u_{j+1} = (w - sum_i q_i (c_i - s_i h/alpha) - u_j h/alpha) / sigma   (and a complex64 copy in vlo)
//   partial[r * gridDim.x + blk] = the part's share of |u_{j+1}|^2 (FP64 values).
// The next slot is next_slot for every active column.  An inactive column's slot next_slot
// lies past its last basis vector (its cycle ended before this step; within one cycle of at
// most m steps the ring does not come back to it), so it is zeroed, with its complex64 copy:
// the batch's preconditioner applies and products then never read stale values for it.
template <class VT, class WT>
__global__ void __launch_bounds__(KR_THREADS) k_update2(VT *V, long long ldj, int m1, const int *nq_r,
                                                        const int *s0_r, int next_slot, const c128 *coef, int cstride,
                                                        const WT *w, long long n, const int *active, c64 *vlo,
                                                        c128 *partial, ActiveLines act) {
    typedef decltype(V->re) T;
    __shared__ c128 cs[2 * KR_MAX_RESTART + 3];
    __shared__ c128 sh[KR_THREADS / 64];
    const int r = blockIdx.y;
    const PartRange pr(act, n, blockIdx.x, gridDim.x);
    const FastDiv fnx(act.lines ? act.nx : 1);
    VT *Vr = V + r * n;
    VT *un = Vr + next_slot * ldj;
    if (!active[r]) {
        for (long long i = pr.lo + threadIdx.x; i < pr.hi; i += KR_THREADS) {
            const long long e = pr.at(i, fnx);
            un[e] = mk((T)0, (T)0);
            if (vlo) vlo[r * n + e] = mk(0.0f, 0.0f);
        }
        return;
    }
    const int nq = nq_r[r], s0 = s0_r[r];
    const c128 *co = coef + (long long)r * cstride;
    for (int i = threadIdx.x; i < 2 * nq + 3; i += KR_THREADS) cs[i] = co[i];
    __syncthreads();
    const double ia = cs[2 * nq].re, isg = cs[2 * nq + 2].re;
    const c128 hu = cs[2 * nq + 1];
    VT *ur = Vr + ring_slot(s0, nq, m1) * ldj;
    const WT *wr = w + r * n;
    c64 *lr = vlo ? vlo + r * n : nullptr;
    double nrm = 0.0;
    for (long long li = pr.lo + threadIdx.x; li < pr.hi; li += KR_THREADS) {
        const long long e = pr.at(li, fnx);
        const c128 u = wide(ur[e]);
        c128 aq = u, aw = wide(wr[e]);
        int i = 0;
        for (; i + 8 <= nq; i += 8) {  // eight loads in flight, products in order of i
            c128 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = wide(Vr[ring_slot(s0, i + k, m1) * ldj + e]);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                aq = cfms(aq, v[k], cs[i + k]);
                aw = cfms(aw, v[k], cs[nq + i + k]);
            }
        }
        for (; i < nq; ++i) {
            const c128 v = wide(Vr[ring_slot(s0, i, m1) * ldj + e]);
            aq = cfms(aq, v, cs[i]);
            aw = cfms(aw, v, cs[nq + i]);
        }
        aw = cfms(aw, u, hu);
        aw = mk(aw.re * isg, aw.im * isg);
        ur[e] = mk((T)(aq.re * ia), (T)(aq.im * ia));
        un[e] = mk((T)aw.re, (T)aw.im);
        if (lr) lr[e] = mk((float)aw.re, (float)aw.im);
        nrm += abs2(aw);
    }
    const c128 t = block_sum_kr(mk(nrm, 0.0), sh);
    if (threadIdx.x == 0) partial[(long long)r * gridDim.x + blockIdx.x] = t;
}

// Zero the listed x-lines (nx elements each) of `count` vectors of n elements, vector v at
// base + v * n (grid.y = vectors).
template <class T>
__global__ void __launch_bounds__(KR_THREADS) k_zero_lines(T *base, long long n, const int *lines, int nlines, int nx) {
    T *v = base + (long long)blockIdx.y * n;
    const long long total = (long long)nlines * nx;
    const FastDiv fnx(nx);
    for (long long i = (long long)blockIdx.x * KR_THREADS + threadIdx.x; i < total; i += (long long)gridDim.x * KR_THREADS) {
        const int li = fnx.div((int)i);
        T z;
        z.re = 0;
        z.im = 0;
        v[(long long)lines[li] * nx + (i - (long long)li * nx)] = z;
    }
}

// On the listed lines (where the operator is the identity, so x = b there exactly) of the right-
// hand sides col0 + blockIdx.y: x = b and r = 0; *nonzero is set where b has an entry there.
__global__ void __launch_bounds__(KR_THREADS) k_identity_lines(c128 *x, const c128 *b, c128 *r, long long n,
                                                               int col0, const int *lines, int nlines, int nx,
                                                               int *nonzero) {
    const long long off = (long long)(col0 + blockIdx.y) * n;
    const long long total = (long long)nlines * nx;
    const FastDiv fnx(nx);
    int nz = 0;
    for (long long i = (long long)blockIdx.x * KR_THREADS + threadIdx.x; i < total; i += (long long)gridDim.x * KR_THREADS) {
        const int li = fnx.div((int)i);
        const long long e = off + (long long)lines[li] * nx + (i - (long long)li * nx);
        const c128 bv = b[e];
        x[e] = bv;
        r[e] = czero<double>();
        nz |= bv.re != 0.0 || bv.im != 0.0;
    }
    if (nz) atomicOr(nonzero, 1);
}

// x_r += sum_{i < jr[r]} z_i,r y_r[i], z_i of column r in the slot (z0_r + i) mod m of the ring
// of m preconditioned vectors (Z in complex128 or complex64).
template <class R>
__global__ void __launch_bounds__(KR_THREADS) k_combine(const cpx<R> *Z, long long ldj, int m, const int *jr,
                                                        const int *z0_r, const c128 *y, int ystride, c128 *x,
                                                        long long n) {
    __shared__ c128 ys[256];
    __shared__ int zs[256];
    const int r = blockIdx.y;
    const int nv = jr[r], z0 = z0_r[r];
    for (int i = threadIdx.x; i < nv; i += KR_THREADS) {
        ys[i] = y[(long long)r * ystride + i];
        zs[i] = z0 + i >= m ? z0 + i - m : z0 + i;
    }
    __syncthreads();
    if (nv == 0) return;
    for (long long e = blockIdx.x * (long long)KR_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * KR_THREADS) {
        c128 acc = x[r * n + e];
        for (int i = 0; i < nv; ++i) {
            cpx<R> z = Z[zs[i] * ldj + r * n + e];
            acc = acc + mk((double)z.re, (double)z.im) * ys[i];
        }
        x[r * n + e] = acc;
    }
}

// First basis vector of a new cycle for the right-hand sides with mask[r] set: u_0 = r / beta
// (zero for a zero beta) into ring slot `slot`, with an optional complex64 copy; the other
// columns are left as they are.
template <class VT>
__global__ void k_store(const c128 *src, VT *V, long long ldj, int slot, c64 *vlo, long long n, const double *beta,
                        const int *mask) {
    typedef decltype(V->re) T;
    const int r = blockIdx.y;
    if (!mask[r]) return;
    const double f = beta[r] > 0.0 ? 1.0 / beta[r] : 0.0;
    VT *v = V + slot * ldj + r * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const c128 a = f * src[r * n + e];
        v[e] = mk((T)a.re, (T)a.im);
        if (vlo) vlo[r * n + e] = mk((float)a.re, (float)a.im);
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
    c128 *h1;    // [R][hstride]: the step's reduction outputs (hstride >= 2m + 3)
    c128 *coef;  // [R][cstride]: the update pass's coefficients (cstride >= 2m + 3)
    c128 *nrm2;  // [R]: |u_{j+1}|^2
    c128 *P;     // [R][m][m+1] column-major: [c; h] of each step (before the second-pass terms)
    c128 *Rm;    // [R][m][m+1] column-major: completed columns after their rotations
    double *cs;  // [R][m]
    c128 *sn;    // [R][m]
    c128 *g;     // [R][m+1]
    c128 *y;     // [R][m]
    double *st;  // [R][4]: provisional |g_{j+1}|, sigma |u_{j+1}|, breakdown, |w|
    double *sig; // [R][m]: sigma_j = |w| of step j (the scale of u_{j+1})
    double *beta; // [R]: |r| of the cycle (the scale of u_0)
    int *active; // [R]
    int m, hstride, cstride;
};

// Complete column jc of right-hand side r: col = P[jc][0..jc] + sigma_jc s[0..jc] with
// subdiagonal sigma_jc alpha; apply rotations 0..jc-1, form rotation jc (c real, s complex), update g and store the
// rotated column.  One wavefront; col / csl / snl are LDS arrays of the caller.
__device__ void finish_column(GState &S, int r, int jc, const c128 *s, double alpha, c128 *col, double *csl,
                              c128 *snl) {
    const int m = S.m, lane = threadIdx.x;
    const c128 *pc = S.P + ((long long)r * m + jc) * (m + 1);
    double *cs = S.cs + (long long)r * m;
    c128 *sn = S.sn + (long long)r * m;
    c128 *g = S.g + (long long)r * (m + 1);
    const double sg = S.sig[(long long)r * m + jc];
    for (int i = lane; i <= jc; i += 64) col[i] = pc[i] + sg * s[i];
    for (int i = lane; i < jc; i += 64) {
        csl[i] = cs[i];
        snl[i] = sn[i];
    }
    __syncthreads();
    if (lane == 0) {
        for (int i = 0; i < jc; ++i) {
            const c128 a = col[i], b = col[i + 1];
            col[i] = csl[i] * a + snl[i] * b;
            col[i + 1] = csl[i] * b - conjg(snl[i]) * a;
        }
        const c128 a = col[jc];
        const double aa = sqrt(abs2(a)), bb = sg * alpha;
        double c;
        c128 sr, rr;
        if (bb == 0.0) {
            c = 1.0;
            sr = czero<double>();
            rr = a;
        } else if (aa == 0.0) {
            c = 0.0;
            sr = mk(1.0, 0.0);
            rr = mk(bb, 0.0);
        } else {
            const double rho = hypot(aa, bb);
            const c128 ph = mk(a.re / aa, a.im / aa);
            c = aa / rho;
            sr = mk(ph.re * bb / rho, ph.im * bb / rho);  // phase * conj(b) / rho, b real
            rr = mk(ph.re * rho, ph.im * rho);
        }
        cs[jc] = c;
        sn[jc] = sr;
        col[jc] = rr;
        const c128 gj = g[jc];
        g[jc + 1] = czero<double>() - conjg(sr) * gj;
        g[jc] = c * gj;
    }
    __syncthreads();
    c128 *rc = S.Rm + ((long long)r * m + jc) * (m + 1);
    for (int i = lane; i <= jc; i += 64) rc[i] = col[i];
}

// After the reduction of a step, per active right-hand side r at its step j = jcol[r] of its
// cycle (one wavefront): alpha, h, sigma,
// the update coefficients, the step's column [c; h], and column j - 1 completed (for j = 0:
// g = (beta alpha, 0, ...), r = beta u_0 = beta alpha q_0).
__global__ void __launch_bounds__(64) k_arnoldi_coef(GState S, const int *jcol, int R) {
    __shared__ c128 col[KR_MAX_RESTART + 1];
    __shared__ double csl[KR_MAX_RESTART];
    __shared__ c128 snl[KR_MAX_RESTART];
    __shared__ double sal;
    __shared__ c128 shu;
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= R || !S.active[r]) return;
    const int m = S.m, j = jcol[r];
    const c128 *h = S.h1 + (long long)r * S.hstride;  // [s (j) | c (j) | a | d | e]
    double ss = 0.0;
    c128 sc = czero<double>();
    for (int i = lane; i < j; i += 64) {
        ss += abs2(h[i]);
        sc = sc + cmulc(h[i], h[j + i]);
    }
    const c128 ssum = wave_sum(mk(ss, 0.0)), csum = wave_sum(sc);
    c128 *pcol = S.P + ((long long)r * m + j) * (m + 1);
    if (lane == 0) {
        const double a2 = h[2 * j].re - ssum.re;
        const double al = a2 > 0.0 ? sqrt(a2) : 0.0;
        const c128 d = h[2 * j + 1] - csum;
        const c128 hh = al > 0.0 ? mk(d.re / al, d.im / al) : czero<double>();
        sal = al;
        shu = al > 0.0 ? mk(hh.re / al, hh.im / al) : czero<double>();
        pcol[j] = hh;
        const double sg = sqrt(h[2 * j + 2].re);
        S.sig[(long long)r * m + j] = sg;
        c128 *co = S.coef + (long long)r * S.cstride;
        co[2 * j + 2] = mk(sg > 0.0 ? 1.0 / sg : 0.0, 0.0);
    }
    __syncthreads();
    const double al = sal;
    const c128 hu = shu;
    c128 *co = S.coef + (long long)r * S.cstride;  // [s (j) | c - s h/alpha (j) | 1/alpha | h/alpha | 1/sigma]
    for (int i = lane; i < j; i += 64) {
        co[i] = h[i];
        co[j + i] = h[j + i] - h[i] * hu;
        pcol[i] = h[j + i];
    }
    if (lane == 0) {
        co[2 * j] = mk(al > 0.0 ? 1.0 / al : 0.0, 0.0);
        co[2 * j + 1] = hu;
    }
    if (j == 0) {
        c128 *g = S.g + (long long)r * (m + 1);
        for (int i = lane; i <= m; i += 64) g[i] = mk(i == 0 ? S.beta[r] * al : 0.0, 0.0);
    } else {
        finish_column(S, r, j - 1, h, al, col, csl, snl);
    }
}

// After the update pass of a step, per active right-hand side r at its step j = jcol[r] (one
// wavefront): the provisional
// residual estimate |g_{j+1}| of column [c; h] with subdiagonal sigma |u_{j+1}| under the
// completed rotations 0..j-1, and the breakdown flag (sigma |u_{j+1}| <= 1e-14 |w|, sigma = |w|).
__global__ void __launch_bounds__(64) k_arnoldi_est(GState S, const int *jcol, int R) {
    __shared__ c128 col[KR_MAX_RESTART + 1];
    __shared__ double csl[KR_MAX_RESTART];
    __shared__ c128 snl[KR_MAX_RESTART];
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= R) return;
    double *st = S.st + 4 * r;
    if (!S.active[r]) {
        if (lane == 0) st[0] = 0.0, st[1] = 0.0, st[2] = 1.0, st[3] = 0.0;
        return;
    }
    const int m = S.m, j = jcol[r];
    const c128 *pc = S.P + ((long long)r * m + j) * (m + 1);
    for (int i = lane; i <= j; i += 64) col[i] = pc[i];
    for (int i = lane; i < j; i += 64) {
        csl[i] = S.cs[(long long)r * m + i];
        snl[i] = S.sn[(long long)r * m + i];
    }
    __syncthreads();
    if (lane == 0) {
        for (int i = 0; i < j; ++i) {
            const c128 a = col[i], b = col[i + 1];
            col[i] = csl[i] * a + snl[i] * b;
            col[i + 1] = csl[i] * b - conjg(snl[i]) * a;
        }
        const double w0 = S.sig[(long long)r * m + j];
        const double aa = sqrt(abs2(col[j])), bb = w0 * sqrt(S.nrm2[r].re);
        const double rho = hypot(aa, bb);
        const double gj = sqrt(abs2(S.g[(long long)r * (m + 1) + j]));
        st[0] = rho > 0.0 ? gj * bb / rho : 0.0;
        st[1] = bb;
        st[2] = (bb <= 1e-14 * w0) ? 1.0 : 0.0;
        st[3] = w0;
    }
}

// End of a cycle, per right-hand side with jr[r] > 0 steps: complete its last column jr - 1 from
// the finishing reduction [s (jr) | a] of u_{jr} against q_0..q_{jr-1}.
__global__ void __launch_bounds__(64) k_arnoldi_final(GState S, const int *jr, int R) {
    __shared__ c128 col[KR_MAX_RESTART + 1];
    __shared__ double csl[KR_MAX_RESTART];
    __shared__ c128 snl[KR_MAX_RESTART];
    __shared__ double sal;
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= R) return;
    const int k = jr[r];
    if (k == 0) return;
    const c128 *h = S.h1 + (long long)r * S.hstride;
    double ss = 0.0;
    for (int i = lane; i < k; i += 64) ss += abs2(h[i]);
    const c128 ssum = wave_sum(mk(ss, 0.0));
    if (lane == 0) {
        const double a2 = h[k].re - ssum.re;
        sal = a2 > 0.0 ? sqrt(a2) : 0.0;
    }
    __syncthreads();
    finish_column(S, r, k - 1, h, sal, col, csl, snl);
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

namespace {
struct Ctx {
    vie_op op;
    hipStream_t s;
    long long n;  // 3N
    int R;
    int nbd, nbu;  // parts per vector of the dot products and of the updates
    c128 *partial;
    double *host;  // pinned scratch
    ActiveLines act;  // lines the basis passes cover (all when act.lines is null)
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

// One Arnoldi step of every active right-hand side (Sec. 1: GMRES; the orthogonalisation is this
// library's choice), column r at its own step jcol[r] with its ring starting in slot s0[r]:
// with z = P^{-1} u and w = A z formed, one reduction pass, the coefficients (completing each
// column's previous Hessenberg column), one update pass (q over u, the next u into next_slot and
// its complex64 copy when vlo is given), |u_next|^2 and the provisional residual estimates.
// max_j bounds jcol over the active columns.
template <class VT, class WT>
vie_status arnoldi_step(Ctx &C, VT *V, long long ldj, int m1, const int *jcol, const int *s0, int max_j,
                        int next_slot, const WT *w, GState &S, c64 *vlo) {
    hipStream_t s = C.s;
    const long long n = C.n;
    const int R = C.R, cnt = 2 * max_j + 3;
    {
        ProfScope ps("arnoldi_dots", s);
        hipLaunchKernelGGL((k_dots2<VT, WT>), dim3(C.nbd, R), dim3(KR_THREADS), 0, s, (const VT *)V, ldj, m1, jcol, s0, w, n,
                           (const int *)S.active, 0, cnt, C.partial, C.act);
        VIE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce, dim3(cnt, R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbd, cnt, S.h1,
                       S.hstride);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_arnoldi_coef, dim3(R), dim3(64), 0, s, S, jcol, R);
    VIE_HIP(hipGetLastError());
    {
        ProfScope ps("arnoldi_update", s);
        hipLaunchKernelGGL((k_update2<VT, WT>), dim3(C.nbu, R), dim3(KR_THREADS), 0, s, V, ldj, m1, jcol, s0, next_slot,
                           (const c128 *)S.coef, S.cstride, w, n, (const int *)S.active, vlo, C.partial, C.act);
        VIE_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce, dim3(1, R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbu, 1, S.nrm2, 1);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_arnoldi_est, dim3(R), dim3(64), 0, s, S, jcol, R);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// End of the cycles of the right-hand sides with jr[r] > 0 (max_jr the largest): the reduction of
// u_{jr} against q_0..q_{jr-1} in each one's ring, and its last column completed.
template <class VT>
vie_status arnoldi_finish(Ctx &C, const VT *V, long long ldj, int m1, const int *jr_dev, const int *s0,
                          int max_jr, GState &S) {
    hipStream_t s = C.s;
    const int cnt = max_jr + 1;
    hipLaunchKernelGGL((k_dots2<VT, c128>), dim3(C.nbd, C.R), dim3(KR_THREADS), 0, s, V, ldj, m1, jr_dev, s0,
                       (const c128 *)nullptr, C.n, (const int *)nullptr, 1, cnt, C.partial, C.act);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(cnt, C.R), dim3(KR_THREADS), 0, s, (const c128 *)C.partial, C.nbd, cnt, S.h1,
                       S.hstride);
    VIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_arnoldi_final, dim3(C.R), dim3(64), 0, s, S, jr_dev, C.R);
    VIE_HIP(hipGetLastError());
    return VIE_OK;
}

// Pinned host scratch of the solves (read-backs of norms and column states), kept for reuse per
// device: freeing pinned memory waits for the whole device, which would make every finishing
// solve wait for the work that concurrent solves have queued on other streams.
struct PinnedPool {
    std::mutex mu;
    std::vector<std::pair<int, std::pair<size_t, void *>>> idle;  // (device, (bytes, pointer))
};
static PinnedPool &pinned_pool() {
    static PinnedPool *p = new PinnedPool();  // never destroyed: the buffers live until exit
    return *p;
}
static vie_status pinned_get(size_t bytes, void **out, size_t *got) {
    int dev = 0;
    VIE_HIP(hipGetDevice(&dev));
    {
        PinnedPool &pp = pinned_pool();
        std::lock_guard<std::mutex> lk(pp.mu);
        for (size_t i = 0; i < pp.idle.size(); ++i)
            if (pp.idle[i].first == dev && pp.idle[i].second.first >= bytes) {
                *out = pp.idle[i].second.second;
                *got = pp.idle[i].second.first;
                pp.idle.erase(pp.idle.begin() + i);
                return VIE_OK;
            }
    }
    VIE_HIP(hipHostMalloc(out, bytes, hipHostMallocDefault));
    *got = bytes;
    return VIE_OK;
}
static void pinned_put(size_t bytes, void *p) {
    int dev = 0;
    if (!p || hipGetDevice(&dev) != hipSuccess) return;
    PinnedPool &pp = pinned_pool();
    std::lock_guard<std::mutex> lk(pp.mu);
    pp.idle.push_back({dev, {bytes, p}});
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
    return std::max((long long)kr_parts(n, KR_EPT_DOTS) * (2 * restart + 3), (long long)kr_parts(n, KR_EPT_UPD));
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
    const int m = o->restart, m1 = m + 1;
    const long long n = 3LL * op->N;
    const long long Rn = (long long)R * n;
    Ctx C{op, s, n, R, kr_parts(n, KR_EPT_DOTS), kr_parts(n, KR_EPT_UPD), nullptr, nullptr, ActiveLines{}};
    // Lines whose contrast vanishes along all of x: there the operator is the identity and the
    // solution equals b.  With x = b and r = 0 there from the start and every preconditioned
    // vector projected to zero there, every basis vector and every product is zero on those
    // lines (A z = z on them), so the basis passes skip them.
    const bool skip = op->n_line_zero > 0;
    const int *zero_lines = skip ? op->lines.as<const int>() + op->n_line_act : nullptr;
    if (skip) C.act = ActiveLines{op->lines.as<const int>(), op->n_line_act, op->nx};
    const unsigned gzl = (unsigned)std::min<long long>(1024, ((long long)op->n_line_zero * op->nx + KR_THREADS - 1) / KR_THREADS);
    // zero the skipped lines of `count` vectors of n elements from base (complex64 or complex128)
    auto zero_skipped = [&](void *base, bool c64v, long long count) -> vie_status {
        for (long long v0 = 0; v0 < count; v0 += 65535) {
            const unsigned gy = (unsigned)std::min<long long>(65535, count - v0);
            if (c64v)
                hipLaunchKernelGGL(k_zero_lines<c64>, dim3(gzl, gy), dim3(KR_THREADS), 0, s, (c64 *)base + v0 * n, n,
                                   zero_lines, op->n_line_zero, op->nx);
            else
                hipLaunchKernelGGL(k_zero_lines<c128>, dim3(gzl, gy), dim3(KR_THREADS), 0, s, (c128 *)base + v0 * n, n,
                                   zero_lines, op->n_line_zero, op->nx);
            VIE_HIP(hipGetLastError());
        }
        return VIE_OK;
    };
    // mixed: basis V and flexible basis Z in complex64, FP64 sums and w.  mixed_pc: V in
    // complex128 with a complex64 copy of its newest vector (vlo) for the preconditioner, Z in
    // complex64, each z_j widened (zw) for the complex128 product.  V is a ring of m + 1 slots
    // and Z one of m slots per right-hand side (see ring_slot).
    const bool v32 = mixed;
    const size_t vsz = v32 ? sizeof(c64) : sizeof(c128);
    const size_t zsz = lowpc ? sizeof(c64) : sizeof(c128);
    DevBuf Vb, Zb, wb, rb, part, small, w32, vlo, zw;
    VIE_CHECK(Vb.ensure(vsz * Rn * m1));
    VIE_CHECK(Zb.ensure(zsz * Rn * m));
    if (mixed_pc) {
        VIE_CHECK(vlo.ensure(sizeof(c64) * Rn));
        VIE_CHECK(zw.ensure(sizeof(c128) * Rn));
    }
    if (!mixed) VIE_CHECK(wb.ensure(sizeof(c128) * Rn));  // mixed: the Arnoldi passes read w32
    VIE_CHECK(rb.ensure(sizeof(c128) * Rn));
    VIE_CHECK(part.ensure(sizeof(c128) * (size_t)R * arnoldi_partials(n, m)));
    if (mixed) VIE_CHECK(w32.ensure(sizeof(c64) * Rn));
    DevBuf nzflag;
    // ring slots whose skipped lines are zero: a slot is zeroed there before its first use (slot
    // 0 now, every other one before the update pass that writes the next u into it), since the
    // passes write the covered lines only and the preconditioner reads whole vectors
    std::vector<char> vzero(m1, 0);
    auto zero_slot = [&](int slot) -> vie_status {
        if (!skip || vzero[slot]) return VIE_OK;
        vzero[slot] = 1;
        return zero_skipped((char *)Vb.p + vsz * Rn * slot, v32, R);
    };
    if (skip) {
        VIE_CHECK(zero_slot(0));
        if (mixed_pc) VIE_CHECK(zero_skipped(vlo.p, true, R));
        // the step products leave their outputs' skipped lines as they are
        if (mixed)
            VIE_CHECK(zero_skipped(w32.p, true, R));
        else
            VIE_CHECK(zero_skipped(wb.p, false, R));
        VIE_CHECK(nzflag.ensure(sizeof(int)));
    }
    GState S;
    S.m = m;
    S.hstride = 2 * m + 3;
    S.cstride = 2 * m + 3;
    constexpr int NI = 6;  // device int arrays of R: active, jcol, s0, z0, jend, mask
    size_t nc = (size_t)R * ((size_t)S.hstride + S.cstride + 1 + 2 * (size_t)m * (m + 1) + m + (m + 1) + m);
    size_t nd = (size_t)R * (2 * m + 4 + 1);
    VIE_CHECK(small.ensure(sizeof(c128) * nc + sizeof(double) * nd + sizeof(int) * NI * R));
    c128 *cp = small.as<c128>();
    S.h1 = cp;
    cp += (size_t)R * S.hstride;
    S.coef = cp;
    cp += (size_t)R * S.cstride;
    S.nrm2 = cp;
    cp += R;
    S.P = cp;
    cp += (size_t)R * m * (m + 1);
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
    S.sig = dp;
    dp += (size_t)R * m;
    S.beta = dp;
    dp += R;
    S.active = reinterpret_cast<int *>(dp);
    int *jcol_dev = S.active + R, *s0_dev = jcol_dev + R, *z0_dev = s0_dev + R, *jend_dev = z0_dev + R,
        *mask_dev = jend_dev + R;
    C.partial = part.as<c128>();
    double *host = nullptr;
    size_t host_bytes = 0;
    // pinned layout: doubles [0, 4R) | ints active, jcol, s0, z0, jend, mask [R each]
    VIE_CHECK(pinned_get(sizeof(double) * 4 * (size_t)R + sizeof(int) * NI * R + 64, (void **)&host, &host_bytes));
    struct HostPut {  // back to the pool once this solve's stream is done with it (a no-op wait
        double *p;    // on the normal path; an error return may leave a copy in flight)
        size_t n;
        hipStream_t st;
        ~HostPut() {
            (void)hipStreamSynchronize(st);
            pinned_put(n, p);
        }
    } hp{host, host_bytes, s};
    C.host = host;
    int *hact = reinterpret_cast<int *>(host + 4 * (size_t)R);
    int *hjcol = hact + R, *hs0 = hjcol + R, *hz0 = hs0 + R, *hjend = hz0 + R, *hmask = hjend + R;
    c128 *w = wb.as<c128>(), *r = rb.as<c128>();
    const long long ldj = Rn;  // stride between ring slots
    dim3 grid_e(1024, R);

    // Columns run their own restart cycles.  Without a hook (vie_solve) every column starts at
    // the first step, so all reach the end of a full cycle at the same step, and a column whose
    // estimate converges earlier waits for that common end: one batched true residual per cycle.
    // With a hook (the server) a column ends its cycle at the step its estimate converges, so
    // its request can complete there, and a freed slot takes a queued right-hand side at any step.
    const bool immediate = hook != nullptr;
    std::vector<double> nb(R), beta(R);
    std::vector<int> done(R, 0), act(R, 0), jr(R, 0), t0(R, 0), told(R, 0), pend(R, 0);
    vie_status result = VIE_OK;
    for (int q = 0; q < R; ++q) stats[q] = vie_solve_stats{0, 0, 0.0, VIE_OK};
    VIE_CHECK(norms(C, b, S.nrm2));
    VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
    for (int q = 0; q < R; ++q) nb[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
    for (int q = 0; q < R; ++q)
        if (!std::isfinite(nb[q])) {
            vie_set_error("non-finite right-hand side " + std::to_string(q));
            return VIE_ENONFINITE;
        }
    // x = b on the skipped lines of columns [c0, c0 + cnt), r = 0 there; true when b has an entry
    // there (then r on the other lines needs the product with x)
    auto identity_lines = [&](int c0, int cnt, bool *nonzero) -> vie_status {
        VIE_HIP(hipMemsetAsync(nzflag.p, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_identity_lines, dim3(gzl, cnt), dim3(KR_THREADS), 0, s, x, b, r, n, c0, zero_lines,
                           op->n_line_zero, op->nx, nzflag.as<int>());
        VIE_HIP(hipGetLastError());
        VIE_CHECK(read_host(C, nzflag.p, sizeof(int)));
        *nonzero = *reinterpret_cast<int *>(host) != 0;
        return VIE_OK;
    };
    if (o->x0_given) {
        bool nz = false;  // the product below forms r everywhere anyway
        if (skip) VIE_CHECK(identity_lines(0, R, &nz));
        VIE_CHECK(launch_matvec(op, x, r, R, VIE_C128, s));
        hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, Rn);
        VIE_HIP(hipGetLastError());
    } else {
        VIE_HIP(hipMemsetAsync(x, 0, sizeof(c128) * Rn, s));
        VIE_HIP(hipMemcpyAsync(r, b, sizeof(c128) * Rn, hipMemcpyDeviceToDevice, s));
        bool nz = false;
        if (skip) VIE_CHECK(identity_lines(0, R, &nz));
        if (nz) {
            VIE_CHECK(launch_matvec(op, x, r, R, VIE_C128, s));
            hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, Rn);
            VIE_HIP(hipGetLastError());
        }
    }
    VIE_CHECK(norms(C, r, S.nrm2));
    VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
    for (int q = 0; q < R; ++q) beta[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);

    // the true residual decides: converged, out of iterations, or another cycle
    auto judge = [&](int q) -> vie_status {
        if (!std::isfinite(beta[q])) {
            vie_set_error("non-finite residual for right-hand side " + std::to_string(q));
            return VIE_ENONFINITE;
        }
        const double rel = nb[q] > 0 ? beta[q] / nb[q] : 0.0;
        stats[q].relres = rel;
        if (nb[q] == 0.0 || rel <= o->tol) {
            done[q] = 1;
        } else if (stats[q].iters >= o->maxit) {
            done[q] = 1;
            stats[q].status = VIE_NOT_CONVERGED;
            result = VIE_NOT_CONVERGED;
        }
        return VIE_OK;
    };
    // hand out ended columns, take new right-hand sides into their slots (they join `starting`)
    auto run_hook = [&](std::vector<int> *starting) -> vie_status {
        std::vector<int> ended, refill;
        for (int q = 0; q < R; ++q)
            if (done[q] && !told[q]) {
                told[q] = 1;
                ended.push_back(q);
            }
        VIE_CHECK(hook->boundary(ended, stats, x, const_cast<c128 *>(b), s, &refill));
        if (refill.empty()) return VIE_OK;
        for (int q : refill) {
            VIE_HIP(hipMemsetAsync(x + (long long)q * n, 0, sizeof(c128) * n, s));
            VIE_HIP(hipMemcpyAsync(r + (long long)q * n, b + (long long)q * n, sizeof(c128) * n,
                                   hipMemcpyDeviceToDevice, s));
            bool nz = false;
            if (skip) VIE_CHECK(identity_lines(q, 1, &nz));
            if (nz) {
                VIE_CHECK(launch_matvec(op, x + (long long)q * n, r + (long long)q * n, 1, VIE_C128, s));
                hipLaunchKernelGGL(k_residual, dim3(256), dim3(256), 0, s, b + (long long)q * n, r + (long long)q * n, n);
                VIE_HIP(hipGetLastError());
            }
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
            if (nb[q] == 0.0)
                done[q] = 1;
            else
                starting->push_back(q);
        }
        return VIE_OK;
    };
    long long t = 0;  // global step: the ring slot of the step's input is t mod (m + 1)
    bool dirty = true;  // active / s0 changed since the last upload
    // u_0 = r / beta of each starting column into the slot of step t
    auto start_cycles = [&](const std::vector<int> &cols) -> vie_status {
        if (cols.empty()) return VIE_OK;
        const int slot = (int)(t % m1);
        for (int q = 0; q < R; ++q) {
            hmask[q] = 0;
            host[q] = beta[q];
        }
        for (int q : cols) {
            hmask[q] = 1;
            act[q] = 1;
            jr[q] = 0;
            t0[q] = (int)(t % ((long long)m * m1));  // s0 = t0 mod (m + 1), z0 = t0 mod m
            pend[q] = 0;
        }
        VIE_HIP(hipMemcpyAsync(S.beta, host, sizeof(double) * R, hipMemcpyHostToDevice, s));
        VIE_HIP(hipMemcpyAsync(mask_dev, hmask, sizeof(int) * R, hipMemcpyHostToDevice, s));
        c64 *vl = mixed_pc ? vlo.as<c64>() : nullptr;
        if (v32)
            hipLaunchKernelGGL(k_store<c64>, grid_e, dim3(256), 0, s, (const c128 *)r, Vb.as<c64>(), ldj, slot, vl, n,
                               (const double *)S.beta, (const int *)mask_dev);
        else
            hipLaunchKernelGGL(k_store<c128>, grid_e, dim3(256), 0, s, (const c128 *)r, Vb.as<c128>(), ldj, slot, vl, n,
                               (const double *)S.beta, (const int *)mask_dev);
        VIE_HIP(hipGetLastError());
        // the pinned arrays are reused only after the next read-back has synchronised the stream
        VIE_HIP(hipStreamSynchronize(s));
        dirty = true;
        return VIE_OK;
    };
    // end the cycles of `cols`: last columns completed, x += Z y, the FP64 true residual, judged
    auto end_cycles = [&](const std::vector<int> &cols, std::vector<int> *restart) -> vie_status {
        int max_jr = 0;
        for (int q = 0; q < R; ++q) {
            hjend[q] = 0;
            hz0[q] = t0[q] % m;
        }
        for (int q : cols) {
            hjend[q] = jr[q];
            max_jr = std::max(max_jr, jr[q]);
        }
        VIE_HIP(hipMemcpyAsync(jend_dev, hjend, sizeof(int) * R, hipMemcpyHostToDevice, s));
        VIE_HIP(hipMemcpyAsync(z0_dev, hz0, sizeof(int) * R, hipMemcpyHostToDevice, s));
        if (max_jr > 0) {
            if (v32)
                VIE_CHECK(arnoldi_finish<c64>(C, Vb.as<const c64>(), ldj, m1, jend_dev, s0_dev, max_jr, S));
            else
                VIE_CHECK(arnoldi_finish<c128>(C, Vb.as<const c128>(), ldj, m1, jend_dev, s0_dev, max_jr, S));
            hipLaunchKernelGGL(k_lsq, dim3((R + 63) / 64), dim3(64), 0, s, S, (const int *)jend_dev, R);
            VIE_HIP(hipGetLastError());
            if (lowpc)
                hipLaunchKernelGGL(k_combine<float>, grid_e, dim3(KR_THREADS), 0, s, Zb.as<const c64>(), ldj, m,
                                   (const int *)jend_dev, (const int *)z0_dev, (const c128 *)S.y, m, x, n);
            else
                hipLaunchKernelGGL(k_combine<double>, grid_e, dim3(KR_THREADS), 0, s, Zb.as<const c128>(), ldj, m,
                                   (const int *)jend_dev, (const int *)z0_dev, (const c128 *)S.y, m, x, n);
            VIE_HIP(hipGetLastError());
        }
        for (int q : cols) {
            if (jr[q] > 0) ++stats[q].restarts;
            act[q] = 0;
            pend[q] = 0;
        }
        dirty = true;
        // FP64 true residual r = b - A x of the ended columns (the whole batch when they are at
        // least half of it: the other columns' r is not needed before their own cycles end)
        if (2 * cols.size() >= (size_t)R) {
            VIE_CHECK(launch_matvec(op, x, r, R, VIE_C128, s));
            hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, s, b, r, Rn);
            VIE_HIP(hipGetLastError());
        } else {
            for (int q : cols) {
                VIE_CHECK(launch_matvec(op, x + (long long)q * n, r + (long long)q * n, 1, VIE_C128, s));
                hipLaunchKernelGGL(k_residual, dim3(256), dim3(256), 0, s, b + (long long)q * n, r + (long long)q * n,
                                   n);
                VIE_HIP(hipGetLastError());
            }
        }
        VIE_CHECK(norms(C, r, S.nrm2));
        VIE_CHECK(read_host(C, S.nrm2, sizeof(c128) * R));
        for (int q : cols) beta[q] = sqrt(reinterpret_cast<c128 *>(host)[q].re);
        for (int q : cols) {
            VIE_CHECK(judge(q));
            if (!done[q]) restart->push_back(q);
        }
        return VIE_OK;
    };

    std::vector<int> starting;
    for (int q = 0; q < R; ++q) {
        VIE_CHECK(judge(q));
        if (!done[q]) starting.push_back(q);
    }
    if (hook) VIE_CHECK(run_hook(&starting));
    VIE_CHECK(start_cycles(starting));
    for (;;) {
        int max_j = 0, nact = 0;
        for (int q = 0; q < R; ++q)
            if (act[q]) {
                ++nact;
                max_j = std::max(max_j, jr[q]);
            }
        if (nact == 0) break;
        for (int q = 0; q < R; ++q) hjcol[q] = jr[q];
        VIE_HIP(hipMemcpyAsync(jcol_dev, hjcol, sizeof(int) * R, hipMemcpyHostToDevice, s));
        if (dirty) {
            for (int q = 0; q < R; ++q) {
                hact[q] = act[q];
                hs0[q] = t0[q] % m1;
            }
            VIE_HIP(hipMemcpyAsync(S.active, hact, sizeof(int) * R, hipMemcpyHostToDevice, s));
            VIE_HIP(hipMemcpyAsync(s0_dev, hs0, sizeof(int) * R, hipMemcpyHostToDevice, s));
            dirty = false;
        }
        void *vj = (char *)Vb.p + vsz * Rn * (t % m1);
        void *zj = (char *)Zb.p + zsz * Rn * (t % m);
        // a preconditioner that does not keep the skipped lines at zero (one homogenising over y,
        // say) is projected: FGMRES takes any z, and A z then stays zero there.  One whose
        // identity rows include those lines copies the zeros of u_j there and is not.
        const bool project = skip && pc && !pc->zero_lines_kept;
        if (!lowpc) {
            if (pc)
                VIE_CHECK(pc_apply(pc, vj, zj, R, VIE_C128, s));
            else
                VIE_HIP(hipMemcpyAsync(zj, vj, sizeof(c128) * Rn, hipMemcpyDeviceToDevice, s));
            if (project) VIE_CHECK(zero_skipped(zj, false, R));
            VIE_CHECK(launch_matvec(op, zj, w, R, VIE_C128, s, skip));
        } else {
            const void *vin = mixed_pc ? vlo.p : vj;
            if (pc)
                VIE_CHECK(pc_apply(pc, vin, zj, R, VIE_C64, s));
            else
                VIE_HIP(hipMemcpyAsync(zj, vin, sizeof(c64) * Rn, hipMemcpyDeviceToDevice, s));
            if (project) VIE_CHECK(zero_skipped(zj, true, R));
            if (mixed) {
                VIE_CHECK(launch_matvec(op, zj, w32.p, R, VIE_C64, s, skip));  // read as is by the Arnoldi step
            } else {
                hipLaunchKernelGGL(k_widen, dim3(1024), dim3(256), 0, s, (const c64 *)zj, zw.as<c128>(), Rn);
                VIE_HIP(hipGetLastError());
                VIE_CHECK(launch_matvec(op, zw.p, w, R, VIE_C128, s, skip));
            }
        }
        c64 *vl = mixed_pc ? vlo.as<c64>() : nullptr;
        const int next_slot = (int)((t + 1) % m1);
        VIE_CHECK(zero_slot(next_slot));
        if (v32)
            VIE_CHECK((arnoldi_step<c64, c64>(C, Vb.as<c64>(), ldj, m1, jcol_dev, s0_dev, max_j, next_slot,
                                              w32.as<const c64>(), S, vl)));
        else
            VIE_CHECK((arnoldi_step<c128, c128>(C, Vb.as<c128>(), ldj, m1, jcol_dev, s0_dev, max_j, next_slot, w, S,
                                                vl)));
        VIE_CHECK(read_host(C, S.st, sizeof(double) * 4 * R));
        ++t;
        std::vector<int> ending;
        bool full = false;
        for (int q = 0; q < R; ++q) {
            if (!act[q]) continue;
            const double est = host[4 * q] / nb[q];
            if (!std::isfinite(est)) {
                vie_set_error("non-finite Arnoldi step for right-hand side " + std::to_string(q));
                return VIE_ENONFINITE;
            }
            ++stats[q].iters;
            ++jr[q];
            const bool stop = est <= o->tol || host[4 * q + 2] != 0.0 || stats[q].iters >= o->maxit;
            if (jr[q] == m) {
                ending.push_back(q);
                full = true;
            } else if (stop) {
                if (immediate) {
                    ending.push_back(q);
                } else {  // waits for the batch's common cycle end
                    pend[q] = 1;
                    act[q] = 0;
                    dirty = true;
                }
            }
        }
        if (!immediate) {
            int going = 0;
            for (int q = 0; q < R; ++q) going += act[q] && jr[q] < m;
            if (full || going == 0)
                for (int q = 0; q < R; ++q)
                    if (pend[q]) ending.push_back(q);
        }
        starting.clear();
        if (!ending.empty()) VIE_CHECK(end_cycles(ending, &starting));
        if (hook) {
            bool call = !ending.empty();
            for (int q = 0; q < R && !call; ++q) call = done[q] != 0;  // a free slot may take a joiner
            if (call) VIE_CHECK(run_hook(&starting));
        }
        VIE_CHECK(start_cycles(starting));
    }
    return result;
}
