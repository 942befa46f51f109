// LDS-resident Stockham FFT used by the matvec and preconditioner kernels.
//
// A transform of length L = p_1 p_2 ... p_s runs s stages.  Stage t (radix p,
// Ns = p_1 ... p_{t-1}) reads butterfly j's inputs src[j + r L/p], multiplies
// input r by W_L^{r k L/(Ns p)} with k = j mod Ns, applies a length-p DFT and
// writes output r to dst[(j / Ns) Ns p + k + r Ns]; after the last stage the
// result is in natural order (autosort), so no bit reversal is needed.
// Forward uses W_L = exp(-2 pi i / L), inverse its conjugate; neither scales.
#pragma once

#include "vie_internal.h"

template <class R>
struct TwTable;
template <>
struct TwTable<double> {
    static __host__ __device__ __forceinline__ const c128 *get(const FftPlan &p) { return p.tw64; }
};
template <>
struct TwTable<float> {
    static __host__ __device__ __forceinline__ const c64 *get(const FftPlan &p) { return p.tw32; }
};

// Lines addressed inside LDS: line l starts at (l % nl1) * s1 + (l / nl1) * s2,
// element i of a line sits at start + i * es.
struct LdsLines {
    int nl1, s1, s2, es, nlines;
};

template <class R>
__device__ __forceinline__ cpx<R> tw_at(const cpx<R> *tw, int q, bool inv) {
    cpx<R> w = tw[q];
    if (inv) w.im = -w.im;
    return w;
}

template <class R>
__host__ __device__ __forceinline__ void bfly2(cpx<R> *v) {
    cpx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <class R>
__host__ __device__ __forceinline__ void bfly4(cpx<R> *v, bool inv) {
    cpx<R> s02 = v[0] + v[2], d02 = v[0] - v[2];
    cpx<R> s13 = v[1] + v[3], d13 = v[1] - v[3];
    // forward: -i * d13 ; inverse: +i * d13
    cpx<R> rot = inv ? mk(-d13.im, d13.re) : mk(d13.im, -d13.re);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + rot;
    v[3] = d02 - rot;
}

template <class R>
__host__ __device__ __forceinline__ void bfly3(cpx<R> *v, bool inv) {
    const R h = R(0.8660254037844386467637231707529362);  // sqrt(3)/2
    cpx<R> s = v[1] + v[2], d = v[1] - v[2];
    cpx<R> t = mk(v[0].re - R(0.5) * s.re, v[0].im - R(0.5) * s.im);
    // forward: y1 = t - i h d, y2 = t + i h d
    R sg = inv ? R(-1) : R(1);
    cpx<R> u = mk(sg * h * d.im, -sg * h * d.re);  // -i*sg*h*d
    v[0] = v[0] + s;
    v[1] = t + u;
    v[2] = t - u;
}

template <class R>
__host__ __device__ __forceinline__ void bfly5(cpx<R> *v, bool inv) {
    const R c1 = R(0.3090169943749474241022934171828191);
    const R c2 = R(-0.8090169943749474241022934171828191);
    const R s1 = R(0.9510565162951535721164393333793821);
    const R s2 = R(0.5877852522924731291687059546390728);
    R sg = inv ? R(-1) : R(1);
    cpx<R> b1 = v[1] + v[4], b2 = v[2] + v[3];
    cpx<R> d1 = v[1] - v[4], d2 = v[2] - v[3];
    cpx<R> a0 = v[0];
    cpx<R> p1 = mk(a0.re + c1 * b1.re + c2 * b2.re, a0.im + c1 * b1.im + c2 * b2.im);
    cpx<R> p2 = mk(a0.re + c2 * b1.re + c1 * b2.re, a0.im + c2 * b1.im + c1 * b2.im);
    cpx<R> q1 = mk(s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im);
    cpx<R> q2 = mk(s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im);
    // -i*sg*q
    cpx<R> m1 = mk(sg * q1.im, -sg * q1.re);
    cpx<R> m2 = mk(sg * q2.im, -sg * q2.re);
    v[0] = a0 + b1 + b2;
    v[1] = p1 + m1;
    v[4] = p1 - m1;
    v[2] = p2 + m2;
    v[3] = p2 - m2;
}

// One Stockham stage over all lines; src -> dst (both LDS).
template <class R, int P>
__device__ __forceinline__ void stage_fixed(const cpx<R> *src, cpx<R> *dst, const LdsLines &ln, int L,
                                            int Ns, const cpx<R> *tw, bool inv) {
    const int nb = L / P;
    const int total = nb * ln.nlines;
    const int twstep = L / (Ns * P);
    const FastDiv fnb(nb), fnl(ln.nl1), fns(Ns);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int l = fnb.div(t), j = t - l * nb;
        const int l2 = fnl.div(l);
        const int base = (l - l2 * ln.nl1) * ln.s1 + l2 * ln.s2;
        const int jn = fns.div(j), k = j - jn * Ns;
        cpx<R> v[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            cpx<R> a = src[base + (j + r * nb) * ln.es];
            v[r] = (r == 0 || k == 0) ? a : a * tw_at(tw, r * k * twstep, inv);
        }
        if (P == 2) bfly2(v);
        if (P == 3) bfly3(v, inv);
        if (P == 4) bfly4(v, inv);
        if (P == 5) bfly5(v, inv);
        const int d = jn * Ns * P + k;
#pragma unroll
        for (int r = 0; r < P; ++r) dst[base + (d + r * Ns) * ln.es] = v[r];
    }
}

// Generic prime radix: out[s] = sum_r src[j + r L/p] W_L^{r (k + s Ns) L/(Ns p)}.
template <class R>
__device__ void stage_generic(const cpx<R> *src, cpx<R> *dst, const LdsLines &ln, int L, int Ns, int P,
                              const cpx<R> *tw, bool inv) {
    const int nb = L / P;
    const int total = nb * ln.nlines * P;
    const int step = L / (Ns * P);
    const FastDiv fp(P), fnb(nb), fnl(ln.nl1), fns(Ns);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int u = fp.div(t), s = t - u * P;
        const int l = fnb.div(u), j = u - l * nb;
        const int l2 = fnl.div(l);
        const int base = (l - l2 * ln.nl1) * ln.s1 + l2 * ln.s2;
        const int jn = fns.div(j), k = j - jn * Ns;
        int e = (k + s * Ns) * step;  // < L
        cpx<R> acc = czero<R>();
        int q = 0;
        for (int r = 0; r < P; ++r) {
            acc = acc + src[base + (j + r * nb) * ln.es] * tw_at(tw, q, inv);
            q += e;
            if (q >= L) q -= L;
        }
        const int d = jn * Ns * P + k;
        dst[base + (d + s * Ns) * ln.es] = acc;
    }
}

// Transform all lines of `a`; `b` is a same-shaped scratch buffer.  Returns the
// buffer holding the result.  Caller must __syncthreads() before (data ready).
template <class R>
__device__ cpx<R> *fft_lds(cpx<R> *a, cpx<R> *b, const LdsLines &ln, const FftPlan &plan, bool inv) {
    const cpx<R> *tw = TwTable<R>::get(plan);
    const int L = plan.L;
    int Ns = 1;
    cpx<R> *src = a, *dst = b;
    for (int st = 0; st < plan.nrad; ++st) {
        int P = plan.rad[st];
        switch (P) {
            case 2: stage_fixed<R, 2>(src, dst, ln, L, Ns, tw, inv); break;
            case 3: stage_fixed<R, 3>(src, dst, ln, L, Ns, tw, inv); break;
            case 4: stage_fixed<R, 4>(src, dst, ln, L, Ns, tw, inv); break;
            case 5: stage_fixed<R, 5>(src, dst, ln, L, Ns, tw, inv); break;
            default: stage_generic<R>(src, dst, ln, L, Ns, P, tw, inv); break;
        }
        __syncthreads();
        Ns *= P;
        cpx<R> *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// In-place variant for radices 2..5: each thread keeps the inputs of up to FFT_BPT
// butterflies in registers across a barrier, so one LDS buffer suffices (long lines).
// Requires (L / smallest radix) * nlines <= FFT_BPT * blockDim.x.
#define FFT_BPT 4  // largest number of butterflies per thread an in-place transform may need
template <class R, int P, int BPT>
__device__ __forceinline__ void stage_inplace(cpx<R> *buf, const LdsLines &ln, int L, int Ns, const cpx<R> *tw,
                                              bool inv) {
    const int nb = L / P;
    const int total = nb * ln.nlines;
    const int twstep = L / (Ns * P);
    const FastDiv fnb(nb), fnl(ln.nl1), fns(Ns);
    cpx<R> v[BPT][P];
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        int t = threadIdx.x + q * blockDim.x;
        if (t < total) {
            const int l = fnb.div(t), j = t - l * nb;
            const int l2 = fnl.div(l);
            const int base = (l - l2 * ln.nl1) * ln.s1 + l2 * ln.s2;
            const int k = j - fns.div(j) * Ns;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                cpx<R> a = buf[base + (j + r * nb) * ln.es];
                v[q][r] = (r == 0 || k == 0) ? a : a * tw_at(tw, r * k * twstep, inv);
            }
            if (P == 2) bfly2(v[q]);
            if (P == 3) bfly3(v[q], inv);
            if (P == 4) bfly4(v[q], inv);
            if (P == 5) bfly5(v[q], inv);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        int t = threadIdx.x + q * blockDim.x;
        if (t < total) {
            const int l = fnb.div(t), j = t - l * nb;
            const int l2 = fnl.div(l);
            const int base = (l - l2 * ln.nl1) * ln.s1 + l2 * ln.s2;
            const int jn = fns.div(j), k = j - jn * Ns;
            const int d = jn * Ns * P + k;
#pragma unroll
            for (int r = 0; r < P; ++r) buf[base + (d + r * Ns) * ln.es] = v[q][r];
        }
    }
    __syncthreads();
}

__host__ __device__ inline bool fft_plan_inplace(const FftPlan &plan) {
    if (plan.L > 2 * FFT_BPT * 1024) return false;  // radix-2 stage must fit 1024 threads
    for (int i = 0; i < plan.nrad; ++i)
        if (plan.rad[i] > 5) return false;
    return true;
}

// Transform in place (plans with radices <= 5 only); caller syncs before.  BPT butterflies
// per thread at most: (L / smallest radix) * nlines <= BPT * blockDim.x.
template <class R, int BPT>
__device__ void fft_lds_inplace(cpx<R> *buf, const LdsLines &ln, const FftPlan &plan, bool inv) {
    const cpx<R> *tw = TwTable<R>::get(plan);
    const int L = plan.L;
    int Ns = 1;
    for (int st = 0; st < plan.nrad; ++st) {
        int P = plan.rad[st];
        switch (P) {
            case 2: stage_inplace<R, 2, BPT>(buf, ln, L, Ns, tw, inv); break;
            case 3: stage_inplace<R, 3, BPT>(buf, ln, L, Ns, tw, inv); break;
            case 4: stage_inplace<R, 4, BPT>(buf, ln, L, Ns, tw, inv); break;
            default: stage_inplace<R, 5, BPT>(buf, ln, L, Ns, tw, inv); break;
        }
        Ns *= P;
    }
}

// One line per workgroup.  Ping-pong (2 L of LDS, no register staging) when both buffers fit
// in FFT_PINGPONG_LDS bytes, otherwise in place (L of LDS; plans with radices <= 5).
#define FFT_PINGPONG_LDS 65536
__host__ __device__ inline bool fft_line_inplace(const FftPlan &plan, size_t esz) {
    return 2 * esz * (size_t)plan.L > FFT_PINGPONG_LDS && fft_plan_inplace(plan);
}

template <class R, int BPT>
__device__ __forceinline__ cpx<R> *fft_line(cpx<R> *a, const FftPlan &plan, bool inv) {
    LdsLines ln = {1, 0, 0, 1, 1};
    if (BPT > 0 && fft_line_inplace(plan, sizeof(cpx<R>))) {
        fft_lds_inplace<R, (BPT > 0 ? BPT : 1)>(a, ln, plan, inv);
        return a;
    }
    return fft_lds<R>(a, a + plan.L, ln, plan, inv);
}

// Host: expand X(B) for the butterflies-per-thread value fft_line_shape selected.
#define VIE_BPT_SWITCH(bpt, X) \
    do {                         \
        if ((bpt) == 0) {        \
            X(0);                \
        } else if ((bpt) == 2) { \
            X(2);                \
        } else {                 \
            X(4);                \
        }                        \
    } while (0)

// Launch shape of a one-line-per-workgroup transform: threads, LDS bytes and the
// butterflies-per-thread template argument (0 = ping-pong).  t_req > 0 asks for that many
// threads (a multiple of 64, <= 1024); returns false if an in-place transform would then
// need more than 4 butterflies per thread.
inline bool fft_line_shape(const FftPlan &plan, size_t esz, int *threads, size_t *lds, int *bpt, int t_req = 0) {
    int L = plan.L;
    int t = 64;
    while (t < 256 && t * 4 < L) t *= 2;
    if (fft_line_inplace(plan, esz)) {
        t = 64;
        while (t < 1024 && (long long)t * 2 * 2 < L) t *= 2;  // radix-2 stage with 2 per thread
        if (t_req > 0) t = t_req;
        int b = 2;
        while ((long long)t * b * 2 < L) b *= 2;
        *bpt = b;
        *lds = esz * (size_t)L;
        *threads = t;
        return b <= 4;
    }
    if (t_req > 0) t = t_req;
    *bpt = 0;
    *lds = 2 * esz * (size_t)L;
    *threads = t;
    return true;
}

extern __shared__ __align__(16) unsigned char vie_smem[];
