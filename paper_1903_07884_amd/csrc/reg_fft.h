// Register-resident DFTs of small compile-time lengths.
//
// Dft<R, N, INV>::run(v) replaces v[0..N) by its DFT, v[k] <- sum_n v[n] W^{nk} with
// W = exp(-2 pi i / N) (INV: the conjugate; neither direction scales).  Lengths 2..5 are the
// butterflies of fft_device.h; a composite length N = A B runs B length-A DFTs over the
// stride-B subsequences, multiplies by W_N^{b k1} and finishes with A length-B DFTs (Cooley-
// Tukey decimation in time), every index and twiddle a compile-time constant, so the whole
// transform unrolls into straight-line code on registers.  The twiddle constants come from a
// constexpr evaluation of cos / sin (exact reduction of 2 pi q / n to a multiple of pi / 2 plus
// an angle of at most pi / 4, then the Taylor series), correct to about one unit in the last
// place of a double.
#pragma once

#include <utility>

#include "fft_device.h"

namespace rfft {

// ---------------------------------------------------------------- compile-time loops
template <class F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N-1
template <int N, class F>
__host__ __device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Workgroup barrier that orders LDS accesses only: global loads and stores issued before it
// stay in flight (for kernels whose workgroups exchange nothing through global memory).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- constexpr cos / sin
constexpr double kQuarterPi = 0.78539816339744830961566084581987572;

constexpr double taylor_sin(double x) {  // |x| <= pi / 4
    double term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {  // |x| <= pi / 4
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

struct CS {
    double c, s;
};

// cos and sin of 2 pi q / n.  The angle is (pi / 4) (8 t / n) with t = q mod n; with octant
// o = floor(8 t / n) it is j (pi / 2) + a for j = o / 2 and a = (pi / 4)(8 t - o n) / n when o
// is even, j = (o + 1) / 2 and a = -(pi / 4)((o + 1) n - 8 t) / n when o is odd; |a| <= pi / 4
// and the quarter turns j are exact.
constexpr CS cos_sin_2pi(long long q, long long n) {
    long long t = q % n;
    if (t < 0) t += n;
    const long long o = (8 * t) / n;
    long long j = 0;
    double a = 0.0;
    if (o % 2 == 0) {
        j = o / 2;
        a = kQuarterPi * (double)(8 * t - o * n) / (double)n;
    } else {
        j = (o + 1) / 2;
        a = -kQuarterPi * (double)((o + 1) * n - 8 * t) / (double)n;
    }
    const double ca = taylor_cos(a), sa = taylor_sin(a);
    switch (j % 4) {
        case 0: return CS{ca, sa};
        case 1: return CS{-sa, ca};
        case 2: return CS{-ca, -sa};
        default: return CS{sa, -ca};
    }
}

// W_N^Q = exp(-2 pi i Q / N) (INV: exp(+2 pi i Q / N)) as a constant.
template <class R, int N, int Q, bool INV>
__host__ __device__ __forceinline__ cpx<R> tw() {
    constexpr CS cs = cos_sin_2pi(Q, N);
    return mk<R>((R)cs.c, INV ? (R)cs.s : (R)-cs.s);
}

// a * W_N^Q with the exact cases (quarter turns) done without multiplications.
template <class R, int N, int Q, bool INV>
__host__ __device__ __forceinline__ cpx<R> twmul(cpx<R> a) {
    constexpr int q = Q % N;
    if constexpr (q == 0) {
        return a;
    } else if constexpr (4 * q == N) {  // -i (INV: +i)
        return INV ? mk(-a.im, a.re) : mk(a.im, -a.re);
    } else if constexpr (2 * q == N) {
        return mk(-a.re, -a.im);
    } else if constexpr (4 * q == 3 * N) {  // +i (INV: -i)
        return INV ? mk(a.im, -a.re) : mk(-a.im, a.re);
    } else {
        return a * tw<R, N, q, INV>();
    }
}

// ---------------------------------------------------------------- DFTs
template <class R, int N, bool INV>
struct Dft;

template <class R, bool INV>
struct Dft<R, 1, INV> {
    static __host__ __device__ __forceinline__ void run(cpx<R> *) {}
};
template <class R, bool INV>
struct Dft<R, 2, INV> {
    static __host__ __device__ __forceinline__ void run(cpx<R> *v) { bfly2(v); }
};
template <class R, bool INV>
struct Dft<R, 3, INV> {
    static __host__ __device__ __forceinline__ void run(cpx<R> *v) { bfly3(v, INV); }
};
template <class R, bool INV>
struct Dft<R, 4, INV> {
    static __host__ __device__ __forceinline__ void run(cpx<R> *v) { bfly4(v, INV); }
};
template <class R, bool INV>
struct Dft<R, 5, INV> {
    static __host__ __device__ __forceinline__ void run(cpx<R> *v) { bfly5(v, INV); }
};

constexpr bool smooth235(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

// first factor of a composite length (4 before 2, then 3, 5)
constexpr int first_factor(int n) { return n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : 5; }

template <class R, int N, bool INV>
struct Dft {
    static_assert(smooth235(N), "lengths with prime factors 2, 3 and 5 only");
    static constexpr int A = first_factor(N), B = N / A;
    static __host__ __device__ __forceinline__ void run(cpx<R> *v) {
        cpx<R> u[N];
        // B DFTs of length A over the subsequences v[b + B a]; twiddle W_N^{b k1}
        sfor<B>([&](auto bi) {
            constexpr int b = decltype(bi)::value;
            cpx<R> t[A];
            sfor<A>([&](auto ai) { t[decltype(ai)::value] = v[b + B * decltype(ai)::value]; });
            Dft<R, A, INV>::run(t);
            sfor<A>([&](auto ki) {
                constexpr int k1 = decltype(ki)::value;
                u[b * A + k1] = twmul<R, N, (b * k1) % N, INV>(t[k1]);
            });
        });
        // A DFTs of length B over b: output k1 + A k2
        sfor<A>([&](auto ki) {
            constexpr int k1 = decltype(ki)::value;
            cpx<R> t[B];
            sfor<B>([&](auto bi) { t[decltype(bi)::value] = u[decltype(bi)::value * A + k1]; });
            Dft<R, B, INV>::run(t);
            sfor<B>([&](auto k2) { v[k1 + A * decltype(k2)::value] = t[decltype(k2)::value]; });
        });
    }
};

// ---------------------------------------------------------------- line transforms
// Register Stockham transform of one line per workgroup, length L = R1 R2 R3 R4 fixed at
// compile time (radices <= 16, trailing 1s unused), on T = L / max radix threads.  Step s
// (radix Rs, Ns = R1..R(s-1)) takes butterfly j in [0, L/Rs): inputs j + r L/Rs, times
// W_L^{r k L/(Ns Rs)} with k = j mod Ns (table tw of W_L^q), a length-Rs DFT on registers,
// outputs (j / Ns) Ns Rs + k + r Ns.  The first step reads the line through ld(i), the last
// writes it through st(i, v), both in natural order and coalesced (consecutive threads take
// consecutive i); the steps between exchange through one LDS line of L entries (every thread
// reads its inputs, barrier, writes its outputs).
template <int R1, int R2, int R3, int R4>
struct Radices {
    static constexpr int L = R1 * R2 * R3 * R4;
    static constexpr int RMAX = R1 > R2 ? (R1 > R3 ? (R1 > R4 ? R1 : R4) : (R3 > R4 ? R3 : R4))
                                        : (R2 > R3 ? (R2 > R4 ? R2 : R4) : (R3 > R4 ? R3 : R4));
    static constexpr int T = L / RMAX;  // threads
    static constexpr int NSTEP = 1 + (R2 > 1) + (R3 > 1) + (R4 > 1);
};

// One step: SRC / DST 0 = LDS line, 1 = device memory (through the ld / st callbacks).
template <class R, int L, int RS, int NS, int T, bool INV, class Ld, class St>
__device__ __forceinline__ void xstep(const cpx<R> *__restrict__ tw, Ld ld, St st, bool sync_between) {
    constexpr int NB = L / RS, BPT = NB / T;
    static_assert(NB % T == 0, "whole butterflies per thread");
    cpx<R> v[BPT][RS];
    const int t = threadIdx.x;
    sfor<BPT>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int j = t + b * T;
        sfor<RS>([&](auto rc) { v[b][decltype(rc)::value] = ld(j + decltype(rc)::value * NB); });
        if constexpr (NS > 1) {
            const int k = j % NS;
            sfor<RS - 1>([&](auto rc) {
                constexpr int r = decltype(rc)::value + 1;
                const cpx<R> w = tw[r * k * (L / (NS * RS))];
                v[b][r] = v[b][r] * (INV ? conjg(w) : w);
            });
        }
        Dft<R, RS, INV>::run(v[b]);
    });
    if (sync_between) lds_barrier();
    sfor<BPT>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        const int j = t + b * T, k = j % NS, base = (j / NS) * NS * RS + k;
        sfor<RS>([&](auto rc) { st(base + decltype(rc)::value * NS, v[b][decltype(rc)::value]); });
    });
}


// The whole transform of one line (see above); vie_smem holds the LDS line.
template <class R, int R1, int R2, int R3, int R4, bool INV, class Ld, class St>
__device__ __forceinline__ void reg_line(const cpx<R> *__restrict__ tw, Ld ld_first, St st_last) {
    typedef Radices<R1, R2, R3, R4> RD;
    constexpr int L = RD::L, T = RD::T;
    cpx<R> *S = reinterpret_cast<cpx<R> *>(vie_smem);
    auto ld_lds = [&](int i) -> cpx<R> { return S[i]; };
    auto st_lds = [&](int i, cpx<R> v) { S[i] = v; };
    constexpr int N2 = R1, N3 = R1 * R2, N4 = R1 * R2 * R3;
    if constexpr (RD::NSTEP == 2) {
        xstep<R, L, R1, 1, T, INV>(tw, ld_first, st_lds, false);
        lds_barrier();
        xstep<R, L, R2, N2, T, INV>(tw, ld_lds, st_last, false);
    } else if constexpr (RD::NSTEP == 3) {
        xstep<R, L, R1, 1, T, INV>(tw, ld_first, st_lds, false);
        lds_barrier();
        xstep<R, L, R2, N2, T, INV>(tw, ld_lds, st_lds, true);
        lds_barrier();
        xstep<R, L, R3, N3, T, INV>(tw, ld_lds, st_last, false);
    } else {
        xstep<R, L, R1, 1, T, INV>(tw, ld_first, st_lds, false);
        lds_barrier();
        xstep<R, L, R2, N2, T, INV>(tw, ld_lds, st_lds, true);
        lds_barrier();
        xstep<R, L, R3, N3, T, INV>(tw, ld_lds, st_lds, true);
        lds_barrier();
        xstep<R, L, R4, N4, T, INV>(tw, ld_lds, st_last, false);
    }
}

}  // namespace rfft
