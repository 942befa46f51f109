// Internal declarations shared by the HIP translation units of libvie.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vie.h"

// ---------------------------------------------------------------- complex
template <class R>
struct alignas(2 * sizeof(R)) cpx {
    R re, im;
};
typedef cpx<double> c128;
typedef cpx<float> c64;

template <class R>
__host__ __device__ __forceinline__ cpx<R> mk(R a, R b) {
    cpx<R> z;
    z.re = a;
    z.im = b;
    return z;
}
template <class R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <class R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <class R>
__host__ __device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R>
__host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return mk(s * a.re, s * a.im); }
template <class R>
__host__ __device__ __forceinline__ cpx<R> conjg(cpx<R> a) { return mk(a.re, -a.im); }
// conj(a) * b
template <class R>
__host__ __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class R>
__host__ __device__ __forceinline__ R abs2(cpx<R> a) { return a.re * a.re + a.im * a.im; }
// a + b*c as four fused multiply-adds (the sum of a product into an accumulator without the
// separate rounding of the product)
__host__ __device__ __forceinline__ float rfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double rfma(double a, double b, double c) { return fma(a, b, c); }
template <class R>
__host__ __device__ __forceinline__ cpx<R> cfma(cpx<R> a, cpx<R> b, cpx<R> c) {
    return mk<R>(rfma(-b.im, c.im, rfma(b.re, c.re, a.re)), rfma(b.im, c.re, rfma(b.re, c.im, a.im)));
}
// a - b*c
template <class R>
__host__ __device__ __forceinline__ cpx<R> cfms(cpx<R> a, cpx<R> b, cpx<R> c) {
    return mk(a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re);
}
template <class R>
__host__ __device__ __forceinline__ cpx<R> cdiv(cpx<R> a, cpx<R> b) {
    R d = b.re * b.re + b.im * b.im;
    return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
template <class R>
__host__ __device__ __forceinline__ cpx<R> czero() { return mk<R>(R(0), R(0)); }

// Complex bfloat16 (stored preconditioner factors): real part in the low 16 bits, imaginary
// part in the high 16 bits; bfloat16 = the upper half of an IEEE binary32.
struct bf16c {
    uint32_t v;
};
// Load a stored factor entry as working precision (identity for complex float/double).
template <class R>
__device__ __forceinline__ cpx<R> ldf(const cpx<R> *p) {
    return *p;
}
__device__ __forceinline__ c64 ldf(const bf16c *p) {
    const uint32_t v = p->v;
    return mk(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
}
// Round a float to bfloat16, to nearest with ties to even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// Division of small non-negative ints (numerator < 2^20) by a runtime divisor: a float
// reciprocal estimate and one correction step each way replace the integer division sequence.
struct FastDiv {
    int d;
    float inv;
    __device__ __forceinline__ explicit FastDiv(int dd) : d(dd), inv(__builtin_amdgcn_rcpf((float)dd)) {}
    __device__ __forceinline__ int div(int a) const {
        int q = (int)((float)a * inv);
        const int r = a - q * d;
        if (r >= d) ++q;
        else if (r < 0) --q;
        return q;
    }
};

// ---------------------------------------------------------------- errors
void vie_set_error(const std::string &msg);

#define VIE_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            vie_set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
            return (e_ == hipErrorOutOfMemory) ? VIE_EOOM : VIE_EDEVICE;               \
        }                                                                               \
    } while (0)

#define VIE_CHECK(st)                      \
    do {                                   \
        vie_status s_ = (st);              \
        if (s_ < 0) return s_;             \
    } while (0)

// device buffer owned by a handle
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    vie_status ensure(size_t nbytes);  // grow (contents not preserved)
    void release();
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

// The stream of the library call in progress on this thread: buffers released during it are
// handed out again only after the work queued on it so far has finished.
// Before a stream created by the library is destroyed: the pool waits for the blocks released
// on it and drops their events.
void pool_stream_retired(hipStream_t s);

struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
};

// LDS bytes a workgroup may use on the current device (api.cpp).
size_t max_lds();

// Allow a kernel to request more than the default dynamic LDS.
inline void vie_lds_attr(const void *kernel, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------- FFT plans
// A length-L transform factored into radices (applied first to last).
// Twiddles: table of W_L^q = exp(-2 pi i q / L), q in [0, L), complex double
// (a complex float copy for single precision).
#define VIE_MAX_RADICES 24
struct FftPlan {
    int L = 0;
    int nrad = 0;
    int rad[VIE_MAX_RADICES];
    const c128 *tw64 = nullptr;  // device
    const c64 *tw32 = nullptr;   // device
};

// Owns device twiddle tables, keyed by length.
struct FftCache {
    struct Entry {
        int L;
        DevBuf t64, t32;
    };
    std::vector<Entry *> entries;
    vie_status get(int L, FftPlan *plan);
    ~FftCache();
};

bool fft_supported_length(int L);  // every prime factor <= VIE_FFT_MAX_PRIME
#define VIE_FFT_MAX_PRIME 61
int fft_good_length(int minL);     // smallest 2^a 3^b 5^c >= minL

// ---------------------------------------------------------------- handles
// A handle is read-only once built, so calls on different streams may share it.  What a call
// writes (intermediate spectra, schedules, flags, tuned launch parameters) lives in a workspace
// per (handle, stream): created on the stream's first call, kept until the handle is destroyed.
// Calls on one stream hold its workspace's lock, so host threads sharing a stream take turns
// (as the stream itself orders their work).
template <class W>
struct WsTable {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, std::unique_ptr<W>>> v;
    W *get(hipStream_t s) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &e : v)
            if (e.first == s) return e.second.get();
        v.emplace_back(s, std::unique_ptr<W>(new W()));
        return v.back().second.get();
    }
    // Return stream s's scratch (its buffers go back to the cache of released blocks, reusable
    // once the work queued on s so far is done).  No call may be using it on s.
    void drop(hipStream_t s) {
        std::unique_ptr<W> gone;
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].first == s) {
                gone = std::move(v[i].second);
                v.erase(v.begin() + (long)i);
                break;
            }
    }
};

// Operator product scratch of one stream.
struct OpWs {
    std::mutex mu;
    DevBuf ybuf;             // split plane pass: y-spectra and coupled y-spectra, 2 x nrhs*Px*3nz*Py
    DevBuf work;             // x-spectra, nrhs*3*ny*nz*Px complex
    // FFT launch parameters per vector precision (0 = default; autotuned for tuned_nrhs)
    int cfg_plane_thr[2] = {0, 0}, cfg_x_thr[2] = {0, 0}, tuned_nrhs[2] = {-1, -1};
};

// Preconditioner apply scratch of one stream.
struct PcWs {
    std::mutex mu;
    DevBuf work;             // apply intermediate: nrhs * nboxes * m * modes complex (vector prec)
    DevBuf workc;            // x-DFT of the identity rows, nrhs * nboxes * (m_full - m) * bx
    DevBuf cflag;            // int32: epoch of the last apply whose identity rows held input
    uint32_t epoch = 0;
    DevBuf work1;            // 2-level: x-DFT lines of the full cross-section before the y-DFT
    // block-solve schedule for sched_nrhs right-hand sides
    int sched_nrhs = 0, n_wide = 0, n_narrow = 0, wide_ct = 1, narrow_rc = 1;
    DevBuf sched;            // int4 wide items [n_wide], then int4 narrow items of narrow_rc columns
                             // (m <= 64: of 64/m columns)
    DevBuf wide_scratch;     // wide-solve tiles: n_wide * m * 16*wide_ct complex
    DevBuf wide_bf16;        // bfloat16 hi + lo split of the solved rows (BF16 factors)
    // block-solve launch parameters (defaults or autotuned for tuned_nrhs right-hand sides)
    int cfg_gmax = 0;        // widest column group of the wide solve (0: widest giving >= 512 groups)
    int cfg_nw = 0;          // wavefronts per wide workgroup (0: 16 for FP32, 8 for FP64)
    int cfg_rc = 0;          // columns per narrow workgroup (0: register-budget rule)
    int cfg_min_rhs = 8;     // blocks go wide from this many right-hand sides on
    int tuned_nrhs = -1;
};

struct vie_op_s {
    int nx, ny, nz;
    long long N;             // nx*ny*nz
    double delta, kb, kappa;
    int Px, Py, Pz;          // circulant embedding periods (>= 2n - 1, 2-3-5 smooth)
    int Hx, Hy, Hz;          // octant extents Px/2+1 ...
    DevBuf M64, M32;         // contrast per voxel (c128 / c64)
    DevBuf gen;              // FP64 octant generator [6][nz][ny][nx]
    DevBuf khat64, khat32;   // octant kernel transform [Hx][Hz][Hy][6] scaled by 1/(Px Py Pz), or with
                             // direct_z the (x, y)-transform [Hx][Hy][nz][6] scaled by 1/(Px Py)
    bool has_c64 = false;
    bool direct_z = false;   // kernel transform along x, y only; z handled as a direct Toeplitz sum
    bool split_plane = false; // direct z, but the (y, z) plane exceeds one workgroup's LDS: the plane
                             // pass runs as y-FFT, z coupling and inverse y-FFT through ybuf
    FftCache fft;
    FftPlan px, py, pz;      // plans for the three periods
    // x lines too long for one workgroup's LDS: four-step transform Px = L1 * L2 (xsplit = L2,
    // plans of L1 = px1.L and L2 = px2.L); x-frequency kx then sits at (kx mod L2) L1 + kx / L2
    int xsplit = 1;
    FftPlan px1, px2;
    WsTable<OpWs> ws;        // product scratch per stream
    // x-lines (component, z, y) of the vectors (layout [c][z][y][x]): on a line whose contrast is
    // zero at every x the operator is the identity.  lines = the other lines (n_line_act), then
    // these (n_line_zero); both counts 0 when every line has contrast somewhere.
    DevBuf lines;
    int n_line_act = 0, n_line_zero = 0;
    DevBuf yzflag;           // int32 [nz][ny]: 1 where the line has contrast (with the lists only)
};

// Flags on a stored-block index (block_of_mode) or a mode entry (mode_list): the mode is a
// reflection of the block's own mode, solved as S D_k^{-1} S.  X: x-mode n - kx, S = -1 on the
// x-component rows (block rows [0, m/3)); Y (2-level): y-mode by - ky, S = -1 on the y-component
// rows [m/3, 2m/3); both: the product.
#define VIE_MODE_MIRROR_X (1 << 30)
#define VIE_MODE_MIRROR_Y (1 << 29)
#define VIE_MODE_MIRROR (VIE_MODE_MIRROR_X | VIE_MODE_MIRROR_Y)

struct vie_pc_s {
    vie_op op = nullptr;
    int nboxes = 0, bx = 0, by = 0, bz = 0;
    int levels = 1;          // 1: blocks per x-mode; 2: blocks per (x-mode, y-mode) pair
    int nm = 0;              // modes per box: bx (1-level) or bx*by (2-level, mode ky*bx + kx)
    int m = 0;               // order of the factorised blocks (active rows)
    int m_full = 0;          // 3*by*bz rows of a box cross-section
    // boxes of several shapes / levels / homogenisations: one preconditioner per group, applied
    // in turn (this handle then holds no factors of its own)
    std::vector<vie_pc_s *> children;
    ~vie_pc_s() {
        for (vie_pc_s *c : children) delete c;
    }
    std::vector<int> boxes;  // nboxes*6
    bool covers_all = true;
    int prec = 0;            // factor precision
    int nstored = 0;
    std::vector<int> block_of_mode_host;  // [nboxes*bx]
    DevBuf block_of_mode;    // int32 [nboxes*bx] -> stored block index (| VIE_MODE_MIRROR)
    DevBuf factors;          // [nstored][m][m] column-major LU (complex, factor precision)
    DevBuf perm;             // int32 [nstored][m] row permutation: (P r)[i] = r[perm[i]]
    DevBuf info;             // int32 [nstored] 0 or first zero-pivot column + 1
    // Cross-section rows in solve order: rows[0..m) have M~ != 0 in some box (factorised),
    // rows[m..m_full) are identity rows of every D_k.  Entry = a*by*bz + z*by + y.
    DevBuf rows;             // int32 [m_full]
    std::vector<int> rows_host;
    // every line of the operator without contrast is an identity row of every box: the apply
    // copies its input there (zero in, zero out exactly), so the solver need not project z
    bool zero_lines_kept = false;
    DevBuf chan64, mt64;     // FP64 C^_k table / M~ for the coupling of an FP64 apply
    // 2-level: the identity map of the x-DFT lines of the full cross-section
    DevBuf rows1;
    FftPlan pyb2;            // length by (the y-DFT of the 2-level circulant)
    FftPlan pxb;             // length bx
    // block-solve schedule
    std::vector<int> mode_ptr, mode_list;  // CSR: modes using stored block s (ascending, | VIE_MODE_MIRROR)
    int mirror_rows = 0;                   // block rows per component (m/3): x rows first, then y
    std::vector<int> block_box;            // box of stored block s
    DevBuf modes_dev;                      // int32 mode_ptr [nstored+1] then mode_list
    // refinement of VIE_BF16C solves
    int refine = 0;
    DevBuf chan32;                         // complex float C^_k tables [n][6][2bz-1][2by-1] per box length
                                           // (refinement, and the coupling of an FP32 apply)
    DevBuf mt32;                           // complex float M~ [nboxes][bz][by]
    DevBuf smode_dev;                      // int32 [nstored] mode of each stored block
    WsTable<PcWs> ws;                      // apply scratch per stream
};

// ---------------------------------------------------------------- profiling
// Inside an allocation-free entry point (on this thread): profiling records nothing, since it
// would create events.
struct NoAllocScope {
    NoAllocScope();
    ~NoAllocScope();
};
bool in_noalloc();

// Records a pair of HIP events around a launch on `s` while profiling is on.
struct ProfScope {
    int slot = -1;
    hipStream_t s;
    ProfScope(const char *name, hipStream_t stream);
    ~ProfScope();
};

// ---------------------------------------------------------------- autotuner (tune.cpp)
bool tune_enabled();
bool tune_active();  // candidates are running: profiling records nothing
bool tune_lookup(const std::string &key, std::vector<int> *choice);
void tune_store(const std::string &key, const std::vector<int> &choice, double ms, int candidates);
// one warm-up run, then `reps` runs bracketed by events on `s`; *ms = time per run
// VIE_EARG unless `choice` (from the cache, possibly set by vie_autotune_set) is one of `cands`.
vie_status tune_check_choice(const std::string &key, const std::vector<int> &choice,
                             const std::vector<std::vector<int>> &cands);
vie_status tune_time(hipStream_t s, int reps, const std::function<vie_status()> &run, double *ms);

// ---------------------------------------------------------------- launchers
// generator.hip
vie_status launch_generator(vie_op op, hipStream_t s);
// matvec.hip
vie_status build_kernel_transform(vie_op op, hipStream_t s);
// zero_skipped_in: x is zero on the lines of zero contrast (op->lines) and y is not needed there
// (left as it is); the passes then skip those lines.  Otherwise y = x there, which is exact.
vie_status launch_matvec(vie_op op, const void *x, void *y, int nrhs, int prec, hipStream_t s,
                         bool zero_skipped_in = false);
// api.cpp: the argument checks of vie_matvec and its allocation-free variant (`who` names the call)
vie_status matvec_check_args(const char *who, vie_op op, const void *x, const void *y, int32_t nrhs, int prec);
vie_status launch_rhs(vie_op op, const c128 *e, c128 *b, int nrhs, hipStream_t s);
vie_status launch_contrast(vie_op op, const c128 *chi_dev, hipStream_t s);
vie_status launch_check_chi(const c128 *chi, long long N, int *bad, hipStream_t s);
// flags[yz] = 1 where the contrast of cross-section position yz = z ny + y is nonzero at some x
vie_status launch_line_flags(vie_op op, int *flags, hipStream_t s);
// precond.hip
vie_status pc_build(vie_pc pc, const vie_pc_opts *o, hipStream_t s);
// Drop the per-stream scratch of an operator / a preconditioner (and its box groups) for s.
void op_drop_ws(vie_op op, hipStream_t s);
void pc_drop_ws(vie_pc pc, hipStream_t s);
// api.cpp: device bytes of a request before its operator exists: what a cached operator +
// preconditioner keep (resident), what building them needs on top while it runs (build), and
// what one solve of nrhs right-hand sides adds (run: Krylov workspace, the product's and the
// apply's per-stream scratch, incident fields and right-hand sides)
vie_status request_footprint(const int32_t grid[3], bool c64, const vie_pc_opts *pco, int32_t nrhs,
                             const vie_solve_opts *so, uint64_t *resident, uint64_t *build, uint64_t *run);
// Largest GMRES restart length (the Givens kernel sizes its LDS by it).
#define VIE_MAX_RESTART 200
// Checks of the solver settings shared by vie_solve and the server's submit (`who` names the call).
vie_status solve_opts_check(const char *who, const vie_solve_opts &o);
vie_status pc_apply(vie_pc pc, const void *r, void *z, int nrhs, int prec, hipStream_t s);
// block_solve.hip: the per-mode block solves, in place in the apply work buffer
vie_status launch_block_solve(vie_pc pc, PcWs *w, void *work, int nrhs, hipStream_t s);
// krylov.hip
// complex partial sums per right-hand side kept by the Arnoldi reductions (vector length n)
long long arnoldi_partials(long long n, int restart);
// Called by the batched GMRES before the first step and then after every step at which a
// column ended a restart cycle or a slot is free (columns run their own cycles when a hook is
// given): `ended` lists the columns (slots) whose solve ended since the previous call; their
// stats are final and so is their column of x once the work queued on s is done.  The hook may
// put a new right-hand side into free slots (writing b on s) and returns those slots in
// `refill`: the solver starts them from x = 0 with fresh statistics at the next step.
struct SolveHook {
    virtual ~SolveHook() = default;
    virtual vie_status boundary(const std::vector<int> &ended, const vie_solve_stats *stats, const c128 *x,
                                c128 *b, hipStream_t s, std::vector<int> *refill) = 0;
};
vie_status solve_gmres(vie_op op, vie_pc pc, const c128 *b, c128 *x, int nrhs,
                       const vie_solve_opts *o, vie_solve_stats *stats, hipStream_t s, SolveHook *hook = nullptr);
