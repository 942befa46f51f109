/*
 * vie.h -- C ABI of the MI355X voxel volume-integral-equation solver.
 *
 * Problem (Groth, Polimeridis, Tambova & White, arXiv:1903.07884, Sec. 2,
 * eq. discrete_form): on a uniform grid of nx*ny*nz cubic voxels of edge
 * Delta, solve
 *
 *        (I - M N) w = b,      b = M e_inc  (the factor j w eps0 is dropped),
 *
 * where M = (eps_r - 1)/eps_r is the diagonal contrast (eq. JVIE) and
 * N^{ab}_{ij} = <N p_j^b, p_i^a> is the Galerkin matrix of the operator
 * curl curl int exp(-j k R)/(4 pi R) on the orthonormal piecewise-constant
 * voxel basis (eq. op_N).  Permittivities are relative to a homogeneous
 * background of wavenumber k_background (Sec. 3, Table ref_ind).
 *
 * Vectors.  Every vector is interleaved complex (re, im) with layout
 * [nrhs][3][nz][ny][nx] (component a = x, y, z slowest within one RHS, x
 * fastest), i.e. the unknown ordering w = [w^x; w^y; w^z] of eq. sys_mat.
 * VIE_C128 vectors are complex<double>, VIE_C64 vectors complex<float>.
 * Vector arguments are DEVICE pointers owned by the caller; the library never
 * frees or retains them beyond the call.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = legacy default
 * stream).  vie_matvec, vie_rhs and precond_apply are asynchronous on it;
 * vie_create, precond_setup and vie_solve synchronise it before returning.
 * Handles are read-only once built: calls on different streams (and host
 * threads) may use one operator / preconditioner at the same time.  What a
 * call writes besides its outputs (intermediate spectra, block-solve schedules,
 * tuned launch parameters) lives in scratch owned by the handle per stream:
 * created on the stream's first call, grown as needed, kept until the handle is
 * destroyed.  Calls on one stream from several host threads take turns on that
 * scratch.  A handle must not be destroyed while calls using it are running.
 *
 * Errors.  Every call returns a vie_status.  Negative values are failures;
 * outputs are then unspecified and *out handles are set to NULL.
 * vie_last_error() returns a thread-local message describing the last
 * failure.  Argument errors are detected before any device work.  No C++
 * exception crosses this interface.
 */
#ifndef VIE_H
#define VIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vie_op_s *vie_op; /* owns M, the FP64 generator and the kernel transforms */
typedef struct vie_pc_s *vie_pc; /* owns boxes, homogenised contrasts, block map, LU factors */

typedef enum {
    VIE_C128 = 0, /* complex<double> */
    VIE_C64 = 1,  /* complex<float>  */
    VIE_BF16C = 2 /* preconditioner factors only: complex bfloat16 pairs (4 bytes); the
                     factorisation runs in FP32 and the vectors of such a preconditioner
                     are VIE_C64 */
} vie_prec;

typedef enum {
    VIE_OK = 0,
    VIE_NOT_CONVERGED = 1, /* vie_solve: best iterate returned, stats filled */
    VIE_EARG = -1,         /* invalid argument (checked before device work)  */
    VIE_EOOM = -2,         /* device allocation failed                        */
    VIE_EDEVICE = -3,      /* HIP runtime error                               */
    VIE_ESINGULAR = -4,    /* a preconditioner block has a zero pivot         */
    VIE_ENONFINITE = -5,   /* non-finite input or residual                    */
    VIE_EBUDGET = -6       /* request larger than the server's device-memory budget */
} vie_status;

/* ---- operator ------------------------------------------------------------ */

typedef struct {
    /* Also build the complex64 kernel transform so vie_matvec accepts VIE_C64. */
    int32_t build_c64;
    /* Debug / testing: host array of 12*nx*ny*nz doubles holding the generator
     * K^{ab}(d) (N = I + K) on the octant d >= 0 as [6][nz][ny][nx] interleaved
     * complex, components (xx, yy, zz, xy, xz, yz).  NULL = compute it by
     * quadrature on the device (the normal path). */
    const double *generator;
    /* Testing: 1 = run the product's (y, z) plane pass as three passes through device memory
     * (y-FFT, z coupling, inverse y-FFT) even when the plane fits one workgroup's LDS; the
     * split form is taken anyway for cross-sections too wide for the fused pass. */
    int32_t split_plane;
} vie_create_opts;

/* Build the operator of eq. discrete_form.
 *   grid[3]       = {nx, ny, nz}, each >= 1 (x is the long, Toeplitz-innermost axis)
 *   voxel_size    = Delta in metres (> 0)
 *   k_background  = background wavenumber k_b = 2 pi sqrt(eps_b)/lambda0 in 1/m (>= 0)
 *   chi           = host OR device array of 2*nx*ny*nz doubles, interleaved complex
 *                   relative contrast chi = eps/eps_b - 1 per voxel, [nz][ny][nx];
 *                   every entry finite with 1 + chi != 0 (checked; VIE_EARG otherwise)
 *   opts          = nullable
 * The generator is computed in FP64 (Sec. 2, eq. op_N; six unique blocks, each
 * defined by one octant through its per-axis parity), embedded in a circulant
 * and transformed by FFT.  Synchronises `stream`. */
vie_status vie_create(const int32_t grid[3], double voxel_size, double k_background,
                      const double *chi, const vie_create_opts *opts, void *stream,
                      vie_op *out);
vie_status vie_destroy(vie_op op);

/* Copy the FP64 octant generator (12*nx*ny*nz doubles, layout as in
 * vie_create_opts.generator) to the HOST array `out`.  Synchronous. */
vie_status vie_generator(vie_op op, double *out);

/* b = M e_inc per voxel and component (right-hand side of eq. discrete_form
 * without the factor j w eps0).  e_inc, b: device, c128, nrhs vectors. */
vie_status vie_rhs(vie_op op, const void *e_inc, void *b, int32_t nrhs, void *stream);

/* y = (I - M N) x  (eq. discrete_form) for nrhs vectors.  x, y: device, in
 * precision `prec` (VIE_C64 needs build_c64).  x and y must not overlap.
 * The product with the three-level Toeplitz N uses FFTs of the embedded
 * circulant (Sec. 1: O(n log n) products). */
vie_status vie_matvec(vie_op op, const void *x, void *y, int32_t nrhs, vie_prec prec,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the product of vie_matvec, same
 * arguments, same kernels and the same result, with no allocation of any kind.  Its scratch
 * (the x-spectra of every line, plus the y-spectra of the split plane pass) lives in one
 * fixed device array of VIE_MATVEC_NOALLOC_MAX_BYTES per GPU, which the library holds until
 * the process ends.  A product needing more (about 16*3*ny*nz*Px*nrhs bytes in FP64, half in
 * complex64, Px the x period) returns VIE_EARG before any device work; vie_matvec serves any
 * size.  Every call on one GPU shares that array and leaves its contents behind (nothing in
 * it needs to start at zero): calls that overlap on one GPU (different streams, or host
 * threads without ordering) race and must be serialised by the caller.  Asynchronous on
 * `stream`; argument errors as vie_matvec. */
#define VIE_MATVEC_NOALLOC_MAX_BYTES (64u << 20)
vie_status vie_matvec_noalloc(vie_op op, const void *x, void *y, int32_t nrhs, vie_prec prec,
                              void *stream);

/* ---- preconditioner ------------------------------------------------------ */

typedef enum {
    VIE_HOMOG_NONE = 0,    /* use M itself; it must not vary along x inside a box */
    VIE_HOMOG_MODE = 1,    /* Sec. 5.2, item 1: modal value of M over the box     */
    VIE_HOMOG_MEAN = 2,    /* Sec. 5.2, item 2: mean of M along x                 */
    VIE_HOMOG_REALMEAN = 3 /* Sec. 5.2, item 3: real part of the mean along x     */
} vie_homog;

typedef struct {
    int32_t homog;       /* vie_homog */
    int32_t nboxes;      /* 0 = one box covering the whole grid */
    const int32_t *boxes;/* HOST, nboxes*6: {x0, y0, z0, bx, by, bz} per box; boxes must
                            lie inside the grid and must not overlap; they may differ in
                            shape (boxes of one shape, level and homogenisation share one
                            factor store).  Voxels outside every box are left unchanged
                            (Sec. 5.3: blocked-circulant preconditioner). */
    int32_t reduce;      /* 1 = memory-reduced 1-level preconditioner (Sec. 5.1.1) */
    double reduce_tol;   /* keep mode k iff |v_k|/||v||_inf > reduce_tol (paper: 1e-3) */
    int32_t factor_prec; /* vie_prec of the stored LU factors */
    int32_t proxy;       /* column of the proxy entry of eq. proxy1, whose printed index
                            "ceil(ny/2) ceil(nz/2)" is ambiguous: 0 = the 1-based linear
                            cross-section index ceil(by/2)*ceil(bz/2) (y fastest); 1 = the
                            cross-section centre voxel (ceil(by/2), ceil(bz/2)) */
    int32_t refine_steps;/* VIE_BF16C factors only (else 0): 0 or 1 iterative-refinement
                            steps of every block solve D_k z = r: the residual r - D_k z is
                            formed in FP32 from D_k = I - diag(M~) C^_k itself (not from the
                            rounded factors) and a second solve corrects z */
    int32_t keep_zero_rows; /* 0 (default): cross-section rows (a, y, z) whose homogenised
                            contrast M~(y, z) is zero in every box are identity rows of every
                            D_k (eq. Di with M~ = 0), so only the other rows are factorised and
                            solved; input on the identity rows enters the solve through the
                            exact coupling term M~ C^_k r^ (skipped on the device when that
                            input is zero, as for every Krylov vector of a right-hand side
                            that vanishes where M = 0).  1 = factorise the full cross-section. */
    int32_t levels;         /* 0 or 1: the 1-level circulant (one 3*by*bz block per x-mode);
                            2: the 2-level circulant of Sec. 4 (the Chan approximation applied
                            again along y: one 3*bz block per (x-mode, y-mode) pair), for boxes
                            too wide in y for the 1-level blocks.  Needs a homogenised contrast
                            that does not vary along y (e.g. homog = MODE, the modal average),
                            factor_prec VIE_C128 or VIE_C64, no memory reduction; keep_zero_rows
                            does not apply. */
    const int32_t *box_levels; /* HOST, nboxes entries or NULL: the level of each box, in place
                            of `levels` (Sec. 5.3: e.g. a 1-level box around a bus guide and a
                            2-level box around a disk) */
    const int32_t *box_homog;  /* HOST, nboxes entries or NULL: the vie_homog of each box, in
                            place of `homog` */
    double share_tol;       /* 1-level only; 0 = off.  Stronger compression (a reading of the
                            outlook of Sec. 6): walking the kept modes in ascending order, a mode
                            whose proxy value v_k (eq. proxy1) is within share_tol (relative) of
                            the first mode of the current run uses that mode's block, else it
                            starts a new run (the central mode of the memory reduction always
                            starts one).  Fewer stored blocks, an approximate solve for the
                            shared modes. */
    int32_t no_mirror;      /* 0 (default): the blocks use the reflection symmetry of the
                            operator along x (1-level without sharing, and 2-level): the
                            components xy and xz of the x-level Toeplitz sequences are odd in the
                            x offset and the others even, so T. Chan's circulant has the same
                            parities and D_{n-k} = S D_k S with S = diag(-1 on the x rows, +1 on
                            the y and z rows) (exact up to the rounding of the x-DFT).  Modes
                            k > n/2 are then solved with the factors of mode n - k (about half
                            the stored blocks; a block's factors serve both modes in one read).
                            Under the memory reduction the keep decision of mode k > n/2 is taken
                            at n - k (the proxy is even in x), so kept modes pair.  The 2-level
                            blocks pair along y as well (xy and yz are odd in the y offset): a
                            quarter of the blocks.  1 = factorise every mode. */
} vie_pc_opts;

typedef struct {
    int32_t nboxes, box_nx, block_m;  /* per-box length along x, block size m = 3*by*bz */
    int32_t modes;                    /* nboxes * box_nx Fourier modes */
    int32_t stored_blocks;            /* LU-factored blocks held on the device */
    int64_t factor_bytes;             /* bytes of LU factors (+ pivots) */
    int32_t active_m;                 /* order of the factorised blocks: block_m less the
                                         identity rows (keep_zero_rows = 0) */
    int32_t levels;                   /* 1 or 2; with 2, block_m = 3*bz and modes counts the
                                         (x-mode, y-mode) pairs */
} vie_pc_info;

/* Build the 1-level Chan-Olkin block-circulant preconditioner (Sec. 4): per box,
 * T. Chan's optimal circulant (eq. Chan) of every x-level Toeplitz block of
 * I - M~ N, a DFT along x, and the permuted diagonal blocks D_k (eq. Di), each
 * LU-factorised with partial pivoting.  Synchronises `stream`. */
vie_status precond_setup(vie_op op, const vie_pc_opts *opts, void *stream, vie_pc *out);
vie_status precond_info(vie_pc pc, vie_pc_info *info);
vie_status precond_destroy(vie_pc pc);

/* z = P^{-1} r: per box, DFT along x, block solves with the LU factors of the
 * D_k, inverse DFT (Sec. 4, inverse after eq. Di); identity outside the boxes.
 * r, z: device, precision `prec` (VIE_C64 for VIE_BF16C factors), nrhs vectors; must
 * not overlap.  With VIE_BF16C factors every block is solved on the matrix cores and, with
 * refine_steps = 1, refined once against D_k in FP32. */
vie_status precond_apply(vie_pc pc, const void *r, void *z, int32_t nrhs, vie_prec prec,
                         void *stream);

/* ---- solver ---------------------------------------------------------------- */

typedef enum {
    VIE_MODE_FP64 = 0,      /* GMRES, everything in complex128 */
    VIE_MODE_MIXED = 1,     /* flexible GMRES: complex64 matvec and preconditioner,
                               complex64 basis, FP64 Arnoldi/Givens and FP64 true residual */
    VIE_MODE_MIXED_PC = 2   /* flexible GMRES with only the preconditioner in reduced precision
                               (complex64 or bfloat16 factors, complex64 Z): complex128 operator
                               product and basis, FP64 Arnoldi/Givens.  The inner products then
                               carry no complex64 operator error, which bounds what one restart
                               cycle of VIE_MODE_MIXED can gain on ill-conditioned problems. */
} vie_mode;

typedef struct {
    double tol;        /* relative residual ||b - A x|| / ||b|| (default 1e-6) */
    int32_t restart;   /* Krylov dimension per cycle (default 50, max 200) */
    int32_t maxit;     /* total Arnoldi steps per right-hand side (default 5000) */
    int32_t mode;      /* vie_mode */
    int32_t x0_given;  /* 1 = x holds the initial guess, 0 = start from zero */
} vie_solve_opts;

typedef struct {
    int32_t iters;     /* Arnoldi steps summed over cycles */
    int32_t restarts;  /* completed cycles */
    double relres;     /* true relative residual of the returned x (FP64) */
    int32_t status;    /* VIE_OK or VIE_NOT_CONVERGED */
} vie_solve_stats;

/* Right-preconditioned restarted GMRES for (I - M N) x = b (Sec. 1; restart,
 * side and tolerance are this library's choices, the paper reports 1e-4).
 * b, x: device c128, nrhs vectors.  pc = NULL solves unpreconditioned.
 * stats: HOST array of nrhs entries.  Synchronises `stream`. */
vie_status vie_solve(vie_op op, vie_pc pc, const void *b, void *x, int32_t nrhs,
                     const vie_solve_opts *opts, vie_solve_stats *stats, void *stream);

/* ---- serving ------------------------------------------------------------------
 * A request scheduler for many solves of different devices on one GPU (the solver of
 * Sec. 1 applied to a stream of devices; the scheduling is this library's).  Requests are
 * queued on submit and admitted while their device-memory footprint fits the budget;
 * operators and preconditioners stay resident in a cache keyed by the device (grid, voxel
 * size, wavenumber, a hash of the contrast) and the preconditioner options, evicted least
 * recently used when memory is needed; each worker thread owns a HIP stream, so admitted
 * solves run side by side on the device; requests waiting for the same device, options and
 * solver settings are merged into one multi-RHS solve.  The right-hand sides of a running
 * solve are slots (continuous batching): at every GMRES restart boundary a request whose
 * columns have all ended completes (its waiter returns while the others go on) and a queued
 * request of the same device and settings that fits the freed slots joins the solve.  A
 * result does not depend on what it was solved beside: columns of a merged solve equal the
 * single solves (the batched GMRES runs every right-hand side on its own, with reductions
 * whose order does not depend on the batch).  Thread-safe: any thread may submit and wait. */
typedef struct vie_server_s *vie_server;

typedef struct {
    int32_t workers;        /* concurrent solves, one HIP stream each (0: 4; at most 16) */
    int32_t max_batch_rhs;  /* merge queued requests of one device up to this many right-hand
                               sides per solve (0: 64; 1: no merging) */
    uint64_t hbm_budget;    /* device bytes the server may commit (0: 90% of the free memory at
                               vie_server_create); admission uses the vie_footprint bounds */
} vie_server_opts;

typedef struct {
    int32_t grid[3];
    double voxel_size;
    double k_background;
    const double *chi;      /* HOST, 2*N doubles as in vie_create; copied by vie_server_submit */
    const double *e_inc;    /* HOST, nrhs*6*N doubles: incident fields [nrhs][3][nz][ny][nx]
                               interleaved complex (b = M e_inc is formed on the device); copied */
    int32_t nrhs;
    int32_t precond;        /* 0: unpreconditioned; 1: preconditioner built with `pc` */
    vie_pc_opts pc;         /* boxes (if any) copied */
    vie_solve_opts solve;   /* x0_given must be 0 */
} vie_request;

typedef struct {
    double queue_ms;        /* submit -> start of its solve */
    double run_ms;          /* start -> result on the host (build or cache lookup, solve, copy) */
    double total_ms;        /* submit -> result */
    int32_t cache_hit;      /* operator and preconditioner came from the resident cache */
    int32_t merged;         /* requests that took part in the same multi-RHS solve up to this
                               one's completion, itself included */
    int32_t joined;         /* 1: joined a running solve at a restart boundary (continuous
                               batching), 0: admitted with the solve */
} vie_request_times;

typedef struct {
    int64_t submitted, completed, solves, cache_hits, evictions;
    int32_t cached_entries, queued, running;
    uint64_t committed_bytes, peak_committed_bytes, budget_bytes;
    int64_t shared_runs;    /* solves admitted onto an entry another solve was running on */
    int64_t cache_trims;    /* admissions that returned the released blocks cached for reuse to the
                               driver (committed + request + cached blocks above the budget) */
} vie_server_info;

vie_status vie_server_create(const vie_server_opts *opts, vie_server *out);
/* Queue a request; returns at once with its id.  x_out (HOST, nrhs*6*N doubles) and stats_out
 * (HOST, nrhs entries) are written when it completes and must stay valid until
 * vie_server_wait returns for it.  VIE_EARG for invalid arguments, VIE_EBUDGET when the
 * request alone exceeds the budget. */
vie_status vie_server_submit(vie_server srv, const vie_request *req, double *x_out,
                             vie_solve_stats *stats_out, int64_t *id);
/* Block until request `id` completes; returns its status (VIE_OK, VIE_NOT_CONVERGED or the
 * error of its build or solve) and, if times != NULL, its timings.  Each id is waited once. */
vie_status vie_server_wait(vie_server srv, int64_t id, vie_request_times *times);
vie_status vie_server_query(vie_server srv, int64_t id, int32_t *done);
vie_status vie_server_info_get(vie_server srv, vie_server_info *info);
/* Finish queued and running requests, free the cache and the server. */
vie_status vie_server_destroy(vie_server srv);

/* ---- diagnostics ----------------------------------------------------------- */

/* Kernel timing with HIP events recorded on the stream each kernel is launched
 * on.  vie_profile_begin() clears the record and starts recording;
 * vie_profile_kernel() synchronises the recorded events and returns, for one
 * kernel name, the summed duration in milliseconds and the number of
 * launches; vie_profile_end() stops recording.  Names: "generator",
 * "matvec_xfwd", "matvec_plane", "matvec_xinv", "precond_xfft", "block_solve" (all block
 * solves of an apply), "refine_residual" (the refinement residual and correcting solve),
 * "precond_ixfft", "precond_identity_rows" (copy of the identity rows and, when they hold
 * input, its coupling into the solved rows), "lu_panel", "lu_swap_trsm", "lu_update", "lu_invert_diag",
 * "arnoldi_dots", "arnoldi_update".  Recording adds two event records per launch. */
vie_status vie_profile_begin(void);
vie_status vie_profile_kernel(const char *name, double *total_ms, int64_t *launches);
vie_status vie_profile_end(void);

/* ---- footprint ------------------------------------------------------------------
 * Upper bound, in bytes, of the device memory held by `op` (with the transient of its
 * creation) plus, when `pc` is not NULL, a
 * preconditioner built from those options (every mode stored, i.e. no memory reduction
 * credited, factorisation temporaries and LU workspace included) plus, when `so` is not
 * NULL, one vie_solve of `nrhs` right-hand sides with those options (Krylov basis, flexible
 * basis, residual and reduction workspace, and the per-call matvec / apply scratch the solve
 * grows), with autotuning off.  An admission controller compares it with the free HBM
 * before it creates the preconditioner or starts the solve.  Argument errors as for
 * precond_setup / vie_solve. */
vie_status vie_footprint(vie_op op, const vie_pc_opts *pc, int32_t nrhs, const vie_solve_opts *so,
                         uint64_t *bytes);

/* Device bytes currently held by all handles and calls of this library (process-wide) and
 * the high-water mark since the last reset (reset_peak != 0 first sets it to the current
 * value).  Either output may be NULL. */
vie_status vie_device_bytes(uint64_t *current, uint64_t *peak, int32_t reset_peak);

/* Device memory released by handles and calls is kept by the library for reuse (freeing and
 * re-allocating tens of GB costs the driver up to seconds); vie_trim returns that cache to
 * the driver.  The cache is also returned, and the allocation retried, whenever the device
 * runs out of memory.  vie_device_bytes counts only memory held by handles and calls. */
vie_status vie_trim(void);

/* ---- autotuning ----------------------------------------------------------------
 * With autotuning on, the first precond_apply (and vie_solve) for a new problem shape and
 * right-hand-side count times every candidate launch configuration of the block solves
 * (column-group width and workgroup height of the matrix-core solve, right-hand sides per
 * workgroup of the per-mode solve, and the right-hand-side count from which blocks use the
 * matrix-core solve) on a copy of the data; the first vie_matvec for a new shape and
 * right-hand-side count times the right-hand sides per workgroup of the register plane pass
 * (or the threads of the LDS plane pass) and the threads of the LDS x-line passes; and
 * precond_setup times the sub-panels per macro panel (1, 2, 4, 8) and the sub-panel width
 * (32, 16 columns) of the batched LU on a copy of the first min(blocks, 256) blocks.  The fastest is kept for the rest of the
 * process, keyed by the shape.  Results never depend on the choice beyond rounding order.
 * vie_autotune_report writes the cache as text ("key -> choice (ms, candidates)" lines)
 * into buf (truncated to size - 1 characters, NUL-terminated); *needed receives the full
 * length + 1.  vie_autotune_set stores the n values `choice` under `key` (a key as the
 * report prints it; n = 0 removes the entry), so that tuned parameters can be restored in
 * a later process or a candidate forced: with autotuning on, a call whose shape has that
 * key uses the stored values without timing, and fails with VIE_EARG (nothing launched) if
 * they are not one of that shape's candidates.  VIE_EARG for a null key, n outside 0..16 or
 * a null choice with n > 0.  All three calls are process-wide and thread-safe. */
vie_status vie_autotune(int32_t enable);
vie_status vie_autotune_report(char *buf, int64_t size, int64_t *needed);
vie_status vie_autotune_set(const char *key, const int32_t *choice, int32_t n);

/* Thread-local description of the last failure ("" if none). */
const char *vie_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VIE_H */
