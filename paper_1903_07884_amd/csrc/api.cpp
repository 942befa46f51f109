// C ABI entry points: argument validation, handle ownership, orchestration.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>

#include "fft_device.h"

static thread_local std::string g_err;
void vie_set_error(const std::string &msg) { g_err = msg; }
extern "C" const char *vie_last_error(void) { return g_err.c_str(); }

static vie_status arg_error(const std::string &msg) {
    g_err = msg;
    return VIE_EARG;
}

size_t max_lds() {
    static size_t v = 0;
    if (!v) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            v = p.sharedMemPerBlock;
        else
            v = 65536;
    }
    return v;
}

extern "C" vie_status vie_create(const int32_t grid[3], double voxel_size, double k_background, const double *chi,
                                 const vie_create_opts *opts, void *stream, vie_op *out) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    if (!out) return arg_error("vie_create: out is NULL");
    *out = nullptr;
    if (!grid) return arg_error("vie_create: grid is NULL");
    if (!chi) return arg_error("vie_create: chi is NULL");
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1) return arg_error("vie_create: every grid dimension must be >= 1");
    if (!(voxel_size > 0) || !std::isfinite(voxel_size)) return arg_error("vie_create: voxel_size must be > 0");
    if (!(k_background >= 0) || !std::isfinite(k_background))
        return arg_error("vie_create: k_background must be finite and >= 0");
    long long N = (long long)grid[0] * grid[1] * grid[2];
    if (N > (1LL << 31)) return arg_error("vie_create: grid too large");
    bool chi_on_device = false;
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, chi) == hipSuccess && attr.type == hipMemoryTypeDevice)
            chi_on_device = true;
        (void)hipGetLastError();
    }
    if (!chi_on_device)
        for (long long i = 0; i < N; ++i) {
            double re = chi[2 * i], im = chi[2 * i + 1];
            if (!std::isfinite(re) || !std::isfinite(im)) return arg_error("vie_create: non-finite contrast");
            if (re == -1.0 && im == 0.0) return arg_error("vie_create: 1 + chi must be non-zero");
        }
    vie_create_opts o{};
    if (opts) o = *opts;
    vie_op op = new (std::nothrow) vie_op_s();
    if (!op) return VIE_EOOM;
    hipStream_t s = (hipStream_t)stream;
    op->nx = grid[0];
    op->ny = grid[1];
    op->nz = grid[2];
    op->N = N;
    op->delta = voxel_size;
    op->kb = k_background;
    op->kappa = k_background * voxel_size;
    op->Px = fft_good_length(2 * op->nx - 1);
    op->Py = fft_good_length(2 * op->ny - 1);
    op->Pz = fft_good_length(2 * op->nz - 1);
    op->Hx = op->Px / 2 + 1;
    op->Hy = op->Py / 2 + 1;
    op->Hz = op->Pz / 2 + 1;
    op->has_c64 = o.build_c64 != 0;
    // few z layers: keep the z coupling as a direct Toeplitz sum (no z transform); the
    // (y, z) plane working set must fit the LDS either way
    op->direct_z = op->nz <= 16;
    const bool fused_plane = 3LL * op->nz * op->Py <= 2LL * FFT_BPT * 1024 &&
                             sizeof(c128) * ((size_t)6 * op->nz * op->Py + (size_t)6 * op->Hy * op->nz) <= max_lds();
    op->split_plane = op->direct_z && (!fused_plane || o.split_plane);
    auto fail = [&](vie_status st) {
        delete op;
        return st;
    };
    if (op->split_plane && 2 * sizeof(c128) * op->Py > max_lds())
        return fail(arg_error("vie_create: y extent too long for the LDS line transform"));
    if (!op->direct_z && 6 * sizeof(c128) * op->Py * op->Pz > max_lds())
        return fail(arg_error("vie_create: cross-section too large for the LDS plane transform"));
    vie_status st;
    if ((st = op->fft.get(op->Px, &op->px)) < 0) return fail(st);
    if ((st = op->fft.get(op->Py, &op->py)) < 0) return fail(st);
    if ((st = op->fft.get(op->Pz, &op->pz)) < 0) return fail(st);
    {
        int thr, bpt;
        size_t lds;
        fft_line_shape(op->px, sizeof(c128), &thr, &lds, &bpt);
        if (lds > max_lds()) {
            // four-step: Px = L1 L2 with L2 the largest divisor <= sqrt(Px) that leaves L1 a
            // multiple of the column tile (16) and both factors within one workgroup's LDS
            int L2 = 0;
            for (int d = 1; (long long)d * d <= op->Px; ++d)
                if (op->Px % d == 0 && (op->Px / d) % 16 == 0) L2 = d;
            if (L2 < 2 || L2 > 512 || sizeof(c128) * (size_t)L2 * 16 > max_lds())
                return fail(arg_error("vie_create: no four-step split of the x period " + std::to_string(op->Px)));
            op->xsplit = L2;
            if ((st = op->fft.get(op->Px / L2, &op->px1)) < 0) return fail(st);
            if ((st = op->fft.get(L2, &op->px2)) < 0) return fail(st);
            fft_line_shape(op->px1, sizeof(c128), &thr, &lds, &bpt);
            if (lds > max_lds())
                return fail(arg_error("vie_create: x period " + std::to_string(op->Px) + " too long"));
        }
    }
    if ((st = op->M64.ensure(sizeof(c128) * N)) < 0) return fail(st);
    if ((st = op->M32.ensure(sizeof(c64) * N)) < 0) return fail(st);
    if ((st = op->gen.ensure(sizeof(c128) * 6 * N)) < 0) return fail(st);
    {
        DevBuf chid;
        if ((st = chid.ensure(sizeof(c128) * N)) < 0) return fail(st);
        if (hipMemcpyAsync(chid.p, chi, sizeof(c128) * N,
                           chi_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(VIE_EDEVICE);
        if (chi_on_device) {
            DevBuf bad;
            int hbad = 0;
            if ((st = bad.ensure(sizeof(int))) < 0) return fail(st);
            if (hipMemsetAsync(bad.p, 0, sizeof(int), s) != hipSuccess) return fail(VIE_EDEVICE);
            if ((st = launch_check_chi(chid.as<c128>(), N, bad.as<int>(), s)) < 0) return fail(st);
            if (hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(VIE_EDEVICE);
            if (hbad) return fail(arg_error("vie_create: non-finite contrast or 1 + chi == 0"));
        }
        if ((st = launch_contrast(op, chid.as<c128>(), s)) < 0) return fail(st);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(VIE_EDEVICE);
    }
    {
        // lines of the vectors with contrast somewhere along x, then the others (identity rows of
        // the operator); the solver restricts its basis passes to the former
        const int nyz = op->ny * op->nz;
        DevBuf &fl = op->yzflag;
        if ((st = fl.ensure(sizeof(int) * nyz)) < 0) return fail(st);
        if ((st = launch_line_flags(op, fl.as<int>(), s)) < 0) return fail(st);
        std::vector<int> hf(nyz);
        if (hipMemcpyAsync(hf.data(), fl.p, sizeof(int) * nyz, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(VIE_EDEVICE);
        std::vector<int> act, zero;
        for (int c = 0; c < 3; ++c)
            for (int yz = 0; yz < nyz; ++yz) (hf[yz] ? act : zero).push_back(c * nyz + yz);
        if (!zero.empty()) {
            act.insert(act.end(), zero.begin(), zero.end());
            if ((st = op->lines.ensure(sizeof(int) * act.size())) < 0) return fail(st);
            if (hipMemcpyAsync(op->lines.p, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(VIE_EDEVICE);
            op->n_line_zero = (int)zero.size();
            op->n_line_act = (int)act.size() - op->n_line_zero;
        } else {
            fl.release();
        }
    }
    if (o.generator) {
        if (hipMemcpyAsync(op->gen.p, o.generator, sizeof(c128) * 6 * N, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(VIE_EDEVICE);
    } else if ((st = launch_generator(op, s)) < 0)
        return fail(st);
    // twiddles of the x-length (the default preconditioner box) computed on the host while the
    // generator runs, instead of with the device idle at the preconditioner setup
    if (fft_supported_length(op->nx)) {
        FftPlan px_box;
        if ((st = op->fft.get(op->nx, &px_box)) < 0) return fail(st);
    }
    if ((st = build_kernel_transform(op, s)) < 0) return fail(st);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        g_err = std::string("vie_create: ") + hipGetErrorString(e);
        return fail(VIE_EDEVICE);
    }
    *out = op;
    return VIE_OK;
}

extern "C" vie_status vie_destroy(vie_op op) {
    if (!op) return VIE_OK;
    delete op;
    return VIE_OK;
}

extern "C" vie_status vie_generator(vie_op op, double *out) {
    if (!op || !out) return arg_error("vie_generator: NULL argument");
    VIE_HIP(hipDeviceSynchronize());
    VIE_HIP(hipMemcpy(out, op->gen.p, sizeof(c128) * 6 * op->N, hipMemcpyDeviceToHost));
    return VIE_OK;
}

extern "C" vie_status vie_rhs(vie_op op, const void *e_inc, void *b, int32_t nrhs, void *stream) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    if (!op || !e_inc || !b) return arg_error("vie_rhs: NULL argument");
    if (nrhs < 1) return arg_error("vie_rhs: nrhs must be >= 1");
    return launch_rhs(op, (const c128 *)e_inc, (c128 *)b, nrhs, (hipStream_t)stream);
}

void op_drop_ws(vie_op op, hipStream_t s) {
    if (op) op->ws.drop(s);
}

void pc_drop_ws(vie_pc pc, hipStream_t s) {
    if (!pc) return;
    for (vie_pc c : pc->children) pc_drop_ws(c, s);
    pc->ws.drop(s);
}

vie_status matvec_check_args(const char *who, vie_op op, const void *x, const void *y, int32_t nrhs, int prec) {
    const std::string w(who);
    if (!op || !x || !y) return arg_error(w + ": NULL argument");
    if (nrhs < 1) return arg_error(w + ": nrhs must be >= 1");
    if (prec != VIE_C128 && prec != VIE_C64) return arg_error(w + ": unknown precision");
    if (prec == VIE_C64 && !op->has_c64) return arg_error(w + ": operator built without complex64 transform");
    if (x == y) return arg_error(w + ": x and y must not overlap");
    return VIE_OK;
}

extern "C" vie_status vie_matvec(vie_op op, const void *x, void *y, int32_t nrhs, vie_prec prec, void *stream) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    VIE_CHECK(matvec_check_args("vie_matvec", op, x, y, nrhs, prec));
    return launch_matvec(op, x, y, nrhs, prec, (hipStream_t)stream);
}

// One preconditioner over boxes that share shape, level and homogenisation (the boxes were
// validated by the caller).  covers_all: the boxes cover the grid (else the apply copies r to z
// first); a group inside a composite is built with covers_all = true, the composite copies.
static vie_status build_group(vie_op op, const vie_pc_opts &o, const std::vector<int> &boxes, int levels,
                              bool covers_all, hipStream_t s, vie_pc *out) {
    const int nb = (int)boxes.size() / 6;
    const int bx = boxes[3], by = boxes[4], bz = boxes[5];
    int m = 3 * by * bz;
    if (!fft_supported_length(bx))
        return arg_error("precond_setup: box length " + std::to_string(bx) + " has a prime factor above " +
                         std::to_string(VIE_FFT_MAX_PRIME));
    {
        FftPlan tmp;
        if (op->fft.get(bx, &tmp) < 0) return VIE_EARG;
        int thr, bpt;
        size_t lds;
        fft_line_shape(tmp, sizeof(c128), &thr, &lds, &bpt);
        if (lds > max_lds()) return arg_error("precond_setup: box too long for the LDS transform");
    }
    if (levels == 2) {
        if (o.reduce || o.factor_prec == VIE_BF16C || o.share_tol > 0)
            return arg_error("precond_setup: the 2-level circulant takes VIE_C128 or VIE_C64 factors and no memory reduction");
        if (!fft_supported_length(by))
            return arg_error("precond_setup: box width " + std::to_string(by) + " has a prime factor above " +
                             std::to_string(VIE_FFT_MAX_PRIME));
        FftPlan tmp;
        if (op->fft.get(by, &tmp) < 0) return VIE_EARG;
        m = 3 * bz;
    }
    if (m > 1280) return arg_error("precond_setup: cross-section block (3*by*bz) above 1280 is not supported");
    vie_pc pc = new (std::nothrow) vie_pc_s();
    if (!pc) return VIE_EOOM;
    pc->op = op;
    pc->nboxes = nb;
    pc->bx = bx;
    pc->by = by;
    pc->bz = bz;
    pc->levels = levels;
    pc->nm = levels == 2 ? bx * by : bx;
    pc->m = m;
    pc->m_full = m;
    pc->boxes = boxes;
    pc->covers_all = covers_all;
    pc->prec = o.factor_prec;
    pc->refine = o.refine_steps;
    vie_status st = pc_build(pc, &o, s);
    if (st < 0) {
        delete pc;
        return st;
    }
    *out = pc;
    return VIE_OK;
}

extern "C" vie_status precond_setup(vie_op op, const vie_pc_opts *opts, void *stream, vie_pc *out) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    if (!out) return arg_error("precond_setup: out is NULL");
    *out = nullptr;
    if (!op || !opts) return arg_error("precond_setup: NULL argument");
    const vie_pc_opts &o = *opts;
    if (o.homog < VIE_HOMOG_NONE || o.homog > VIE_HOMOG_REALMEAN) return arg_error("precond_setup: unknown homog");
    if (o.factor_prec != VIE_C128 && o.factor_prec != VIE_C64 && o.factor_prec != VIE_BF16C)
        return arg_error("precond_setup: unknown factor precision");
    if (o.refine_steps < 0 || o.refine_steps > 1) return arg_error("precond_setup: refine_steps must be 0 or 1");
    if (o.refine_steps && o.factor_prec != VIE_BF16C)
        return arg_error("precond_setup: refine_steps needs VIE_BF16C factors");
    if (o.keep_zero_rows != 0 && o.keep_zero_rows != 1)
        return arg_error("precond_setup: keep_zero_rows must be 0 or 1");
    if (o.levels < 0 || o.levels > 2) return arg_error("precond_setup: levels must be 0, 1 or 2");
    if (o.factor_prec == VIE_BF16C && !op->has_c64)
        return arg_error("precond_setup: VIE_BF16C factors need an operator built with build_c64");
    if (o.proxy != 0 && o.proxy != 1) return arg_error("precond_setup: proxy must be 0 or 1");
    if (o.reduce && (!(o.reduce_tol >= 0) || !std::isfinite(o.reduce_tol)))
        return arg_error("precond_setup: reduce_tol must be finite and >= 0");
    if (!(o.share_tol >= 0) || !std::isfinite(o.share_tol))
        return arg_error("precond_setup: share_tol must be finite and >= 0");
    std::vector<int> boxes;
    if (o.nboxes < 0) return arg_error("precond_setup: nboxes < 0");
    if (o.nboxes == 0) {
        boxes = {0, 0, 0, op->nx, op->ny, op->nz};
    } else {
        if (!o.boxes) return arg_error("precond_setup: boxes is NULL");
        boxes.assign(o.boxes, o.boxes + 6 * o.nboxes);
    }
    int nb = (int)boxes.size() / 6;
    const int dims[3] = {op->nx, op->ny, op->nz};
    long long vol = 0;
    std::vector<int> lev(nb), hom(nb);
    for (int b = 0; b < nb; ++b) {
        const int *B = &boxes[6 * b];
        for (int a = 0; a < 3; ++a)
            if (B[a] < 0 || B[3 + a] < 1 || B[a] + B[3 + a] > dims[a])
                return arg_error("precond_setup: box " + std::to_string(b) + " outside the grid");
        for (int c = 0; c < b; ++c) {
            const int *C = &boxes[6 * c];
            bool ov = true;
            for (int a = 0; a < 3; ++a)
                if (B[a] + B[3 + a] <= C[a] || C[a] + C[3 + a] <= B[a]) ov = false;
            if (ov) return arg_error("precond_setup: boxes overlap");
        }
        vol += (long long)B[3] * B[4] * B[5];
        const int lv = o.nboxes > 0 && o.box_levels ? o.box_levels[b] : o.levels;
        const int hm = o.nboxes > 0 && o.box_homog ? o.box_homog[b] : o.homog;
        if (lv < 0 || lv > 2) return arg_error("precond_setup: box_levels entries must be 0, 1 or 2");
        if (hm < VIE_HOMOG_NONE || hm > VIE_HOMOG_REALMEAN) return arg_error("precond_setup: unknown box_homog entry");
        lev[b] = lv == 2 ? 2 : 1;
        hom[b] = hm;
    }
    // group the boxes by (shape, level, homogenisation): one factor store per group
    std::vector<std::vector<int>> groups;  // box indices
    for (int b = 0; b < nb; ++b) {
        bool placed = false;
        for (auto &g : groups) {
            const int f = g[0];
            bool same = lev[f] == lev[b] && hom[f] == hom[b];
            for (int a = 3; a < 6; ++a) same = same && boxes[6 * f + a] == boxes[6 * b + a];
            if (same) {
                g.push_back(b);
                placed = true;
                break;
            }
        }
        if (!placed) groups.push_back({b});
    }
    const bool covers_all = vol == op->N;
    hipStream_t s = (hipStream_t)stream;
    auto group_boxes = [&](const std::vector<int> &g) {
        std::vector<int> gb;
        for (int b : g) gb.insert(gb.end(), boxes.begin() + 6 * b, boxes.begin() + 6 * b + 6);
        return gb;
    };
    if (groups.size() == 1) {
        vie_pc_opts go = o;
        go.homog = hom[0];
        return build_group(op, go, group_boxes(groups[0]), lev[0], covers_all, s, out);
    }
    vie_pc parent = new (std::nothrow) vie_pc_s();
    if (!parent) return VIE_EOOM;
    parent->op = op;
    parent->nboxes = nb;
    parent->boxes = boxes;
    parent->covers_all = covers_all;
    parent->prec = o.factor_prec;
    parent->refine = o.refine_steps;
    for (auto &g : groups) {
        vie_pc_opts go = o;
        go.homog = hom[g[0]];
        vie_pc child = nullptr;
        const vie_status st = build_group(op, go, group_boxes(g), lev[g[0]], true, s, &child);
        if (st < 0) {
            delete parent;
            return st;
        }
        parent->children.push_back(child);
        parent->nstored += child->nstored;
        parent->levels = std::max(parent->levels, child->levels);
        parent->m = std::max(parent->m, child->m);
        parent->m_full = std::max(parent->m_full, child->m_full);
    }
    *out = parent;
    return VIE_OK;
}

// Device bytes an operator of this grid holds (contrast, generator, kernel transforms) and the
// transient of its creation (the transformed circulant embedding and the contrast upload),
// computed from the grid alone (the sizes vie_create allocates).
static void op_bytes_estimate(int nx, int ny, int nz, bool c64, uint64_t *held, uint64_t *transient, int *Px_out) {
    const uint64_t N = (uint64_t)nx * ny * nz;
    const int Px = fft_good_length(2 * nx - 1), Py = fft_good_length(2 * ny - 1), Pz = fft_good_length(2 * nz - 1);
    const uint64_t Hx = Px / 2 + 1, Hy = Py / 2 + 1, Hz = Pz / 2 + 1;
    // (x, y) transform with z offsets, or the full octant: the larger of the two
    const uint64_t kh = Hx * Hy * std::max<uint64_t>((uint64_t)nz, Hz) * 6;
    *held = 16 * N + 8 * N + 16 * 6 * N + kh * 16 + (c64 ? kh * 8 : 0);
    *transient = 6ULL * 16 * Px * Py * Pz + 16 * N;
    *Px_out = Px;
}

// Footprint of the preconditioner (held, with its setup temporaries), its apply scratch, the
// matvec scratch and the solve workspace for nrhs right-hand sides.
static vie_status footprint_parts(int nx, int ny, int nz, int Px, int Py, bool split, const vie_pc_opts *pco,
                                  int32_t nrhs, const vie_solve_opts *so, uint64_t *mv_scratch, uint64_t *pc_held,
                                  uint64_t *apply_scratch, uint64_t *solve_bytes) {
    const uint64_t N = (uint64_t)nx * ny * nz, R = (uint64_t)nrhs, n3 = 3 * N;
    const uint64_t lines = 3ULL * ny * nz * R;
    *mv_scratch = sizeof(c128) * lines * (uint64_t)Px;
    if (split) *mv_scratch += 2 * sizeof(c128) * R * (uint64_t)Px * 3 * nz * (uint64_t)Py;  // split plane pass
    *pc_held = *apply_scratch = *solve_bytes = 0;
    if (pco) {
        const vie_pc_opts &o = *pco;
        if (o.factor_prec != VIE_C128 && o.factor_prec != VIE_C64 && o.factor_prec != VIE_BF16C)
            return arg_error("vie_footprint: unknown factor precision");
        if (o.nboxes < 0 || (o.nboxes > 0 && !o.boxes)) return arg_error("vie_footprint: bad boxes");
        const int nbox = o.nboxes ? o.nboxes : 1;
        // group the boxes by shape and level (one factor store each) and sum the groups
        std::vector<std::array<int, 5>> groups;  // bx, by, bz, level, count
        for (int b = 0; b < nbox; ++b) {
            const int *B = o.nboxes ? o.boxes + 6 * b : nullptr;
            const int gbx = B ? B[3] : nx, gby = B ? B[4] : ny, gbz = B ? B[5] : nz;
            if (gbx < 1 || gby < 1 || gbz < 1) return arg_error("vie_footprint: bad box shape");
            const int lv = (o.nboxes && o.box_levels ? o.box_levels[b] : o.levels) == 2 ? 2 : 1;
            bool found = false;
            for (auto &g : groups)
                if (g[0] == gbx && g[1] == gby && g[2] == gbz && g[3] == lv) {
                    g[4]++;
                    found = true;
                }
            if (!found) groups.push_back({gbx, gby, gbz, lv, 1});
        }
        const uint64_t fesz = o.factor_prec == VIE_C128 ? 16 : o.factor_prec == VIE_BF16C ? 4 : 8;
        const uint64_t vesz = o.factor_prec == VIE_C128 ? 16 : 8;  // vector / factorisation precision
        for (const auto &g : groups) {
            const uint64_t bx = g[0], by = g[1], bz = g[2], nb = g[4];
            const bool two = g[3] == 2;
            const uint64_t m = two ? 3 * bz : 3 * by * bz, modes = two ? nb * bx * by : nb * bx;
            const uint64_t table = bx * 6 * (2 * by - 1) * (2 * bz - 1) + (two ? bx * by * 6 * (2 * bz - 1) : 0);
            // stored blocks: every mode, or with the reflection pairing the x-modes 0..bx/2
            // (2-level: times the y-modes 0..by/2)
            const bool mirror = !o.no_mirror && (two || (!o.reduce && !(o.share_tol > 0)));
            const uint64_t stored = mirror ? nb * (bx / 2 + 1) * (two ? by / 2 + 1 : 1) : modes;
            uint64_t pcb = stored * m * m * fesz + stored * m * 8 + modes * 16;  // factors, pivots, maps
            if (o.factor_prec == VIE_BF16C) pcb += stored * m * m * 8;         // complex-float factorisation copy
            pcb += table * 16 + stored * m * 4 + stored * 64 * 64 * vesz;       // Chan table, LU workspace
            if (o.refine_steps || !o.keep_zero_rows) pcb += table * 8 + nb * by * bz * 8;
            if (!o.keep_zero_rows && o.factor_prec == VIE_C128) pcb += table * 16 + nb * by * bz * 16;
            pcb += 3 * by * bz * 4 + 64;  // row orders, coupling flag
            *pc_held += pcb;
            // apply: x-DFT lines plus the matrix-core solve scratch (once more for the bfloat16
            // hi + lo copy of the solved rows, which a refined apply's two solves share)
            const uint64_t cols = modes * R;
            const uint64_t wide = (cols + 64 * modes) * m * vesz;
            *apply_scratch += R * nb * m * (modes / nb) * vesz + wide * (o.factor_prec == VIE_BF16C ? 2 : 1);
            if (two) *apply_scratch += R * nb * 3 * by * bz * bx * vesz;  // x-stage lines
        }
    }
    if (so) {
        if (so->restart < 1 || so->restart > VIE_MAX_RESTART)
            return arg_error("vie_footprint: restart must be in [1, " + std::to_string(VIE_MAX_RESTART) + "]");
        const uint64_t rs = (uint64_t)so->restart;
        const bool mixed = so->mode == VIE_MODE_MIXED, mixed_pc = so->mode == VIE_MODE_MIXED_PC;
        const uint64_t vb = mixed ? 8 : 16;              // basis precision
        const uint64_t zb = mixed || mixed_pc ? 8 : 16;  // preconditioned vectors
        // complex64 product output (mixed, which has no complex128 one); complex64 copy of v_j +
        // widened z_j (mixed_pc)
        const uint64_t extra = mixed ? 8 : mixed_pc ? 8 + 16 : 0;
        *solve_bytes = vb * R * n3 * (rs + 1) + zb * R * n3 * rs + (mixed ? 1 : 2) * 16 * R * n3 +
                       16 * R * (uint64_t)arnoldi_partials((long long)n3, (int)rs) + extra * R * n3 +
                       2 * 16 * R * (rs + 2) * (rs + 4);
    }
    return VIE_OK;
}

extern "C" vie_status vie_footprint(vie_op op, const vie_pc_opts *pco, int32_t nrhs, const vie_solve_opts *so,
                                   uint64_t *bytes) {
    if (!op || !bytes) return arg_error("vie_footprint: NULL argument");
    if (nrhs < 1) return arg_error("vie_footprint: nrhs must be >= 1");
    // operator: contrast, generator, kernel transforms (held) and the matvec scratch
    uint64_t b = op->M64.bytes + op->M32.bytes + op->gen.bytes + op->khat64.bytes + op->khat32.bytes;
    b += 6ULL * 16 * op->Px * op->Py * op->Pz;  // the circulant embedding transformed during vie_create
    uint64_t mv, pcb, ap, sb;
    VIE_CHECK(footprint_parts(op->nx, op->ny, op->nz, op->Px, op->Py, op->split_plane, pco, nrhs, so, &mv, &pcb, &ap,
                              &sb));
    *bytes = b + mv + pcb + ap + sb;
    return VIE_OK;
}

vie_status request_footprint(const int32_t grid[3], bool c64, const vie_pc_opts *pco, int32_t nrhs,
                             const vie_solve_opts *so, uint64_t *resident, uint64_t *build, uint64_t *run) {
    uint64_t held, transient, mv, pcb, ap, sb;
    int Px;
    op_bytes_estimate(grid[0], grid[1], grid[2], c64, &held, &transient, &Px);
    const int Py = fft_good_length(2 * grid[1] - 1), Hy = Py / 2 + 1, nz = grid[2];
    const bool fused = 3LL * nz * Py <= 2LL * FFT_BPT * 1024 &&
                       sizeof(c128) * ((size_t)6 * nz * Py + (size_t)6 * Hy * nz) <= max_lds();
    VIE_CHECK(footprint_parts(grid[0], grid[1], grid[2], Px, Py, nz <= 16 && !fused, pco, nrhs, so, &mv, &pcb, &ap,
                              &sb));
    *resident = held + pcb;                     // kept by a cached operator + preconditioner
    *build = transient;                         // the transformed embedding while the operator is built
    *run = sb + mv + ap + 2 * 16 * 3ULL * grid[0] * grid[1] * grid[2] * nrhs;  // workspace, scratch, e/b
    return VIE_OK;
}

extern "C" vie_status precond_info(vie_pc pc, vie_pc_info *info) {
    if (!pc || !info) return arg_error("precond_info: NULL argument");
    if (!pc->children.empty()) {  // boxes of several shapes / levels: sums over the groups
        vie_pc_info ci{};
        *info = vie_pc_info{};
        info->nboxes = pc->nboxes;
        for (vie_pc c : pc->children) {
            VIE_CHECK(precond_info(c, &ci));
            info->box_nx = std::max(info->box_nx, ci.box_nx);
            info->block_m = std::max(info->block_m, ci.block_m);
            info->active_m = std::max(info->active_m, ci.active_m);
            info->levels = std::max(info->levels, ci.levels);
            info->modes += ci.modes;
            info->stored_blocks += ci.stored_blocks;
            info->factor_bytes += ci.factor_bytes;
        }
        return VIE_OK;
    }
    info->nboxes = pc->nboxes;
    info->box_nx = pc->bx;
    info->block_m = pc->m_full;
    info->active_m = pc->m;
    info->levels = pc->levels;
    info->modes = pc->nboxes * pc->nm;
    info->stored_blocks = pc->nstored;
    size_t esz = pc->prec == VIE_C128 ? sizeof(c128) : pc->prec == VIE_C64 ? sizeof(c64) : sizeof(bf16c);
    info->factor_bytes = (int64_t)pc->nstored * pc->m * ((int64_t)pc->m * esz + sizeof(int));
    return VIE_OK;
}

extern "C" vie_status precond_destroy(vie_pc pc) {
    if (pc) delete pc;
    return VIE_OK;
}

extern "C" vie_status precond_apply(vie_pc pc, const void *r, void *z, int32_t nrhs, vie_prec prec, void *stream) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    if (!pc || !r || !z) return arg_error("precond_apply: NULL argument");
    if (nrhs < 1) return arg_error("precond_apply: nrhs must be >= 1");
    if (r == z) return arg_error("precond_apply: r and z must not overlap");
    return pc_apply(pc, r, z, nrhs, prec, (hipStream_t)stream);
}

vie_status solve_opts_check(const char *who, const vie_solve_opts &o) {
    const std::string w(who);
    if (!(o.tol > 0) || !std::isfinite(o.tol)) return arg_error(w + ": tol must be finite and > 0");
    if (o.restart < 1 || o.restart > VIE_MAX_RESTART)
        return arg_error(w + ": restart must be in [1, " + std::to_string(VIE_MAX_RESTART) + "]");
    if (o.maxit < 1) return arg_error(w + ": maxit must be >= 1");
    if (o.mode != VIE_MODE_FP64 && o.mode != VIE_MODE_MIXED && o.mode != VIE_MODE_MIXED_PC)
        return arg_error(w + ": unknown mode");
    return VIE_OK;
}

extern "C" vie_status vie_solve(vie_op op, vie_pc pc, const void *b, void *x, int32_t nrhs,
                                const vie_solve_opts *opts, vie_solve_stats *stats, void *stream) {
    StreamScope scope((hipStream_t)stream);  // buffers released in this call wait for its stream
    if (!op || !b || !x || !stats) return arg_error("vie_solve: NULL argument");
    if (nrhs < 1) return arg_error("vie_solve: nrhs must be >= 1");
    if (pc && pc->op != op) return arg_error("vie_solve: preconditioner built for another operator");
    vie_solve_opts o{1e-6, 50, 5000, VIE_MODE_FP64, 0};
    if (opts) o = *opts;
    VIE_CHECK(solve_opts_check("vie_solve", o));
    hipStream_t s = (hipStream_t)stream;
    vie_status st = solve_gmres(op, pc, (const c128 *)b, (c128 *)x, nrhs, &o, stats, s);
    hipError_t e = hipStreamSynchronize(s);
    if (st >= 0 && e != hipSuccess) {
        g_err = std::string("vie_solve: ") + hipGetErrorString(e);
        return VIE_EDEVICE;
    }
    return st;
}
