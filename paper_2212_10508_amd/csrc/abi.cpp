// C ABI of snapmd: context, workspace, argument validation and the entry points
// declared in include/snapmd.h.  Every step of the propagation runs in the HIP
// kernels of kernels.hip; this file only validates, uploads small parameter arrays
// and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/snapmd.h"
#include "kernels.h"
#include "snapmd_internal.h"

using namespace snapmd;

namespace {

constexpr double kKB = 8.617333262145179e-5;       // eV/K
constexpr double kMVV2E = 1.0364269652680506e-4;   // eV per amu A^2/ps^2

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
};

struct SnapDevTables {
    int J = -1;
    double *nrm = nullptr, *ymult = nullptr, *ycoef = nullptr, *bcg = nullptr;
    int *ystart = nullptr, *bstart = nullptr, *bel = nullptr;
    uint32_t *yidx = nullptr, *bidx = nullptr;
    std::vector<double> beta;  // coefficients ycoef was built for
    std::vector<double> ycoef_host;
    AdjointHost adj;
    double *adj_cgm = nullptr, *adj_coef = nullptr;
    int *adj_coef_off = nullptr, *adj_roles = nullptr;
};

}  // namespace

struct snapmd_ctx {
    int device = 0;
    std::string err;
    // batch
    DBuf<int> d_off;
    DBuf<double> d_box;
    std::vector<int> h_off;
    std::vector<double> h_box;
    // workspace
    size_t cap_atoms = 0;
    Work w;
    double *d_f = nullptr;  // force scratch [3][N]
    // per-system Langevin arrays
    DBuf<double> d_sig;
    DBuf<int64_t> d_step0;
    DBuf<int> d_noise;
    std::map<int, SnapDevTables> snap;
    std::vector<void *> allocs;
};

namespace {

int fail(snapmd_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, SNAPMD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

template <class T>
int dalloc(snapmd_ctx *ctx, T **p, size_t n) {
    if (*p) {
        (void)hipFree(*p);
        ctx->allocs.erase(std::remove(ctx->allocs.begin(), ctx->allocs.end(), (void *)*p), ctx->allocs.end());
        *p = nullptr;
    }
    if (n == 0) return SNAPMD_OK;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, SNAPMD_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
    }
    ctx->allocs.push_back((void *)*p);
    return SNAPMD_OK;
}

template <class T>
int ensure(snapmd_ctx *ctx, DBuf<T> &b, size_t n) {
    if (b.n >= n && b.p) return SNAPMD_OK;
    int rc = dalloc(ctx, &b.p, std::max<size_t>(n, 1));
    b.n = rc == SNAPMD_OK ? std::max<size_t>(n, 1) : 0;
    return rc;
}

template <class T>
int upload(snapmd_ctx *ctx, T *dst, const T *src, size_t n, hipStream_t st) {
    if (n == 0) return SNAPMD_OK;
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, st));
    return SNAPMD_OK;
}

int ensure_atoms(snapmd_ctx *ctx, size_t N) {
    if (N <= ctx->cap_atoms) return SNAPMD_OK;
    size_t cap = std::max<size_t>(N, 64);
    Work &w = ctx->w;
    w.Pcap = cap * kMaxNeigh;
    int rc;
    if ((rc = dalloc(ctx, &w.nbr, cap * kMaxNeigh))) return rc;
    if ((rc = dalloc(ctx, &w.cnt, cap))) return rc;
    if ((rc = dalloc(ctx, &w.poff, cap + 1))) return rc;
    if ((rc = dalloc(ctx, &w.pair_i, w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.pair_j, w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.rev, w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.rho, cap))) return rc;
    if ((rc = dalloc(ctx, &w.geo, 20 * w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.dedr, 3 * w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.u, (size_t)n_half(kMaxJ) * cap))) return rc;
    if ((rc = dalloc(ctx, &w.ytil, (size_t)n_half(kMaxJ) * cap))) return rc;
    if ((rc = dalloc(ctx, &ctx->d_f, 3 * cap))) return rc;
    ctx->cap_atoms = cap;
    return SNAPMD_OK;
}

// Validate the batch, upload it if it changed; fill bd.  min_half_box receives the
// smallest half box edge over all systems.
int prepare_batch(snapmd_ctx *ctx, const snapmd_batch *batch, BatchDev &bd, double &min_half_box,
                  hipStream_t st) {
    if (!batch) return fail(ctx, SNAPMD_EINVAL, "batch is NULL");
    if (batch->n_sys < 1) return fail(ctx, SNAPMD_EINVAL, "batch.n_sys must be >= 1 (got %d)", batch->n_sys);
    if (!batch->offset || !batch->box) return fail(ctx, SNAPMD_EINVAL, "batch.offset and batch.box must be set");
    const int S = batch->n_sys;
    if (batch->offset[0] != 0) return fail(ctx, SNAPMD_EINVAL, "batch.offset[0] must be 0");
    min_half_box = INFINITY;
    for (int s = 0; s < S; ++s) {
        if (batch->offset[s + 1] < batch->offset[s])
            return fail(ctx, SNAPMD_EINVAL, "batch.offset must be nondecreasing (system %d)", s);
        for (int a = 0; a < 3; ++a) {
            const double L = batch->box[3 * s + a];
            if (!(L > 0.0) || !std::isfinite(L))
                return fail(ctx, SNAPMD_EINVAL, "box edge %d of system %d must be finite and > 0", a, s);
            min_half_box = std::min(min_half_box, 0.5 * L);
        }
    }
    const int N = batch->offset[S];
    int rc;
    if ((rc = ensure_atoms(ctx, (size_t)N))) return rc;
    const bool same = (int)ctx->h_off.size() == S + 1 &&
                      std::equal(ctx->h_off.begin(), ctx->h_off.end(), batch->offset) &&
                      std::equal(ctx->h_box.begin(), ctx->h_box.end(), batch->box);
    if (!same) {
        if ((rc = ensure(ctx, ctx->d_off, (size_t)S + 1))) return rc;
        if ((rc = ensure(ctx, ctx->d_box, 3 * (size_t)S))) return rc;
        ctx->h_off.assign(batch->offset, batch->offset + S + 1);
        ctx->h_box.assign(batch->box, batch->box + 3 * S);
        if ((rc = upload(ctx, ctx->d_off.p, ctx->h_off.data(), S + 1, st))) return rc;
        if ((rc = upload(ctx, ctx->d_box.p, ctx->h_box.data(), 3 * (size_t)S, st))) return rc;
    }
    bd.N = N;
    bd.n_sys = S;
    bd.off = ctx->d_off.p;
    bd.box = ctx->d_box.p;
    return SNAPMD_OK;
}

int prepare_snap(snapmd_ctx *ctx, const snapmd_snap *s, double min_half_box, SnapDev &sd, hipStream_t st) {
    if (!s) return fail(ctx, SNAPMD_EINVAL, "snap is NULL");
    const int J = s->twojmax;
    if (J != 2 && J != 4 && J != 6 && J != 8)
        return fail(ctx, SNAPMD_EUNSUPPORTED, "twojmax must be one of 2, 4, 6, 8 (got %d)", J);
    const SnapTables &T = snap_tables(J);
    if (s->n_coeff != T.K)
        return fail(ctx, SNAPMD_EINVAL, "n_coeff must be %d for twojmax %d (got %d)", T.K, J, s->n_coeff);
    if (!s->beta) return fail(ctx, SNAPMD_EINVAL, "snap.beta is NULL");
    if (!(s->rcut > 0.0) || !(s->rmin0 >= 0.0) || !(s->rmin0 < s->rcut))
        return fail(ctx, SNAPMD_EINVAL, "need 0 <= rmin0 < rcut (rcut %g, rmin0 %g)", s->rcut, s->rmin0);
    if (!(s->rfac0 > 0.0 && s->rfac0 < 1.0)) return fail(ctx, SNAPMD_EINVAL, "need 0 < rfac0 < 1 (got %g)", s->rfac0);
    if (!(s->rcut < min_half_box))
        return fail(ctx, SNAPMD_EINVAL, "rcut %g must be < half the smallest box edge %g", s->rcut, min_half_box);
    for (int k = 0; k <= T.K; ++k)
        if (!std::isfinite(s->beta[k])) return fail(ctx, SNAPMD_EINVAL, "beta[%d] is not finite", k);
    SnapDevTables &D = ctx->snap[J];
    int rc;
    if (D.J != J) {
        D.J = J;
        if ((rc = dalloc(ctx, &D.nrm, T.nh)) || (rc = dalloc(ctx, &D.ymult, T.nh)) ||
            (rc = dalloc(ctx, &D.ystart, T.ystart.size())) || (rc = dalloc(ctx, &D.yidx, T.yidx.size())) ||
            (rc = dalloc(ctx, &D.ycoef, T.ycg.size())) || (rc = dalloc(ctx, &D.bstart, T.bstart.size())) ||
            (rc = dalloc(ctx, &D.bidx, T.bidx.size())) || (rc = dalloc(ctx, &D.bel, T.bel.size())) ||
            (rc = dalloc(ctx, &D.bcg, T.bcg.size())))
            return rc;
        HIPCHK(hipMemcpy(D.nrm, T.nrm.data(), T.nh * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.ymult, T.ymult.data(), T.nh * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.ystart, T.ystart.data(), T.ystart.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.yidx, T.yidx.data(), T.yidx.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.bstart, T.bstart.data(), T.bstart.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.bidx, T.bidx.data(), T.bidx.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.bel, T.bel.data(), T.bel.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(D.bcg, T.bcg.data(), T.bcg.size() * sizeof(double), hipMemcpyHostToDevice));
        D.beta.clear();
    }
    if (D.beta.size() != (size_t)T.K + 1 || !std::equal(D.beta.begin(), D.beta.end(), s->beta)) {
        D.beta.assign(s->beta, s->beta + T.K + 1);
        D.ycoef_host.resize(T.ycg.size());
        for (size_t t = 0; t < T.ycg.size(); ++t) {
            const int b = T.yblock[t];
            D.ycoef_host[t] = T.ycg[t] * T.zb_wt[b] * D.beta[1 + T.zb_canon[b]];
        }
        if ((rc = upload(ctx, D.ycoef, D.ycoef_host.data(), D.ycoef_host.size(), st))) return rc;
    }
    {
        AdjointHost &A = D.adj;
        const int oldJ = A.J;
        adjoint_tables(J, s->beta, A);
        if (oldJ != J) {
            if ((rc = dalloc(ctx, &D.adj_cgm, A.cgm.size())) || (rc = dalloc(ctx, &D.adj_roles, A.roles.size())) ||
                (rc = dalloc(ctx, &D.adj_coef, A.coef.size())) ||
                (rc = dalloc(ctx, &D.adj_coef_off, A.coef_off.size())))
                return rc;
            HIPCHK(hipMemcpy(D.adj_cgm, A.cgm.data(), A.cgm.size() * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(D.adj_roles, A.roles.data(), A.roles.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(D.adj_coef_off, A.coef_off.data(), A.coef_off.size() * sizeof(int),
                             hipMemcpyHostToDevice));
        }
        if (A.coef_changed) {
            if ((rc = upload(ctx, D.adj_coef, A.coef.data(), A.coef.size(), st))) return rc;
            A.coef_changed = false;
        }
        sd.adj = AdjointDev{D.adj_cgm, D.adj_coef, D.adj_coef_off, D.adj_roles, A.role_len};
    }
    sd.J = J;
    sd.K = T.K;
    sd.nh = T.nh;
    sd.gp = SnapGeoParams{s->rcut, s->rfac0, s->rmin0};
    sd.beta0 = s->beta[0];
    sd.nrm = D.nrm;
    sd.ymult = D.ymult;
    sd.ystart = D.ystart;
    sd.yidx = D.yidx;
    sd.ycoef = D.ycoef;
    sd.bstart = D.bstart;
    sd.bidx = D.bidx;
    sd.bel = D.bel;
    sd.bcg = D.bcg;
    return SNAPMD_OK;
}

int prepare_fs(snapmd_ctx *ctx, const snapmd_fs *fs, double min_half_box, FsParams &fp) {
    if (!fs) return fail(ctx, SNAPMD_EINVAL, "fs is NULL");
    if (!(fs->d > 0.0) || !(fs->c > 0.0)) return fail(ctx, SNAPMD_EINVAL, "FS cutoffs d and c must be > 0");
    if (!(std::max(fs->d, fs->c) < min_half_box))
        return fail(ctx, SNAPMD_EINVAL, "FS cutoff %g must be < half the smallest box edge %g",
                    std::max(fs->d, fs->c), min_half_box);
    fp = FsParams{fs->A, fs->d, fs->c, fs->c0, fs->c1, fs->c2};
    return SNAPMD_OK;
}

int check_launch(snapmd_ctx *ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, SNAPMD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return SNAPMD_OK;
}

// Force of the chosen potential at x into f (overwrite), e_atom (nullable, overwrite).
void enqueue_forces(snapmd_ctx *ctx, int potential, const BatchDev &bd, const double *x, const FsParams *fp,
                    const SnapDev *sd, double *f, double *e_atom, hipStream_t st) {
    double rc = 0.0;
    if (fp) rc = std::max(fp->d, fp->c);
    if (potential == SNAPMD_POT_FS_SNAP) rc = std::max(rc, sd->gp.rcut);
    launch_neighbors(bd, x, rc, ctx->w, st);
    launch_fs(bd, x, *fp, ctx->w, f, e_atom, 0, st);
    if (potential == SNAPMD_POT_FS_SNAP) launch_snap(sd->J, bd, x, *sd, ctx->w, f, e_atom, 1, st);
}

}  // namespace

// ===========================================================================
extern "C" {

int snapmd_create(snapmd_ctx **out, int hip_device) {
    if (!out) return SNAPMD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return SNAPMD_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess) return SNAPMD_EHIP;
    snapmd_ctx *ctx = new snapmd_ctx();
    ctx->device = hip_device;
    adjoint_init_attributes();
    if (dalloc(ctx, &ctx->w.status, 1) != SNAPMD_OK || hipMemset(ctx->w.status, 0, sizeof(int)) != hipSuccess) {
        snapmd_destroy(ctx);
        return SNAPMD_ENOMEM;
    }
    *out = ctx;
    return SNAPMD_OK;
}

void snapmd_destroy(snapmd_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (void *p : ctx->allocs) (void)hipFree(p);
    delete ctx;
}

const char *snapmd_last_error(const snapmd_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int snapmd_sync(snapmd_ctx *ctx, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    int st = 0;
    HIPCHK(hipMemcpy(&st, ctx->w.status, sizeof(int), hipMemcpyDeviceToHost));
    if (st) {
        HIPCHK(hipMemset(ctx->w.status, 0, sizeof(int)));
        if (st & 1) return fail(ctx, SNAPMD_EOVERFLOW, "an atom has more than %d neighbours", kMaxNeigh);
        return fail(ctx, SNAPMD_EINVAL, "inconsistent neighbour list (status %d)", st);
    }
    return SNAPMD_OK;
}

int snap_forces(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch, const double *x, double *f,
                double *e_atom, uint32_t flags, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (!x || !f) return fail(ctx, SNAPMD_EINVAL, "x and f must be device pointers");
    BatchDev bd;
    double mh;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    launch_neighbors(bd, x, snap->rcut, ctx->w, st);
    launch_snap(sd.J, bd, x, sd, ctx->w, f, e_atom, (flags & SNAPMD_ACCUMULATE) ? 1 : 0, st);
    return check_launch(ctx);
}

int eam_forces(snapmd_ctx *ctx, const snapmd_fs *fs, const snapmd_batch *batch, const double *x, double *f,
               double *e_atom, uint32_t flags, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (!x || !f) return fail(ctx, SNAPMD_EINVAL, "x and f must be device pointers");
    BatchDev bd;
    double mh;
    FsParams fp;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    launch_neighbors(bd, x, std::max(fp.d, fp.c), ctx->w, st);
    launch_fs(bd, x, fp, ctx->w, f, e_atom, (flags & SNAPMD_ACCUMULATE) ? 1 : 0, st);
    return check_launch(ctx);
}

int langevin_steps(snapmd_ctx *ctx, int potential, const snapmd_snap *snap, const snapmd_fs *fs,
                   const snapmd_batch *batch, const snapmd_langevin *lang, int32_t n_steps, double *x, double *p,
                   double *f_out, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (potential != SNAPMD_POT_FS && potential != SNAPMD_POT_FS_SNAP)
        return fail(ctx, SNAPMD_EINVAL, "potential must be SNAPMD_POT_FS or SNAPMD_POT_FS_SNAP");
    if (!x || !p) return fail(ctx, SNAPMD_EINVAL, "x and p must be device pointers");
    if (n_steps < 0) return fail(ctx, SNAPMD_EINVAL, "n_steps must be >= 0");
    if (!lang) return fail(ctx, SNAPMD_EINVAL, "lang is NULL");
    if (lang->scheme != 0) return fail(ctx, SNAPMD_EINVAL, "only scheme 0 (BAOAB) is supported");
    if (!(lang->dt > 0.0) || !(lang->gamma >= 0.0) || !(lang->mass > 0.0))
        return fail(ctx, SNAPMD_EINVAL, "need dt > 0, gamma >= 0, mass > 0");
    BatchDev bd;
    double mh;
    FsParams fp;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if (potential == SNAPMD_POT_FS_SNAP && (rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    const int S = bd.n_sys;
    if (!lang->T_sys || !lang->step0_sys || !lang->noise_id_sys)
        return fail(ctx, SNAPMD_EINVAL, "lang.T_sys, step0_sys and noise_id_sys must be set");
    const double c1 = std::exp(-lang->gamma * lang->dt);
    std::vector<double> sig(S);
    for (int s = 0; s < S; ++s) {
        if (!(lang->T_sys[s] >= 0.0)) return fail(ctx, SNAPMD_EINVAL, "T_sys[%d] must be >= 0", s);
        if (lang->noise_id_sys[s] < 0) return fail(ctx, SNAPMD_EINVAL, "noise_id_sys[%d] must be >= 0", s);
        sig[s] = std::sqrt((1.0 - c1 * c1) * lang->mass * kKB * lang->T_sys[s] / kMVV2E);
    }
    if ((rc = ensure(ctx, ctx->d_sig, S)) || (rc = ensure(ctx, ctx->d_step0, S)) || (rc = ensure(ctx, ctx->d_noise, S)))
        return rc;
    if ((rc = upload(ctx, ctx->d_sig.p, sig.data(), S, st))) return rc;
    if ((rc = upload(ctx, ctx->d_step0.p, lang->step0_sys, S, st))) return rc;
    if ((rc = upload(ctx, ctx->d_noise.p, lang->noise_id_sys, S, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    LangevinDev ld{lang->dt, c1, lang->mass, lang->seed, ctx->d_sig.p, ctx->d_step0.p, ctx->d_noise.p};
    double *f = ctx->d_f;
    enqueue_forces(ctx, potential, bd, x, &fp, &sd, f, nullptr, st);
    for (int s = 0; s < n_steps; ++s) {
        launch_baoab_pre(bd, x, p, f, ld, s, st);
        enqueue_forces(ctx, potential, bd, x, &fp, &sd, f, nullptr, st);
        launch_baoab_post(bd, p, f, lang->dt, st);
    }
    if (f_out) HIPCHK(hipMemcpyAsync(f_out, f, 3 * (size_t)bd.N * sizeof(double), hipMemcpyDeviceToDevice, st));
    return check_launch(ctx);
}

int parareal_iterate(snapmd_ctx *ctx, const snapmd_snap *, const snapmd_fs *, const snapmd_batch *,
                     const snapmd_langevin *, int32_t, int32_t, int32_t *, double *, double *, double *, double *,
                     double, double *, void *) {
    return fail(ctx, SNAPMD_EUNSUPPORTED, "parareal_iterate: not built yet");
}

int snap_beta_grad(snapmd_ctx *ctx, const snapmd_snap *, const snapmd_batch *, const double *, const double *,
                   double *, double *, void *) {
    return fail(ctx, SNAPMD_EUNSUPPORTED, "snap_beta_grad: not built yet");
}

// Bispectrum of every atom, B[t][i] (device, [K][n_atoms]); used by tests and the
// coefficient gradient.
int snapmd_bispectrum(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch, const double *x,
                      double *B, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (!x || !B) return fail(ctx, SNAPMD_EINVAL, "x and B must be device pointers");
    BatchDev bd;
    double mh;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    launch_neighbors(bd, x, snap->rcut, ctx->w, st);
    launch_snap_density(sd.J, bd, x, sd, ctx->w, st);
    launch_bispectrum(bd, sd, ctx->w, B, st);
    return check_launch(ctx);
}

}  // extern "C"
