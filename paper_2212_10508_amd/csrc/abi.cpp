// C ABI of snapmd: context, workspace, argument validation and the entry points
// declared in include/snapmd.h.  Every step of the propagation runs in the HIP
// kernels of kernels.hip; this file only validates, uploads small parameter arrays
// and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
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
    int *ystart = nullptr, *bstart = nullptr, *bel = nullptr, *ychunk = nullptr;
    int n_ychunk = 0;
    uint32_t *yidx = nullptr, *bidx = nullptr;
    std::vector<double> beta;  // coefficients ycoef was built for
    std::vector<double> ycoef_host;
    AdjointHost adj;
    double *adj_cgm = nullptr, *adj_coef = nullptr;
    int *adj_coef_off = nullptr, *adj_roles = nullptr, *adj_roles8 = nullptr;
};

}  // namespace

struct snapmd_ctx {
    int device = 0;
    int n_cus = 256;  // compute units of the device
    std::string err;
    // batch
    DBuf<int> d_off;
    DBuf<double> d_box;
    std::vector<int> h_off;
    std::vector<double> h_box;
    // workspace
    size_t cap_atoms = 0, cap_atoms_c = 0, cap_atoms_cs = 0;  // fine, coarse lists, coarse SNAP
    Work w, wc;                                   // SNAP / second-stream Finnis-Sinclair workspaces
    double *d_f = nullptr, *d_fc = nullptr;       // their force scratch [3][N]
    // the second SNAP workspace of a parareal iteration (its odd slab chunks run on their
    // own stream beside the even ones); fine_streams 1 runs every chunk on the caller's
    Work w2;
    double *d_f2 = nullptr;
    size_t cap_atoms2 = 0;
    int fine_streams = 2;
    hipStream_t fine2_stream = nullptr;
    // per-system Langevin arrays
    DBuf<double> d_sig, d_sb0, d_sb1;
    DBuf<int64_t> d_step0;
    DBuf<int64_t> seg_step0[3];                   // step offsets advanced by a segmented replay (per workspace)
    DBuf<int> d_noise;
    std::map<int, SnapDevTables> snap;
    std::map<int, KernelShape> shapes;            // kernel shapes set per twojmax (default otherwise)
    std::vector<void *> allocs;
    // parareal buffers
    DBuf<double> pr_xf, pr_pf, pr_xc, pr_pc;     // [3][S*N] fine / coarse copies of prev slabs
    DBuf<double> sw_x, sw_p, sw_out;
    DBuf<unsigned long long> sw_gx, sw_gdfe, sw_gpart;  // multi-workgroup sweep exchange words
    DBuf<int> sw_abort;
    double *h_out = nullptr;                      // pinned [16]: sweep results [0, 8), sweep init [8, 16)
    // pipelined parareal iterations (parareal_iterate_async) whose results are not collected
    static constexpr int kAsyncSlots = 4;
    DBuf<double> sw_out_ring;                     // [kAsyncSlots][8] sweep state of each iteration in flight
    static constexpr int kAsyncStride = 24;
    double *h_async = nullptr;                    // pinned [kAsyncSlots][24]: results [0, 8), init [8, 16),
                                                  // neighbour-list status (an int) at 16
    hipEvent_t async_ev[kAsyncSlots] = {};        // result of slot j copied to the host
    struct AsyncIt {
        int slot;                                 // -1: finished at the call (result below)
        int rc;
        double delta;
        int32_t n_fi;
    };
    std::deque<AsyncIt> async_q;
    uint64_t async_seq = 0;
    std::vector<hipEvent_t> sweep_chunk_ev;       // the last iteration's sweep of chunk c enqueued up to its end
    std::vector<uint64_t> chain_key;              // window, parameters and buffers of the last pipelined iteration
    hipEvent_t chain_end = nullptr;               // the last pipelined iteration done (one of async_ev)
    std::vector<uint64_t> lang_key;               // the per-system Langevin arrays last uploaded
    DBuf<double> sw_noise;                        // Gaussians of the current window
    // parareal over several systems: offsets, windows, jumps in the slot layout, entry
    // sources, sweep arguments and results
    DBuf<int> m_off;
    DBuf<int2> m_win;
    DBuf<int4> m_src;
    DBuf<double> m_jq, m_jp, m_out;
    DBuf<unsigned char> m_tab;
    // device-resident adaptive driver
    DBuf<double> dr_qprev, dr_pprev, dr_out_init, dr_out_it, dr_sig, dr_sb, dr_box, dr_logd;
    DBuf<DrvState> dr_st;
    DBuf<int> dr_act, dr_roff, dr_eoff, dr_noise, dr_err;
    DBuf<int4> dr_ent, dr_cells, dr_logi;
    DBuf<int64_t> dr_step0;
    DBuf<unsigned char> dr_tab_init, dr_tab_it;
    DBuf<double> gB;                              // [K][N] bispectrum / its variation
    // cell grids of the current batch for the last list cutoff, one set per workspace
    struct CellState {
        DBuf<int4> d_cells;
        std::vector<double> key;
        int n_cells = 0;
        bool any = false;
    } cs, csc, cs2;
    std::vector<uint64_t> noise_key;              // (n_in, S, L, N, seed, noise_id) it holds
    KernelProf prof;
    // captured launch sequences of run_langevin, keyed by everything baked into them
    int use_graphs = 1;
    struct GraphEntry {
        std::vector<uint64_t> key;
        hipGraphExec_t exec;
        uint64_t last_use;
    };
    std::vector<GraphEntry> graphs[3];   // one cache per workspace (w, wc, w2): they may be
    hipStream_t cap_stream[3] = {};      // launched from different host threads
    std::mutex err_mu;
    hipStream_t sweep_stream = nullptr;  // the coarse sweep, overlapping the batched propagation
    hipStream_t coarse_stream = nullptr; // the batched coarse propagation of a parareal iteration
    std::vector<hipEvent_t> pipe_ev;
    uint64_t graph_clock[3] = {};
    std::vector<int> chunk_override;     // slab chunks set by snapmd_set_chunk_plan (empty: built in)
    int sweep_k_override = 0;            // sweep workgroups set by snapmd_set_sweep_workgroups (0: built in)
    DBuf<int4> d_ws;                     // Wigner-Seitz lattice of each system
    DBuf<unsigned long long> d_fmax;     // max |F|^2 of the relaxation
    unsigned char *scratch = nullptr;    // this device's address of the allocation-free scratch array
    AdjointHost na_adj;                  // host tables of the allocation-free SNAP forces
    // coarse propagator of parareal_iterate: Finnis-Sinclair, plus SNAP when set
    bool coarse_snap_on = false;
    bool coarse_fs_on = false;           // coarse Finnis-Sinclair parameters of their own
    snapmd_fs coarse_fs{};
    snapmd_snap coarse_snap{};
    std::vector<double> coarse_beta;
};

namespace {

int fail(snapmd_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        std::lock_guard<std::mutex> lk(c->err_mu);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, SNAPMD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// Wait (on the host) for every pipelined parareal iteration in flight; their results stay
// queued for snapmd_parareal_collect.  Every entry point that may reallocate, rewrite or
// drop what such an iteration uses calls this first.
int drain(snapmd_ctx *ctx) {
    if (ctx->chain_end) {
        const hipError_t e = hipEventSynchronize(ctx->chain_end);
        ctx->chain_end = nullptr;
        ctx->chain_key.clear();
        if (e != hipSuccess)
            return fail(ctx, SNAPMD_EHIP, "waiting for a pipelined parareal iteration failed: %s",
                        hipGetErrorString(e));
    }
    return SNAPMD_OK;
}

void drop_graphs(snapmd_ctx *ctx) {
    // a replay may still be queued on the caller's or the context's streams
    bool any = false;
    for (auto &c : ctx->graphs) any = any || !c.empty();
    if (any) (void)hipDeviceSynchronize();
    for (auto &c : ctx->graphs) {
        for (auto &g : c) (void)hipGraphExecDestroy(g.exec);
        c.clear();
    }
}

// (Re)allocate a device buffer.  Freeing one invalidates every captured graph.
template <class T>
int dalloc(snapmd_ctx *ctx, T **p, size_t n) {
    if (*p) {
        drop_graphs(ctx);
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

// The SNAP workspace w (ctx->w or ctx->w2) with its force buffer f and capacity cap_atoms.
int ensure_atoms_ws(snapmd_ctx *ctx, Work &w, double *&f, size_t &cap_atoms, size_t N) {
    if (N <= cap_atoms) return SNAPMD_OK;
    size_t cap = std::max<size_t>(N, 64);
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
    if ((rc = dalloc(ctx, &w.ell, 6 * w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.nbr_t, w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.ph, 3 * cap))) return rc;
    if ((rc = dalloc(ctx, &w.dedr, 3 * w.Pcap))) return rc;
    if ((rc = dalloc(ctx, &w.u, (size_t)n_half(kMaxJ) * cap))) return rc;
    if ((rc = dalloc(ctx, &w.ytil, (size_t)n_half(kMaxJ) * cap))) return rc;
    if ((rc = dalloc(ctx, &w.epart, (size_t)kMaxYChunks * cap))) return rc;
    if ((rc = dalloc(ctx, &f, 3 * cap))) return rc;
    if ((rc = dalloc(ctx, &w.xref, 3 * cap))) return rc;
    if ((rc = dalloc(ctx, &w.cell_of, cap))) return rc;
    if ((rc = dalloc(ctx, &w.cell_atoms, cap))) return rc;
    cap_atoms = cap;
    return SNAPMD_OK;
}

int ensure_atoms(snapmd_ctx *ctx, size_t N) { return ensure_atoms_ws(ctx, ctx->w, ctx->d_f, ctx->cap_atoms, N); }

// Index of a workspace in the per-workspace state (graph caches, cell grids, offsets).
int ws_index(const snapmd_ctx *ctx, const Work &w) { return &w == &ctx->wc ? 1 : &w == &ctx->w2 ? 2 : 0; }

// Workspace of the Finnis-Sinclair propagation that runs beside the SNAP one (its own
// neighbour lists and force buffer; the error bits are shared).
int ensure_atoms_coarse(snapmd_ctx *ctx, size_t N, bool snap = false) {
    Work &w = ctx->wc;
    w.status = ctx->w.status;
    int rc;
    if (!w.flag) {
        if ((rc = dalloc(ctx, &w.flag, 1))) return rc;
        HIPCHK(hipMemset(w.flag, 0, sizeof(int)));
    }
    // the SNAP passes (a coarse potential with SNAP) index their pair buffers with the
    // list's pair capacity, so both sets share one atom capacity
    const size_t need = std::max<size_t>(N, 64);
    const bool grow_list = need > ctx->cap_atoms_c;
    const bool grow_snap = snap && (need > ctx->cap_atoms_cs || ctx->cap_atoms_cs < ctx->cap_atoms_c);
    if (!grow_list && !grow_snap) return SNAPMD_OK;
    const size_t cap = std::max(need, ctx->cap_atoms_c);
    if (grow_list) {
        w.Pcap = cap * kMaxNeigh;
        if ((rc = dalloc(ctx, &w.nbr, cap * kMaxNeigh)) || (rc = dalloc(ctx, &w.cnt, cap)) ||
            (rc = dalloc(ctx, &w.poff, cap + 1)) || (rc = dalloc(ctx, &w.pair_i, w.Pcap)) ||
            (rc = dalloc(ctx, &w.pair_j, w.Pcap)) || (rc = dalloc(ctx, &w.rev, w.Pcap)) ||
            (rc = dalloc(ctx, &w.rho, cap)) || (rc = dalloc(ctx, &ctx->d_fc, 3 * cap)) ||
            (rc = dalloc(ctx, &w.xref, 3 * cap)) || (rc = dalloc(ctx, &w.cell_of, cap)) ||
            (rc = dalloc(ctx, &w.cell_atoms, cap)) || (rc = dalloc(ctx, &w.ph, 3 * cap)))
            return rc;
        ctx->cap_atoms_c = cap;
    }
    if (snap || (ctx->cap_atoms_cs > 0 && grow_list)) {
        const size_t Pc = cap * kMaxNeigh;
        if ((rc = dalloc(ctx, &w.geo, 20 * Pc)) || (rc = dalloc(ctx, &w.ell, 6 * Pc)) ||
            (rc = dalloc(ctx, &w.nbr_t, Pc)) || (rc = dalloc(ctx, &w.dedr, 3 * Pc)) ||
            (rc = dalloc(ctx, &w.u, (size_t)n_half(kMaxJ) * cap)) ||
            (rc = dalloc(ctx, &w.ytil, (size_t)n_half(kMaxJ) * cap)) ||
            (rc = dalloc(ctx, &w.epart, (size_t)kMaxYChunks * cap)))
            return rc;
        ctx->cap_atoms_cs = cap;
    }
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
    bd.max_sys = 0;
    for (int q = 0; q < S; ++q) bd.max_sys = std::max(bd.max_sys, ctx->h_off[q + 1] - ctx->h_off[q]);
    bd.off = ctx->d_off.p;
    bd.box = ctx->d_box.p;
    return SNAPMD_OK;
}

int prepare_snap(snapmd_ctx *ctx, const snapmd_snap *s, double min_half_box, SnapDev &sd, hipStream_t st) {
    if (!s) return fail(ctx, SNAPMD_EINVAL, "snap is NULL");
    const int J = s->twojmax;
    if (J < 2 || J > kMaxJ || (J & 1))
        return fail(ctx, SNAPMD_EUNSUPPORTED, "twojmax must be one of 2, 4, ..., 14 (got %d)", J);
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
        {
            // output-element chunks of about equal term counts for the chunked adjoint
            const int nc = std::min(kMaxYChunks, T.nh);
            const double per = (double)T.ystart[T.nh] / nc;
            std::vector<int> ch{0};
            for (int e = 0; e < T.nh && (int)ch.size() < nc; ++e)
                if (T.ystart[e + 1] >= per * (double)ch.size() && e + 1 > ch.back()) ch.push_back(e + 1);
            if (ch.back() != T.nh) ch.push_back(T.nh);
            D.n_ychunk = (int)ch.size() - 1;
            if ((rc = dalloc(ctx, &D.ychunk, ch.size()))) return rc;
            HIPCHK(hipMemcpy(D.ychunk, ch.data(), ch.size() * sizeof(int), hipMemcpyHostToDevice));
        }
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
    if (J <= kMaxJLds) {  // the LDS-tiled adjoint's tables (above, the coupling program serves)
        AdjointHost &A = D.adj;
        const int oldJ = A.J;
        adjoint_tables(J, s->beta, A);
        if (oldJ != J) {
            if ((rc = dalloc(ctx, &D.adj_cgm, A.cgm.size())) || (rc = dalloc(ctx, &D.adj_roles, A.roles.size())) ||
                (rc = dalloc(ctx, &D.adj_roles8, A.roles8.size())) || (rc = dalloc(ctx, &D.adj_coef, A.coef.size())) ||
                (rc = dalloc(ctx, &D.adj_coef_off, A.coef_off.size())))
                return rc;
            HIPCHK(hipMemcpy(D.adj_cgm, A.cgm.data(), A.cgm.size() * sizeof(double), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(D.adj_roles, A.roles.data(), A.roles.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(D.adj_roles8, A.roles8.data(), A.roles8.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(D.adj_coef_off, A.coef_off.data(), A.coef_off.size() * sizeof(int),
                             hipMemcpyHostToDevice));
        }
        if (A.coef_changed) {
            if ((rc = upload(ctx, D.adj_coef, A.coef.data(), A.coef.size(), st))) return rc;
            A.coef_changed = false;
        }
        sd.adj = AdjointDev{D.adj_cgm, D.adj_coef, D.adj_coef_off, D.adj_roles, A.role_len, D.adj_roles8,
                            A.role_len8};
    }
    {
        auto it = ctx->shapes.find(J);
        sd.shape = it != ctx->shapes.end() ? it->second : KernelShape{};
        sd.simds = 4 * std::max(ctx->n_cus, 1);
        if (J > kMaxJLds) sd.shape = KernelShape{45, 0, 12, 1};
    }
    sd.J = J;
    sd.K = T.K;
    sd.nh = T.nh;
    sd.gp = SnapGeoParams{s->rcut, s->rfac0, s->rmin0};
    sd.beta0 = s->beta[0];
    sd.nrm = D.nrm;
    sd.ymult = D.ymult;
    sd.ystart = D.ystart;
    sd.ychunk = D.ychunk;
    sd.n_ychunk = D.n_ychunk;
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

// Finnis-Sinclair parameters of the coarse propagator: those of snapmd_set_coarse_fs when
// set, else the fine potential's own (fp).
int coarse_fs(snapmd_ctx *ctx, const FsParams &fp, double min_half_box, FsParams &fpc) {
    if (!ctx->coarse_fs_on) {
        fpc = fp;
        return SNAPMD_OK;
    }
    return prepare_fs(ctx, &ctx->coarse_fs, min_half_box, fpc);
}

int check_launch(snapmd_ctx *ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, SNAPMD_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return SNAPMD_OK;
}

// Force of the chosen potential at x into f (overwrite), e_atom (nullable, overwrite).
constexpr double kSkin = 0.3;       // Verlet skin of the batched path (A)
constexpr double kSweepSkin = 0.5;  // Verlet skin of the LDS-resident coarse sweep (A)

// Chunk sizes of a parareal iteration over S slabs of N atoms.  The SNAP adjoint runs
// one 64-atom workgroup per CU at a time, so a chunk costs whole rounds: m_r = the most
// slabs that fit r rounds, counting two CUs per chiplet as taken by the work running
// beside the propagation (the sweep's workgroups).  Chunks of m_2 slabs, then the rest
// split so that the last chunk has m_1 - 1 slabs: the sweep (which starts after the first
// chunk) keeps pace and the part of it left after the last propagation is short.  Where that gives a single chunk,
// sizes in the ratio 4 : 3 : 2 : 1 are used instead.
std::vector<int> chunk_plan(int S, int N, int cus) {
    const long per = (long)std::max(cus - 16, 8) * 64;
    const int m1 = (int)std::max(1L, per / std::max(N, 1)), m2 = (int)std::max(1L, 2 * per / std::max(N, 1));
    std::vector<int> sz;
    int left = S;
    if (left > 0) {
        sz.push_back(std::min(left, m2));
        left -= sz.back();
    }
    while (left > m2 + m1) {
        sz.push_back(m2);
        left -= m2;
    }
    const int last = std::max(1, m1 - 1);
    if (left > last) {
        sz.push_back(left - last);
        left = last;
    }
    if (left > 0) sz.push_back(left);
    if (sz.size() > 1 || S < 2) return sz;
    const int G = std::min(S, 4);
    const int W = G * (G + 1) / 2;
    sz.assign(G, 0);
    int used = 0;
    for (int c = 0; c < G; ++c) {
        sz[c] = std::max(1, S * (G - c) / W);
        used += sz[c];
    }
    for (int c = 0; used > S; c = (c + 1) % G)  // trim (only possible when S < W)
        if (sz[c] > 1) { --sz[c]; --used; }
    for (int c = 0; used < S; c = (c + 1) % G) { ++sz[c]; ++used; }
    return sz;
}

// The chunks of a window of S slabs: the plan set by snapmd_set_chunk_plan when it covers
// exactly S slabs, else the built-in one.
std::vector<int> window_plan(const snapmd_ctx *ctx, int S, int N) {
    int tot = 0;
    for (int v : ctx->chunk_override) tot += v;
    if (!ctx->chunk_override.empty() && tot == S) return ctx->chunk_override;
    return chunk_plan(S, N, ctx->n_cus);
}

// Cell grids (cell edge >= list cutoff rl, >= 3 cells per edge, else brute force) of the
// current batch; rebuilt when the batch or the cutoff changes.
int prepare_cells(snapmd_ctx *ctx, Work &w, BatchDev &bd, double rl, hipStream_t st) {
    const int wi = ws_index(ctx, w);
    snapmd_ctx::CellState &cs = wi == 1 ? ctx->csc : wi == 2 ? ctx->cs2 : ctx->cs;
    std::vector<double> key(ctx->h_box.begin(), ctx->h_box.end());
    key.insert(key.end(), ctx->h_off.begin(), ctx->h_off.end());
    key.push_back(rl);
    if (key != cs.key) {
        const int S = (int)ctx->h_off.size() - 1;
        std::vector<int4> ci(S);
        int C = 0;
        bool any = false;
        for (int s = 0; s < S; ++s) {
            int n3[3];
            for (int a = 0; a < 3; ++a) n3[a] = (int)std::floor(ctx->h_box[3 * s + a] / rl);
            const int natoms = ctx->h_off[s + 1] - ctx->h_off[s];
            // cells pay off for systems above a few hundred atoms
            if (n3[0] >= 3 && n3[1] >= 3 && n3[2] >= 3 && natoms >= 500) {
                ci[s] = make_int4(n3[0], n3[1], n3[2], C);
                C += n3[0] * n3[1] * n3[2];
                any = true;
            } else {
                ci[s] = make_int4(0, 0, 0, C);
            }
        }
        int rc;
        if ((rc = ensure(ctx, cs.d_cells, (size_t)S))) return rc;
        if ((rc = upload(ctx, cs.d_cells.p, ci.data(), S, st))) return rc;
        cs.n_cells = C;
        cs.any = any;
        cs.key = key;
    }
    if (cs.any && (size_t)cs.n_cells + 1 > w.cap_cells) {
        const int C = cs.n_cells;
        int rc;
        if ((rc = dalloc(ctx, &w.cell_cnt, C + 1)) || (rc = dalloc(ctx, &w.cell_fill, C + 1)) ||
            (rc = dalloc(ctx, &w.cell_start, C + 1)))
            return rc;
        w.cap_cells = C + 1;
    }
    bd.cells = cs.any ? cs.d_cells.p : nullptr;
    bd.n_cells = cs.any ? cs.n_cells : 0;
    return SNAPMD_OK;
}

// launch_neighbors with the cell grids of the batch
int neighbors(snapmd_ctx *ctx, Work &w, const BatchDev &bd0, const double *x, double rc, bool force,
              hipStream_t st, bool in_step = false) {
    BatchDev bd = bd0;
    int r;
    if (!bd.cells_given && (r = prepare_cells(ctx, w, bd, rc + kSkin, st))) return r;
    // within a propagation step the displacement test ran in k_baoab_pre and k_fs_rho
    // clears the rebuild flag
    launch_neighbors(bd, x, rc, w, st, force, kSkin, in_step && !force, in_step);
    return SNAPMD_OK;
}

// Forces of a propagation step (e_atom not wanted).  For FS + SNAP the Finnis-Sinclair
// terms ride along the SNAP passes over the same list (the density term in the slot
// table, rho and F'(rho) in the density pass, the pair force in the gather), so the step
// is one chain of kernels.  With p_kick the closing half kick of the step is applied too
// (by the SNAP gather, or by a kernel of its own after the Finnis-Sinclair force).
void enqueue_forces(snapmd_ctx *ctx, Work &w, int potential, const BatchDev &bd, const double *x,
                    const FsParams *fp, const SnapDev *sd, double *f, hipStream_t st, bool fresh = true,
                    double *p_kick = nullptr, double dt = 0.0, const StepOpen *open = nullptr) {
    double rc = 0.0;
    if (fp) rc = std::max(fp->d, fp->c);
    if (potential == SNAPMD_POT_FS_SNAP) rc = std::max(rc, sd->gp.rcut);
    ctx->prof.begin(PROF_NEIGH, st);
    (void)neighbors(ctx, w, bd, x, rc, fresh, st, true);
    ctx->prof.end(st);
    if (potential == SNAPMD_POT_FS_SNAP) {
        launch_snap(sd->J, bd, x, *sd, w, f, nullptr, 0, st, &ctx->prof, nullptr, p_kick, dt, fp, open);
    } else {
        launch_fs(bd, x, *fp, w, f, nullptr, 0, st, true, p_kick, dt);
    }
}

// Steps s_lo .. s_hi - 1 of a call of the batch in place, with the workspace w and the
// force buffer f (which holds the force at x unless `initial` asks to evaluate it first).
// Step s draws the Gaussians of global step step0 + s; with the BBK scheme s = 0 is the
// call's first iterate and s + 1 == n_last its last.
void run_langevin_range(snapmd_ctx *ctx, Work &w, double *f, int potential, const BatchDev &bd, const FsParams &fp,
                        const SnapDev &sd, const LangevinDev &ld, int s_lo, int s_hi, int n_last, bool initial,
                        double *x, double *p, hipStream_t st) {
    if (initial) enqueue_forces(ctx, w, potential, bd, x, &fp, &sd, f, st);
    // BAOAB with SNAP: the gather of step s also opens step s + 1 within the range (one
    // launch less per step); the range's first step is opened by k_baoab_pre
    const bool fuse_open = potential == SNAPMD_POT_FS_SNAP;
    StepOpen open;
    open.x = x;
    open.ld = ld;
    open.off = bd.off;
    open.n_sys = bd.n_sys;
    open.xref = w.xref;
    open.lim2 = 0.25 * kSkin * kSkin;
    open.flag = w.flag;
    for (int s = s_lo; s < s_hi; ++s) {
        if (ld.scheme == SNAPMD_SCHEME_BBK) {
            launch_bbk_pre(bd, x, p, f, ld, s, w, kSkin, st);
            enqueue_forces(ctx, w, potential, bd, x, &fp, &sd, f, st, false);
            launch_bbk_post(bd, p, f, ld, s + 1, n_last, st);
        } else {
            if (!fuse_open || s == s_lo) launch_baoab_pre(bd, x, p, f, ld, s, w, kSkin, st);
            open.open_step = (fuse_open && s + 1 < s_hi) ? s + 1 : -1;
            enqueue_forces(ctx, w, potential, bd, x, &fp, &sd, f, st, false, p, ld.dt, &open);
        }
    }
}

// n_steps steps of the batch in place (force evaluated at the start).
void run_langevin(snapmd_ctx *ctx, Work &w, double *f, int potential, const BatchDev &bd, const FsParams &fp,
                  const SnapDev &sd, const LangevinDev &ld, int n_steps, double *x, double *p, hipStream_t st) {
    run_langevin_range(ctx, w, f, potential, bd, fp, sd, ld, 0, n_steps, n_steps, true, x, p, st);
}

// Cell grids (and their buffers) of the neighbour lists a propagation of the batch uses;
// set up outside any capture.  Once set up for a batch and cutoff this does nothing.
int prepare_propagation_cells(snapmd_ctx *ctx, Work &w, int potential, const BatchDev &bd, const FsParams &fp,
                              const SnapDev &sd, hipStream_t st) {
    BatchDev bc = bd;
    const double rl = (potential == SNAPMD_POT_FS_SNAP ? std::max(sd.gp.rcut, std::max(fp.d, fp.c))
                                                       : std::max(fp.d, fp.c)) + kSkin;
    return prepare_cells(ctx, w, bc, rl, st);
}

// captured launch sequences kept per workspace (a chunk tuner cycles through about 30
// plans of up to 5 chunks; fewer slots made it re-capture inside timed runs)
constexpr size_t kGraphCache = 256;
// Longest call captured into one graph.  A longer call is replayed in segments of
// kGraphSegSteps steps, so no captured chain exceeds about 16 kGraphSegSteps kernel nodes.
constexpr int kGraphMaxSteps = 1000;
constexpr int kGraphSegSteps = 250;
constexpr int kNoLast = 1 << 30;  // n_last of a segment that holds no call's last step

// Replay (capturing on first use) the launch sequence of run_langevin_range for these
// arguments.  The key holds everything baked into the kernel arguments and launch
// shapes: pointers, sizes (including the largest system, which sizes the LDS of the
// neighbour build), parameters and the step range.
int replay_range(snapmd_ctx *ctx, Work &w, double *f, int potential, const BatchDev &bd, const FsParams &fp,
                 const SnapDev &sd, const LangevinDev &ld, int s_lo, int s_hi, int n_last, bool initial, double *x,
                 double *p, hipStream_t st) {
    auto u = [](const void *q) { return (uint64_t)(uintptr_t)q; };
    auto d = [](double v) {
        uint64_t b;
        std::memcpy(&b, &v, sizeof b);
        return b;
    };
    std::vector<uint64_t> key{(uint64_t)potential, (uint64_t)bd.N, (uint64_t)bd.n_sys, (uint64_t)bd.max_sys, u(bd.off),
                              u(bd.box), u(bd.cells), (uint64_t)bd.n_cells, (uint64_t)s_lo, (uint64_t)s_hi,
                              (uint64_t)n_last, (uint64_t)initial, u(x), u(p), u(f),
                              u(w.nbr), u(w.geo), u(w.u), u(w.ytil), u(w.xref), u(w.cell_cnt), u(w.flag), d(fp.A), d(fp.d), d(fp.c), d(fp.c0), d(fp.c1), d(fp.c2),
                              d(ld.dt), d(ld.c1), d(ld.mass), ld.seed, u(ld.sig), u(ld.step0), u(ld.noise_id),
                              (uint64_t)ld.scheme, d(ld.gamma), u(ld.sb0), u(ld.sb1), u(w.ph)};
    if (potential == SNAPMD_POT_FS_SNAP) {
        const uint64_t sk[] = {(uint64_t)sd.J, d(sd.gp.rcut), d(sd.gp.rfac0), d(sd.gp.rmin0), d(sd.beta0),
                               u(sd.nrm), u(sd.adj.coef), u(sd.adj.cgm), u(sd.adj.roles), u(sd.adj.roles8),
                               (uint64_t)sd.shape.dens_acc, (uint64_t)sd.shape.dedr_atoms,
                               (uint64_t)sd.shape.adj_waves, (uint64_t)sd.shape.dens_parts};
        key.insert(key.end(), std::begin(sk), std::end(sk));
    }
    const int ci = ws_index(ctx, w);
    auto &cache = ctx->graphs[ci];
    const uint64_t now = ++ctx->graph_clock[ci];
    for (auto &g : cache)
        if (g.key == key) {
            g.last_use = now;
            HIPCHK(hipGraphLaunch(g.exec, st));
            return SNAPMD_OK;
        }
    // captured on a stream of the context (the caller's may be the null stream), then
    // launched on the caller's stream
    hipStream_t &cs = ctx->cap_stream[ci];
    if (!cs) HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    ++KernelProf::suppress;  // no event records inside a graph
    run_langevin_range(ctx, w, f, potential, bd, fp, sd, ld, s_lo, s_hi, n_last, initial, x, p, cs);
    --KernelProf::suppress;
    HIPCHK(hipStreamEndCapture(cs, &graph));
    hipGraphExec_t exec;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(ctx, SNAPMD_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    if (cache.size() >= kGraphCache) {
        auto it = std::min_element(cache.begin(), cache.end(),
                                   [](const auto &a, const auto &b) { return a.last_use < b.last_use; });
        // the evicted graph may still be queued on some stream: let it finish first
        HIPCHK(hipDeviceSynchronize());
        (void)hipGraphExecDestroy(it->exec);
        cache.erase(it);
    }
    cache.push_back({key, exec, now});
    HIPCHK(hipGraphLaunch(exec, st));
    return SNAPMD_OK;
}

// run_langevin through cached hipGraphs.  A call of up to kGraphMaxSteps steps is one
// captured launch sequence.  A longer one runs as a head segment (the initial force
// evaluation and steps 0 .. kGraphSegSteps - 1), then segments that are all captured
// with the step range [kGraphSegSteps, 2 kGraphSegSteps) and replayed with the step
// offsets of the systems advanced on the device between replays (a copy of the offsets
// owned by the workspace), then a tail segment of the remaining steps, which holds the
// call's last step.  Segment s of the call therefore draws exactly the Gaussians that
// the one-chain launch sequence would, and BBK's first and last iterates stay where
// they are.  The segments bound the length of every captured chain: a capture of
// 10,000 steps, one linear chain of about 160,000 kernel nodes, ended the process with
// a host segmentation fault (see the design notes on graph captures).
// The same with the batch's cell grids already in bd (set up by the caller).
int run_langevin_prepared(snapmd_ctx *ctx, Work &w, double *f, int potential, const BatchDev &bd, const FsParams &fp,
                          const SnapDev &sd, const LangevinDev &ld, int n_steps, double *x, double *p,
                          hipStream_t st) {
    // SNAP propagation stays eager while kernel timing is on (the events time each launch)
    if (!ctx->use_graphs || (ctx->prof.enabled && potential == SNAPMD_POT_FS_SNAP)) {
        run_langevin(ctx, w, f, potential, bd, fp, sd, ld, n_steps, x, p, st);
        return SNAPMD_OK;
    }
    int rc;
    if (n_steps <= kGraphMaxSteps)
        return replay_range(ctx, w, f, potential, bd, fp, sd, ld, 0, n_steps, n_steps, true, x, p, st);
    const int ci = ws_index(ctx, w);
    DBuf<int64_t> &so = ctx->seg_step0[ci];
    if (so.n < (size_t)bd.n_sys || !so.p)
        return fail(ctx, SNAPMD_EINVAL, "segment step offsets not prepared for %d systems", bd.n_sys);
    constexpr int G = kGraphSegSteps;
    HIPCHK(hipMemcpyAsync(so.p, ld.step0, (size_t)bd.n_sys * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    LangevinDev lg = ld;
    lg.step0 = so.p;
    if ((rc = replay_range(ctx, w, f, potential, bd, fp, sd, lg, 0, G, kNoLast, true, x, p, st))) return rc;
    // the copy's offsets lead the caller's by `adv`; a segment covering call steps
    // [g0, g0 + len) is captured as [G, G + len) and needs adv = g0 - G
    int64_t adv = 0;
    for (int g0 = G; g0 < n_steps; g0 += G) {
        const int len = std::min(G, n_steps - g0);
        const bool last = g0 + len == n_steps;
        if (g0 - G != adv) {
            launch_add_i64(bd.n_sys, so.p, (int64_t)(g0 - G) - adv, st);
            adv = g0 - G;
        }
        if ((rc = replay_range(ctx, w, f, potential, bd, fp, sd, lg, G, G + len, last ? G + len : kNoLast, false, x,
                               p, st)))
            return rc;
    }
    return check_launch(ctx);
}

int run_langevin_graph(snapmd_ctx *ctx, Work &w, double *f, int potential, const BatchDev &bd, const FsParams &fp,
                       const SnapDev &sd, const LangevinDev &ld, int n_steps, double *x, double *p,
                       hipStream_t st) {
    if (ctx->use_graphs && !(ctx->prof.enabled && potential == SNAPMD_POT_FS_SNAP)) {
        int rc;
        if ((rc = prepare_propagation_cells(ctx, w, potential, bd, fp, sd, st))) return rc;
    }
    return run_langevin_prepared(ctx, w, f, potential, bd, fp, sd, ld, n_steps, x, p, st);
}

// Per-system Langevin arrays (sigma, step offsets, noise ids) uploaded to the context.
int prepare_langevin(snapmd_ctx *ctx, const snapmd_langevin *lang, int S, const std::vector<double> &T,
                     const std::vector<int64_t> &step0, const std::vector<int> &nid, LangevinDev &ld,
                     hipStream_t st) {
    const double c1 = std::exp(-lang->gamma * lang->dt);
    std::vector<double> sig(S), sb0(S), sb1(S);
    for (int s = 0; s < S; ++s) {
        sig[s] = std::sqrt((1.0 - c1 * c1) * lang->mass * kKB * T[s] / kMVV2E);
        // BBK: (1/2) sqrt(2 gamma m kB T_l dt / mvv2e) with T_0 = C_0 T, T_l = C_l T
        const double base = 2.0 * lang->gamma * lang->mass * kKB * T[s] * lang->dt / kMVV2E;
        sb0[s] = 0.5 * std::sqrt(base * (lang->scheme == SNAPMD_SCHEME_BBK ? lang->bbk_c0 : 1.0));
        sb1[s] = 0.5 * std::sqrt(base * (lang->scheme == SNAPMD_SCHEME_BBK ? lang->bbk_c1 : 1.0));
    }
    int rc;
    if ((rc = ensure(ctx, ctx->d_sig, S)) || (rc = ensure(ctx, ctx->d_step0, S)) || (rc = ensure(ctx, ctx->d_noise, S)) ||
        (rc = ensure(ctx, ctx->d_sb0, S)) || (rc = ensure(ctx, ctx->d_sb1, S)) ||
        (rc = ensure(ctx, ctx->seg_step0[0], S)) || (rc = ensure(ctx, ctx->seg_step0[1], S)) ||
        (rc = ensure(ctx, ctx->seg_step0[2], S)))
        return rc;
    // uploaded only when they change (a pipelined parareal iteration must not rewrite
    // arrays the previous one still reads on another stream)
    std::vector<uint64_t> key{(uint64_t)S, (uint64_t)(uintptr_t)ctx->d_sig.p, (uint64_t)(uintptr_t)ctx->d_step0.p,
                              (uint64_t)(uintptr_t)ctx->d_noise.p, (uint64_t)(uintptr_t)ctx->d_sb0.p,
                              (uint64_t)(uintptr_t)ctx->d_sb1.p};
    auto bits = [](double v) {
        uint64_t b;
        std::memcpy(&b, &v, sizeof b);
        return b;
    };
    for (int s = 0; s < S; ++s) {
        key.push_back(bits(sig[s]));
        key.push_back((uint64_t)step0[s]);
        key.push_back((uint64_t)nid[s]);
        key.push_back(bits(sb0[s]));
        key.push_back(bits(sb1[s]));
    }
    if (key != ctx->lang_key) {
        if ((rc = upload(ctx, ctx->d_sig.p, sig.data(), S, st))) return rc;
        if ((rc = upload(ctx, ctx->d_step0.p, step0.data(), S, st))) return rc;
        if ((rc = upload(ctx, ctx->d_noise.p, nid.data(), S, st))) return rc;
        if ((rc = upload(ctx, ctx->d_sb0.p, sb0.data(), S, st))) return rc;
        if ((rc = upload(ctx, ctx->d_sb1.p, sb1.data(), S, st))) return rc;
        ctx->lang_key = key;
    }
    ld = LangevinDev{lang->dt, c1, lang->mass, lang->seed, ctx->d_sig.p, ctx->d_step0.p, ctx->d_noise.p};
    ld.scheme = lang->scheme;
    ld.gamma = lang->gamma;
    ld.sb0 = ctx->d_sb0.p;
    ld.sb1 = ctx->d_sb1.p;
    return SNAPMD_OK;
}

// Gaussians of every (slab, step, atom) of the window for the LDS-resident sweep, kept
// while the window (and the noise stream) stays the same.
int launch_noise_sweep(snapmd_ctx *ctx, int n_in, int S, int L, int N, const snapmd_langevin *lang, hipStream_t st) {
    // exact integers: two 64-bit seeds can round to the same double
    const std::vector<uint64_t> key{(uint64_t)n_in, (uint64_t)S, (uint64_t)L, (uint64_t)N, lang->seed,
                                    (uint64_t)lang->noise_id_sys[0]};
    if (key == ctx->noise_key) return SNAPMD_OK;
    int rc;
    if ((rc = ensure(ctx, ctx->sw_noise, (size_t)S * L * 3 * N))) return rc;
    launch_noise_table(S, L, N, n_in, lang->seed, (uint64_t)lang->noise_id_sys[0], ctx->sw_noise.p, st);
    ctx->noise_key = key;
    return SNAPMD_OK;
}

int check_lang(snapmd_ctx *ctx, const snapmd_langevin *lang) {
    if (!lang) return fail(ctx, SNAPMD_EINVAL, "lang is NULL");
    if (lang->scheme != SNAPMD_SCHEME_BAOAB && lang->scheme != SNAPMD_SCHEME_BBK)
        return fail(ctx, SNAPMD_EINVAL, "scheme must be SNAPMD_SCHEME_BAOAB or SNAPMD_SCHEME_BBK (got %d)", lang->scheme);
    if (lang->scheme == SNAPMD_SCHEME_BBK &&
        !(lang->bbk_c0 > 0.0 && lang->bbk_c1 > 0.0 && std::isfinite(lang->bbk_c0) && std::isfinite(lang->bbk_c1)))
        return fail(ctx, SNAPMD_EINVAL, "the BBK temperature factors bbk_c0, bbk_c1 must be finite and > 0");
    if (!(lang->dt > 0.0) || !(lang->gamma >= 0.0) || !(lang->mass > 0.0))
        return fail(ctx, SNAPMD_EINVAL, "need dt > 0, gamma >= 0, mass > 0");
    if (!lang->T_sys || !lang->step0_sys || !lang->noise_id_sys)
        return fail(ctx, SNAPMD_EINVAL, "lang.T_sys, step0_sys and noise_id_sys must be set");
    return SNAPMD_OK;
}

}  // namespace

namespace {

// The sequential sweep of one system driven from the host with the batched kernels, one
// small synchronisation per slab for the relative error and the early stop (systems the
// on-device sweeps do not take, the BBK scheme, a coarse potential with SNAP).  q_cur,
// p_cur, q_prev point at the system's first atom in slot 0 of the slot layout [slot][3][ld];
// the jump of slab n_in + s, row al, atom i is at jq[al jsa + s jss + i].
int host_sweep(snapmd_ctx *ctx, int potC, const FsParams &fp, const SnapDev &sdc, const snapmd_langevin *lang,
               double T, int noise_id, int N, const double *box, int L, int n_in, int32_t *n_fi, bool init, size_t ld,
               double *q_cur, double *p_cur, const double *q_prev, const double *jq, const double *jp, size_t jsa,
               size_t jss, double delta_expl, double *delta_out, hipStream_t st, void *stream) {
    int rc;
    if ((rc = ensure(ctx, ctx->sw_x, 3 * (size_t)N)) || (rc = ensure(ctx, ctx->sw_p, 3 * (size_t)N)) ||
        (rc = ensure(ctx, ctx->sw_out, 8)))
        return rc;
    if (!ctx->h_out) HIPCHK(hipHostMalloc((void **)&ctx->h_out, 16 * sizeof(double), hipHostMallocDefault));
    double *wx = ctx->sw_x.p, *wp = ctx->sw_p.p;
    const size_t so = (size_t)n_in * 3 * ld;  // slot n_in
    HIPCHK(hipMemcpy2DAsync(wx, (size_t)N * sizeof(double), q_cur + so, ld * sizeof(double), (size_t)N * sizeof(double),
                            3, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpy2DAsync(wp, (size_t)N * sizeof(double), p_cur + so, ld * sizeof(double), (size_t)N * sizeof(double),
                            3, hipMemcpyDeviceToDevice, st));
    int off1[2] = {0, N};
    snapmd_batch b1{1, off1, box};
    BatchDev bd1;
    double mh1;
    if ((rc = prepare_batch(ctx, &b1, bd1, mh1, st))) return rc;
    double num = 0.0, den = 0.0, delta = 0.0;
    int nfi_new = *n_fi;
    for (int n = n_in; n < *n_fi; ++n) {
        std::vector<double> T1(1, T);
        std::vector<int64_t> s1(1, (int64_t)n * L);
        std::vector<int> id1(1, noise_id);
        LangevinDev ld1;
        if ((rc = prepare_langevin(ctx, lang, 1, T1, s1, id1, ld1, st))) return rc;
        // one captured launch sequence serves every slab: the step offset of the slab
        // is read from device memory (uploaded above) when the sequence runs
        if ((rc = run_langevin_graph(ctx, ctx->w, ctx->d_f, potC, bd1, fp, sdc, ld1, L, wx, wp, st))) return rc;
        const size_t nx = (size_t)(n + 1) * 3 * ld;  // slot n + 1
        launch_slab_end(N, init ? 0 : 1, jsa, jss, (size_t)(n - n_in), wx, wp, jq, jp, ld,
                        init ? nullptr : q_prev + nx, q_cur + nx, p_cur + nx, ctx->sw_out.p, st);
        if ((rc = check_launch(ctx))) return rc;
        HIPCHK(hipMemcpyAsync(ctx->h_out, ctx->sw_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        if ((rc = snapmd_sync(ctx, stream))) return rc;
        if (!std::isfinite(ctx->h_out[2])) return fail(ctx, SNAPMD_ENONFINITE, "state became non-finite in slab %d", n);
        if (!init) {
            num += std::sqrt(ctx->h_out[0]);
            den += std::sqrt(ctx->h_out[1]);
            delta = den > 0.0 ? num / den : 0.0;
            if (delta > delta_expl) {
                nfi_new = std::max(n, n_in + 1);
                break;
            }
        }
    }
    *delta_out = delta;
    *n_fi = nfi_new;
    return SNAPMD_OK;
}

// One system (its states [slot][3][N]): the pipelined path of the bench workload.
// async: a pipelined iteration (parareal_iterate_async): the call returns once the work is
// enqueued and the result is queued for snapmd_parareal_collect.
int parareal_one(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                 const snapmd_langevin *lang, int32_t L, int32_t n_in, int32_t *n_fi, double *q_prev, double *p_prev,
                 double *q_cur, double *p_cur, double delta_expl, double *delta_out, hipStream_t st, void *stream,
                 bool async = false) {
    int rc;
    const bool init = (q_prev == nullptr);
    const int N = batch->offset[1];
    const int S = *n_fi - n_in;
    const double *box = batch->box;
    double mh = 0.5 * std::min(box[0], std::min(box[1], box[2]));
    FsParams fp, fpc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if ((rc = coarse_fs(ctx, fp, mh, fpc))) return rc;
    const double skin = kSweepSkin;
    if (!(std::max(fpc.d, fpc.c) + 2.0 * skin < mh))
        return fail(ctx, SNAPMD_EINVAL, "FS cutoff + %g A must be < half the smallest box edge", 2.0 * skin);
    SnapDev sd;
    const size_t SN3 = 3 * (size_t)S * N;
    // sweep scratch
    if ((rc = ensure(ctx, ctx->sw_out, 8))) return rc;
    // the on-device sweeps integrate BAOAB; the BBK scheme takes the host-driven sweep
    const bool bbk = lang->scheme == SNAPMD_SCHEME_BBK;
    // coarse potential: Finnis-Sinclair, plus SNAP when snapmd_set_coarse_snap set one (the
    // paper's strategy I); the on-device sweeps integrate Finnis-Sinclair only
    const bool csnap = ctx->coarse_snap_on;
    const int potC = csnap ? SNAPMD_POT_FS_SNAP : SNAPMD_POT_FS;
    SnapDev sdc;
    if (csnap) {
        snapmd_snap cs = ctx->coarse_snap;
        cs.beta = ctx->coarse_beta.data();
        if (snap && !init && snap->twojmax == cs.twojmax)
            return fail(ctx, SNAPMD_EINVAL, "the coarse SNAP needs a twojmax other than the fine one (%d)",
                        cs.twojmax);
        if ((rc = prepare_snap(ctx, &cs, mh, sdc, st))) return rc;
    }
    if ((bbk || csnap || !sweep_fits_lds(N)) &&
        ((rc = ensure(ctx, ctx->sw_x, 3 * (size_t)N)) || (rc = ensure(ctx, ctx->sw_p, 3 * (size_t)N))))
        return rc;
    if (!ctx->h_out) HIPCHK(hipHostMalloc((void **)&ctx->h_out, 16 * sizeof(double), hipHostMallocDefault));
    const double c1 = std::exp(-lang->gamma * lang->dt);
    SweepLaunch sw{};
    sw.N = N;
    sw.box[0] = box[0];
    sw.box[1] = box[1];
    sw.box[2] = box[2];
    sw.fp = fpc;
    sw.skin = skin;
    sw.dt = lang->dt;
    sw.c1 = c1;
    sw.mass = lang->mass;
    sw.sig = std::sqrt((1.0 - c1 * c1) * lang->mass * kKB * lang->T_sys[0] / kMVV2E);
    sw.seed = lang->seed;
    sw.noise_id = (uint64_t)lang->noise_id_sys[0];
    sw.L = L;
    sw.n_in = n_in;
    sw.n_fi = *n_fi;
    sw.mode = init ? 0 : 1;
    sw.n_win = n_in;
    {
        // cell grid of the sweep's list build: edges >= list radius, >= 3 cells per edge,
        // at most 512 cells (else every pair is examined)
        int nc[3];
        for (int a = 0; a < 3; ++a) nc[a] = (int)std::floor(box[a] / (std::max(fpc.d, fpc.c) + skin));
        while ((long)nc[0] * nc[1] * nc[2] > 512) *std::max_element(nc, nc + 3) -= 1;
        if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) nc[0] = nc[1] = nc[2] = 0;
        sw.ncx = nc[0];
        sw.ncy = nc[1];
        sw.ncz = nc[2];
    }
    sw.delta_expl = delta_expl;
    sw.q_cur = q_cur;
    sw.p_cur = p_cur;
    sw.q_prev = q_prev;
    sw.p_prev = p_prev;
    // the sweep on the device: several workgroups exchanging through device memory, or
    // one LDS-resident workgroup; else driven from the host
    // width 1 asks for the one-workgroup sweep where it fits
    const bool one_wg = ctx->sweep_k_override == 1 && sweep_fits_lds(N);
    const int mcK = (bbk || csnap || one_wg) ? 0 : sweep_mc_workgroups(N, ctx->sweep_k_override);
    const bool lds_sweep = !bbk && !csnap && (mcK > 0 || sweep_fits_lds(N));
    // A pipelined iteration (on-device sweep, corrected iteration) overlaps the previous
    // pipelined iteration when everything the two share is the same (chain_key: window,
    // chunk plan, state buffers, box, potentials, Langevin parameters, sweep width,
    // stream), so
    // neither allocates nor rewrites what the other reads; every other call first waits
    // for all pipelined iterations in flight.
    const bool pipelined = async && !init && lds_sweep;
    const std::vector<int> plan = init ? std::vector<int>{} : lds_sweep ? window_plan(ctx, S, N) : std::vector<int>{S};
    std::vector<uint64_t> key;
    bool chained = false;
    if (pipelined) {
        auto u = [](const void *q) { return (uint64_t)(uintptr_t)q; };
        auto d = [](double v) {
            uint64_t b;
            std::memcpy(&b, &v, sizeof b);
            return b;
        };
        key = {(uint64_t)n_in, (uint64_t)S, (uint64_t)L, (uint64_t)N, u(q_prev), u(p_prev), u(q_cur), u(p_cur),
               d(box[0]), d(box[1]), d(box[2]), d(fp.A), d(fp.d), d(fp.c), d(fp.c0), d(fp.c1), d(fp.c2),
               d(fpc.A), d(fpc.d), d(fpc.c), d(fpc.c0), d(fpc.c1), d(fpc.c2), (uint64_t)mcK, d(lang->dt),
               d(lang->gamma), d(lang->mass), d(lang->T_sys[0]), lang->seed, (uint64_t)lang->noise_id_sys[0],
               (uint64_t)lang->scheme, snap ? (uint64_t)snap->twojmax : 0, snap ? d(snap->rcut) : 0,
               u(st)};  // a chain on another stream would share the workspace unordered
        for (int v : plan) key.push_back((uint64_t)v);
        chained = ctx->chain_end && key == ctx->chain_key;
    }
    if (!chained && (rc = drain(ctx))) return rc;
    ctx->chain_key.clear();  // set again once a pipelined iteration is fully enqueued
    int aslot = -1;
    double *h0 = ctx->h_out + 8;  // the sweep state's initial values (pinned host)
    sw.out = ctx->sw_out.p;
    if (pipelined) {
        if ((int)ctx->async_q.size() >= snapmd_ctx::kAsyncSlots - 1)
            return fail(ctx, SNAPMD_EINVAL, "at most %d pipelined iterations may wait to be collected",
                        snapmd_ctx::kAsyncSlots - 1);
        if ((rc = ensure(ctx, ctx->sw_out_ring, 8 * (size_t)snapmd_ctx::kAsyncSlots))) return rc;
        if (!ctx->h_async)
            HIPCHK(hipHostMalloc((void **)&ctx->h_async,
                                 snapmd_ctx::kAsyncStride * snapmd_ctx::kAsyncSlots * sizeof(double),
                                 hipHostMallocDefault));
        for (hipEvent_t &e : ctx->async_ev)
            if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // slot of this iteration: at most kAsyncSlots - 1 are uncollected, and the one
        // kAsyncSlots iterations back was collected (its device work done)
        aslot = (int)(ctx->async_seq % snapmd_ctx::kAsyncSlots);
        sw.out = ctx->sw_out_ring.p + 8 * aslot;
        h0 = ctx->h_async + snapmd_ctx::kAsyncStride * aslot + 8;
    }
    {
        // sweep state carried over the launches of this call (a pipelined iteration resets
        // its slot on the sweep stream, behind the sweeps in flight)
        const double init_out[8] = {0.0, (double)*n_fi, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        std::memcpy(h0, init_out, sizeof init_out);
        if (!pipelined) HIPCHK(hipMemcpyAsync(ctx->sw_out.p, h0, 8 * sizeof(double), hipMemcpyHostToDevice, st));
    }
    if (mcK > 0) {
        sw.K = mcK;
        sw.A = (N + mcK - 1) / mcK;
        if ((rc = ensure(ctx, ctx->sw_gx, 12 * (size_t)N)) || (rc = ensure(ctx, ctx->sw_gdfe, 4 * (size_t)N)) ||
            (rc = ensure(ctx, ctx->sw_gpart, 16 * (size_t)mcK)) || (rc = ensure(ctx, ctx->sw_abort, 1)))
            return rc;
        sw.gx = ctx->sw_gx.p;
        sw.gdfe = ctx->sw_gdfe.p;
        sw.gpart = ctx->sw_gpart.p;
        sw.abort = ctx->sw_abort.p;
    }
    // the exchange words of the multi-workgroup sweep carry no live tag at launch
    auto sweep_launch = [&](const SweepLaunch &l, hipStream_t s) -> int {
        if (l.K > 0) {
            HIPCHK(hipMemsetAsync(l.gx, 0, 12 * (size_t)l.N * sizeof(unsigned long long), s));
            HIPCHK(hipMemsetAsync(l.gdfe, 0, 4 * (size_t)l.N * sizeof(unsigned long long), s));
            HIPCHK(hipMemsetAsync(l.gpart, 0, 16 * (size_t)l.K * sizeof(unsigned long long), s));
            HIPCHK(hipMemsetAsync(l.abort, 0, sizeof(int), s));
        }
        launch_coarse_sweep(l, s);
        return check_launch(ctx);
    };
    if (!init) {
        // prev_n := cur_n on [n_in, n_fi] (a pipelined iteration copies chunk by chunk below)
        const size_t slot = 3 * (size_t)N;
        if (!pipelined) {
            HIPCHK(hipMemcpyAsync(q_prev + n_in * slot, q_cur + n_in * slot, (S + 1) * slot * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(p_prev + n_in * slot, p_cur + n_in * slot, (S + 1) * slot * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
        }
        // the batch: S copies of the system, slab s starting at global step (n_in + s) L
        std::vector<int> off(S + 1);
        std::vector<double> boxes(3 * S);
        for (int s = 0; s <= S; ++s) off[s] = s * N;
        for (int s = 0; s < S; ++s)
            for (int a = 0; a < 3; ++a) boxes[3 * s + a] = box[a];
        snapmd_batch sb{S, off.data(), boxes.data()};
        BatchDev bd;
        double mh2;
        if ((rc = prepare_batch(ctx, &sb, bd, mh2, st))) return rc;
        if ((rc = prepare_snap(ctx, snap, mh2, sd, st))) return rc;
        std::vector<double> T(S, lang->T_sys[0]);
        std::vector<int64_t> step0(S);
        std::vector<int> nid(S, lang->noise_id_sys[0]);
        for (int s = 0; s < S; ++s) step0[s] = (int64_t)(n_in + s) * L;
        LangevinDev ld;
        if ((rc = prepare_langevin(ctx, lang, S, T, step0, nid, ld, st))) return rc;
        if ((rc = ensure(ctx, ctx->pr_xf, SN3)) || (rc = ensure(ctx, ctx->pr_pf, SN3)) ||
            (rc = ensure(ctx, ctx->pr_xc, SN3)) || (rc = ensure(ctx, ctx->pr_pc, SN3)))
            return rc;
        if ((rc = ensure_atoms_coarse(ctx, (size_t)S * N, csnap))) return rc;
        // The slabs are propagated in chunks of consecutive slabs (chunk c occupies
        // [3][S_c N] at offset 3 N s0 of the batch buffers).  The SNAP propagation of the
        // chunks runs on the caller's stream; the Finnis-Sinclair propagation, the jumps
        // and (LDS-resident case) the sweep run on a second stream, the sweep over chunk c
        // as soon as the SNAP propagation of chunk c is done, overlapping the later chunks.
        if (!ctx->sweep_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->sweep_stream, hipStreamNonBlocking));
        if (!ctx->coarse_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->coarse_stream, hipStreamNonBlocking));
        // events: fine chunk c done [0, ne), sweep done (ne), start (ne + 1), coarse chunk c
        // done [ne + 2, 2 ne + 2), prev := cur of chunk c done (pipelined) [2 ne + 2, 3 ne + 2),
        // list status read (pipelined) 3 ne + 2; sweep of chunk c enqueued up to its end:
        // sweep_chunk_ev[c]
        const int ne = (int)plan.size();
        for (int c = (int)ctx->pipe_ev.size(); c < 3 * ne + 3; ++c) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            ctx->pipe_ev.push_back(e);
        }
        for (int c = (int)ctx->sweep_chunk_ev.size(); c < ne; ++c) {
            hipEvent_t e;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            ctx->sweep_chunk_ev.push_back(e);
        }
        hipStream_t s2 = ctx->sweep_stream;
        if (lds_sweep) {
            if ((rc = launch_noise_sweep(ctx, n_in, S, L, N, lang, st))) return rc;
            sw.noise = ctx->sw_noise.p;
        }
        const double *qs = q_prev + n_in * slot, *ps = p_prev + n_in * slot;
        auto chunk_of = [&](int c, int s0, BatchDev &bc, LangevinDev &lc) {
            const int nc = plan[c];
            bc = bd;
            bc.N = nc * N;
            bc.n_sys = nc;
            lc = ld;
            lc.sig += s0;
            lc.step0 += s0;
            lc.noise_id += s0;
            lc.sb0 += s0;
            lc.sb1 += s0;
            return nc;
        };
        hipStream_t s3 = ctx->coarse_stream;
        HIPCHK(hipEventRecord(ctx->pipe_ev[ne + 1], st));
        HIPCHK(hipStreamWaitEvent(s2, ctx->pipe_ev[ne + 1], 0));
        HIPCHK(hipStreamWaitEvent(s3, ctx->pipe_ev[ne + 1], 0));
        if (pipelined) HIPCHK(hipMemcpyAsync(sw.out, h0, 8 * sizeof(double), hipMemcpyHostToDevice, s2));
        // Three streams, each fed by its own host thread: the fine propagation of the
        // chunks (caller's stream, this thread), their coarse propagation (s3) and the
        // jumps and sweep of chunk c once both propagations of chunk c are done (s2).  A
        // replay of a long captured launch sequence can hold the calling thread until the
        // device has worked through most of it, so no stream's queueing may wait behind
        // another's.  Everything the replays need (buffers, cell grids) is set up here
        // first: neither helper allocates (an allocation drops the captured graphs).
        if ((rc = prepare_propagation_cells(ctx, ctx->w, SNAPMD_POT_FS_SNAP, bd, fp, sd, st)) ||
            (rc = prepare_propagation_cells(ctx, ctx->wc, potC, bd, fpc, sdc, st)))
            return rc;
        // Two SNAP streams (ctx->fine_streams 2, several chunks): the odd chunks run on a
        // stream of their own with the second workspace, beside the even ones, so that one
        // chunk's small kernels and partial adjoint round fill the CUs the other leaves
        // idle.  Not while kernel timing is on (the timed launches are the caller's).
        const bool two = ctx->fine_streams == 2 && ne > 1 && !ctx->prof.enabled;
        if (two) {
            const int maxc = *std::max_element(plan.begin(), plan.end());
            if ((rc = ensure_atoms_ws(ctx, ctx->w2, ctx->d_f2, ctx->cap_atoms2, (size_t)maxc * N))) return rc;
            ctx->w2.status = ctx->w.status;
            if (!ctx->w2.flag) {
                if ((rc = dalloc(ctx, &ctx->w2.flag, 1))) return rc;
                HIPCHK(hipMemset(ctx->w2.flag, 0, sizeof(int)));
            }
            if (!ctx->fine2_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->fine2_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamWaitEvent(ctx->fine2_stream, ctx->pipe_ev[ne + 1], 0));
            if ((rc = prepare_propagation_cells(ctx, ctx->w2, SNAPMD_POT_FS_SNAP, bd, fp, sd, ctx->fine2_stream)))
                return rc;
        }
        auto side_of = [&](int c) { return two && (c & 1) ? 1 : 0; };
        std::mutex mu;
        std::condition_variable cv;
        int done_c = 0;                                // chunks whose coarse propagation is queued
        std::vector<char> done_f(ne, 0), copied(ne, 0);  // chunk c's fine propagation / prev := cur copy queued
        bool stop = false;                             // a thread failed: the others queue nothing more
        auto publish = [&](int &counter, int value) {
            std::lock_guard<std::mutex> lk(mu);
            counter = value;
            cv.notify_all();
        };
        auto mark = [&](std::vector<char> &flags, int c) {
            std::lock_guard<std::mutex> lk(mu);
            flags[c] = 1;
            cv.notify_all();
        };
        auto halt = [&]() {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
            cv.notify_all();
        };
        struct Quiet {  // kernel timing covers the caller's stream only
            Quiet() { ++KernelProf::suppress; }
            ~Quiet() { --KernelProf::suppress; }
        };
        auto coarse_side = [&]() -> int {
            HIPCHK(hipSetDevice(ctx->device));
            Quiet quiet;
            int r;
            for (int c = 0, s0 = 0; c < (int)plan.size(); s0 += plan[c], ++c) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    if (stop) return SNAPMD_OK;
                }
                if (pipelined) {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || copied[c]; });
                    if (stop) return SNAPMD_OK;
                }
                BatchDev bc;
                LangevinDev lc;
                const int nc = chunk_of(c, s0, bc, lc);
                const size_t o = 3 * (size_t)N * s0;
                if (pipelined) HIPCHK(hipStreamWaitEvent(s3, ctx->pipe_ev[2 * ne + 2 + c], 0));
                launch_slabs_to_batch(nc, N, qs + s0 * slot, ctx->pr_xc.p + o, s3);
                launch_slabs_to_batch(nc, N, ps + s0 * slot, ctx->pr_pc.p + o, s3);
                if ((r = run_langevin_graph(ctx, ctx->wc, ctx->d_fc, potC, bc, fpc, sdc, lc, L,
                                            ctx->pr_xc.p + o, ctx->pr_pc.p + o, s3)))
                    return r;
                HIPCHK(hipEventRecord(ctx->pipe_ev[ne + 2 + c], s3));
                publish(done_c, c + 1);
            }
            return SNAPMD_OK;
        };
        auto sweep_side = [&]() -> int {
            HIPCHK(hipSetDevice(ctx->device));
            Quiet quiet;
            int r;
            for (int c = 0, s0 = 0; c < (int)plan.size(); s0 += plan[c], ++c) {
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || (done_f[c] && done_c > c); });
                    if (stop) return SNAPMD_OK;
                }
                const int nc = plan[c];
                const size_t o = 3 * (size_t)N * s0;
                HIPCHK(hipStreamWaitEvent(s2, ctx->pipe_ev[c], 0));
                HIPCHK(hipStreamWaitEvent(s2, ctx->pipe_ev[ne + 2 + c], 0));
                launch_jumps(3 * (size_t)nc * N, ctx->pr_xf.p + o, ctx->pr_xc.p + o, s2);
                launch_jumps(3 * (size_t)nc * N, ctx->pr_pf.p + o, ctx->pr_pc.p + o, s2);
                if (lds_sweep) {
                    SweepLaunch sc = sw;
                    sc.n_in = n_in + s0;
                    sc.n_fi = n_in + s0 + nc;
                    sc.jq = ctx->pr_xf.p + o;
                    sc.jp = ctx->pr_pf.p + o;
                    sc.noise = sw.noise + (size_t)s0 * L * 3 * N;
                    if ((r = sweep_launch(sc, s2))) return r;
                    HIPCHK(hipEventRecord(ctx->sweep_chunk_ev[c], s2));
                }
            }
            HIPCHK(hipEventRecord(ctx->pipe_ev[ne], s2));
            return SNAPMD_OK;
        };
        // the SNAP propagation of chunk c on SNAP stream `side` (0: the caller's, 1: the
        // second), with the prev := cur copy of its window slots first (pipelined)
        auto fine_chunk = [&](int c, int s0) -> int {
            const int side = side_of(c);
            hipStream_t fst = side ? ctx->fine2_stream : st;
            Work &fw = side ? ctx->w2 : ctx->w;
            double *ff = side ? ctx->d_f2 : ctx->d_f;
            BatchDev bc;
            LangevinDev lc;
            const int nc = chunk_of(c, s0, bc, lc);
            const size_t o = 3 * (size_t)N * s0;
            if (c > 0 && side_of(c - 1) != side) {
                // slot s0 comes with chunk c - 1's copy, queued on the other SNAP stream
                if (pipelined) {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || copied[c - 1]; });
                    if (stop) return SNAPMD_OK;
                    lk.unlock();
                    HIPCHK(hipStreamWaitEvent(fst, ctx->pipe_ev[2 * ne + 2 + c - 1], 0));
                }
                // In an iteration that does not follow a pipelined one the sweep waits for
                // each chunk in turn from the start, so the chunks run one after another:
                // chunk c waits for chunk c - 1 instead of sharing the device with it and
                // delaying the sweep of both (only the order of the launches changes)
                if (!chained) {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || done_f[c - 1]; });
                    if (stop) return SNAPMD_OK;
                    lk.unlock();
                    HIPCHK(hipStreamWaitEvent(fst, ctx->pipe_ev[c - 1], 0));
                }
            }
            if (pipelined) {
                // prev := cur on the window slots s0 .. s0 + nc (s0 + 1 .. for c > 0: slot s0
                // came with the previous chunk): all written by the previous iteration's
                // sweep up to the end of its chunk c
                if (chained) HIPCHK(hipStreamWaitEvent(fst, ctx->sweep_chunk_ev[c], 0));
                const int a = c == 0 ? 0 : s0 + 1, b = s0 + nc;
                const size_t first = (size_t)(n_in + a) * slot, len = (size_t)(b - a + 1) * slot * sizeof(double);
                HIPCHK(hipMemcpyAsync(q_prev + first, q_cur + first, len, hipMemcpyDeviceToDevice, fst));
                HIPCHK(hipMemcpyAsync(p_prev + first, p_cur + first, len, hipMemcpyDeviceToDevice, fst));
                HIPCHK(hipEventRecord(ctx->pipe_ev[2 * ne + 2 + c], fst));
                mark(copied, c);
            }
            launch_slabs_to_batch(nc, N, qs + s0 * slot, ctx->pr_xf.p + o, fst);
            launch_slabs_to_batch(nc, N, ps + s0 * slot, ctx->pr_pf.p + o, fst);
            int r;
            if ((r = run_langevin_graph(ctx, fw, ff, SNAPMD_POT_FS_SNAP, bc, fp, sd, lc, L, ctx->pr_xf.p + o,
                                        ctx->pr_pf.p + o, fst)))
                return r;
            HIPCHK(hipEventRecord(ctx->pipe_ev[c], fst));
            mark(done_f, c);
            return SNAPMD_OK;
        };
        // the chunks of one SNAP stream, in order
        auto fine_side = [&](int side) -> int {
            for (int c = 0, s0 = 0; c < (int)plan.size(); s0 += plan[c], ++c) {
                if (side_of(c) != side) continue;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    if (stop) return SNAPMD_OK;
                }
                int r;
                if ((r = fine_chunk(c, s0))) return r;
            }
            return SNAPMD_OK;
        };
        int rc1 = SNAPMD_OK, rc2 = SNAPMD_OK, rc3 = SNAPMD_OK, rc4 = SNAPMD_OK;
        std::thread t_coarse([&] {
            rc3 = coarse_side();
            if (rc3) halt();
        });
        std::thread t_sweep([&] {
            rc2 = sweep_side();
            if (rc2) halt();
        });
        std::thread t_fine2;
        if (two)
            t_fine2 = std::thread([&] {
                const hipError_t e = hipSetDevice(ctx->device);
                Quiet quiet;
                rc4 = e == hipSuccess ? fine_side(1) : fail(ctx, SNAPMD_EHIP, "hipSetDevice failed");
                if (rc4) halt();
            });
        rc1 = fine_side(0);
        if (pipelined && !rc1) {
            // the neighbour-list error bits once the fine propagation is done (sticky: set by
            // the kernels, cleared by snapmd_sync and snapmd_parareal_collect on an error);
            // the caller's stream waits for the second SNAP stream's chunks first
            if (two && t_fine2.joinable()) t_fine2.join();
            double *h = ctx->h_async + snapmd_ctx::kAsyncStride * aslot;
            hipError_t e = hipSuccess;
            for (int c = 0; c < ne && e == hipSuccess && !rc4; ++c)
                if (side_of(c)) e = hipStreamWaitEvent(st, ctx->pipe_ev[c], 0);
            if (e == hipSuccess && !rc4)
                e = hipMemcpyAsync(reinterpret_cast<int *>(h + 16), ctx->w.status, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && !rc4) e = hipEventRecord(ctx->pipe_ev[3 * ne + 2], st);
            if (e != hipSuccess) rc1 = fail(ctx, SNAPMD_EHIP, "reading the list status failed: %s", hipGetErrorString(e));
        }
        if (rc1) halt();
        if (t_fine2.joinable()) t_fine2.join();
        t_coarse.join();
        t_sweep.join();
        if (pipelined && (rc1 || rc2 || rc3 || rc4)) (void)hipDeviceSynchronize();  // nothing left in flight
        if (rc1) return rc1;
        if (rc4) return rc4;
        if (rc3) return rc3;
        if (rc2) return rc2;
        if (pipelined) {
            // the result (sweep state, neighbour-list status) reaches the pinned slot on the
            // sweep stream; the caller's stream does not wait for the sweep
            double *h = ctx->h_async + snapmd_ctx::kAsyncStride * aslot;
            HIPCHK(hipMemcpyAsync(h, sw.out, 8 * sizeof(double), hipMemcpyDeviceToHost, s2));
            HIPCHK(hipStreamWaitEvent(s2, ctx->pipe_ev[3 * ne + 2], 0));  // the list status read
            HIPCHK(hipEventRecord(ctx->async_ev[aslot], s2));
            ctx->chain_end = ctx->async_ev[aslot];
            ctx->chain_key = key;
            ctx->async_q.push_back({aslot, SNAPMD_OK, 0.0, 0});
            ++ctx->async_seq;
            *delta_out = 0.0;
            return SNAPMD_OK;
        }
        HIPCHK(hipStreamWaitEvent(st, ctx->pipe_ev[ne], 0));
        sw.jq = ctx->pr_xf.p;
        sw.jp = ctx->pr_pf.p;
    } else if (lds_sweep) {
        if ((rc = launch_noise_sweep(ctx, n_in, S, L, N, lang, st))) return rc;
        sw.noise = ctx->sw_noise.p;
        if ((rc = sweep_launch(sw, st))) return rc;
    }
    if (lds_sweep) {
        HIPCHK(hipMemcpyAsync(ctx->h_out, ctx->sw_out.p, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
        if ((rc = snapmd_sync(ctx, stream))) return rc;
        if (ctx->h_out[3] != 0.0)
            return fail(ctx, SNAPMD_EOVERFLOW, "an atom of the coarse sweep has more than its list capacity of "
                                               "neighbours");
        if (ctx->h_out[7] != 0.0)
            return fail(ctx, SNAPMD_EHIP, "the workgroups of the coarse sweep did not meet at a barrier in time");
        if (ctx->h_out[2] >= 0.0)
            return fail(ctx, SNAPMD_ENONFINITE, "state became non-finite in slab %d", (int)ctx->h_out[2]);
        *delta_out = ctx->h_out[0];
        *n_fi = (int32_t)ctx->h_out[1];
        return SNAPMD_OK;
    }
    // Large systems: the same sweep driven from the host with the batched kernels.
    return host_sweep(ctx, potC, fpc, sdc, lang, lang->T_sys[0], lang->noise_id_sys[0], N, box, L, n_in, n_fi, init,
                      (size_t)N, q_cur, p_cur, q_prev, sw.jq, sw.jp, SN3 / 3, (size_t)N, delta_expl, delta_out, st,
                      stream);
}


// Largest chunk of (system, slab) entries propagated in one launch sequence by the
// multi-system path (bounds the neighbour-list and SNAP workspace, ~21 KB per atom).
constexpr long kMultiChunkAtoms = 1L << 20;

// Several systems, each with its own window [n_in[r], n_fi[r]] (n_in[r] = n_fi[r]: none),
// states in the slot layout [slot][3][N_tot].  The fine and coarse propagations of every
// (system, slab) entry of every window run as ragged batches (chunks of at most
// kMultiChunkAtoms atoms, fine then coarse on the caller's stream); the jumps land in the
// slot layout; the sweeps of all systems that the LDS-resident sweep takes run in one
// launch (one workgroup each), the others from the host one system after the other.
int parareal_multi(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                   const snapmd_langevin *lang, int32_t L, const int32_t *n_in, int32_t *n_fi, int32_t n_slots,
                   double *q_prev, double *p_prev, double *q_cur, double *p_cur, double delta_expl,
                   double *delta_out, hipStream_t st, void *stream) {
    int rc;
    const int R = batch->n_sys;
    const int *off = batch->offset;
    const int Nt = off[R];
    const bool init = q_prev == nullptr;
    const bool bbk = lang->scheme == SNAPMD_SCHEME_BBK;
    const bool csnap = ctx->coarse_snap_on;
    const int potC = csnap ? SNAPMD_POT_FS_SNAP : SNAPMD_POT_FS;
    const double skin = kSweepSkin;
    double mh = INFINITY;
    for (int r = 0; r < R; ++r)
        for (int a = 0; a < 3; ++a) mh = std::min(mh, 0.5 * batch->box[3 * r + a]);
    FsParams fp, fpc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if ((rc = coarse_fs(ctx, fp, mh, fpc))) return rc;
    if (!(std::max(fpc.d, fpc.c) + 2.0 * skin < mh))
        return fail(ctx, SNAPMD_EINVAL, "FS cutoff + %g A must be < half the smallest box edge", 2.0 * skin);
    SnapDev sdc;
    if (csnap) {
        snapmd_snap cs = ctx->coarse_snap;
        cs.beta = ctx->coarse_beta.data();
        if (snap && !init && snap->twojmax == cs.twojmax)
            return fail(ctx, SNAPMD_EINVAL, "the coarse SNAP needs a twojmax other than the fine one (%d)",
                        cs.twojmax);
        if ((rc = prepare_snap(ctx, &cs, mh, sdc, st))) return rc;
    }
    for (int r = 0; r < R; ++r) delta_out[r] = 0.0;
    std::vector<int> act;
    for (int r = 0; r < R; ++r)
        if (n_fi[r] > n_in[r] && off[r + 1] > off[r]) act.push_back(r);
    if (act.empty()) return SNAPMD_OK;
    const double c1 = std::exp(-lang->gamma * lang->dt);
    // which sweep each system takes; every buffer is sized before the first launch (a
    // reallocation drops the captured launch sequences)
    std::vector<int> dev_sys, host_sys;
    int max_host = 0;
    for (int r : act) {
        const int Nr = off[r + 1] - off[r];
        if (!bbk && !csnap && sweep_fits_lds(Nr)) {
            dev_sys.push_back(r);
        } else {
            host_sys.push_back(r);
            max_host = std::max(max_host, Nr);
        }
    }
    const size_t ab = sweep_args_bytes();
    if ((rc = ensure(ctx, ctx->m_out, 8 * dev_sys.size())) || (rc = ensure(ctx, ctx->m_tab, ab * dev_sys.size())) ||
        (rc = ensure(ctx, ctx->sw_x, 3 * (size_t)max_host)) || (rc = ensure(ctx, ctx->sw_p, 3 * (size_t)max_host)) ||
        (rc = ensure(ctx, ctx->sw_out, 8)))
        return rc;
    if (!ctx->h_out) HIPCHK(hipHostMalloc((void **)&ctx->h_out, 16 * sizeof(double), hipHostMallocDefault));
    double *jq = nullptr, *jp = nullptr;
    if (!init) {
        // prev := cur on every window
        std::vector<int2> win(R);
        for (int r = 0; r < R; ++r) win[r] = make_int2(n_in[r], n_fi[r]);
        if ((rc = ensure(ctx, ctx->m_off, (size_t)R + 1)) || (rc = ensure(ctx, ctx->m_win, (size_t)R))) return rc;
        const size_t SS = (size_t)n_slots * 3 * Nt;
        if ((rc = ensure(ctx, ctx->m_jq, SS)) || (rc = ensure(ctx, ctx->m_jp, SS))) return rc;
        if ((rc = upload(ctx, ctx->m_off.p, off, (size_t)R + 1, st)) ||
            (rc = upload(ctx, ctx->m_win.p, win.data(), (size_t)R, st)))
            return rc;
        launch_copy_windows(n_slots, Nt, R, ctx->m_off.p, ctx->m_win.p, q_cur, p_cur, q_prev, p_prev, st);
        jq = ctx->m_jq.p;
        jp = ctx->m_jp.p;
        // entries (system, slab), cut into chunks
        struct Ent { int r, n; };
        std::vector<Ent> ent;
        for (int r : act)
            for (int n = n_in[r]; n < n_fi[r]; ++n) ent.push_back({r, n});
        std::vector<size_t> cut{0};
        long acc = 0, maxc = 0;
        for (size_t e = 0; e < ent.size(); ++e) {
            const long na = off[ent[e].r + 1] - off[ent[e].r];
            if (acc > 0 && acc + na > kMultiChunkAtoms) {
                maxc = std::max(maxc, acc);
                cut.push_back(e);
                acc = 0;
            }
            acc += na;
        }
        maxc = std::max(maxc, acc);
        cut.push_back(ent.size());
        const size_t M3 = 3 * (size_t)maxc;
        if ((rc = ensure(ctx, ctx->pr_xf, M3)) || (rc = ensure(ctx, ctx->pr_pf, M3)) ||
            (rc = ensure(ctx, ctx->pr_xc, M3)) || (rc = ensure(ctx, ctx->pr_pc, M3)) ||
            (rc = ensure(ctx, ctx->m_src, ent.size())))
            return rc;
        if ((rc = ensure_atoms(ctx, (size_t)maxc)) || (rc = ensure_atoms_coarse(ctx, (size_t)maxc, csnap))) return rc;
        for (size_t c = 0; c + 1 < cut.size(); ++c) {
            const int ne = (int)(cut[c + 1] - cut[c]);
            std::vector<int> boff(ne + 1, 0);
            std::vector<double> boxes(3 * (size_t)ne), T(ne);
            std::vector<int64_t> step0(ne);
            std::vector<int> nid(ne);
            std::vector<int4> src(ne);
            for (int k = 0; k < ne; ++k) {
                const Ent &e = ent[cut[c] + k];
                boff[k + 1] = boff[k] + (off[e.r + 1] - off[e.r]);
                for (int a = 0; a < 3; ++a) boxes[3 * k + a] = batch->box[3 * e.r + a];
                T[k] = lang->T_sys[e.r];
                step0[k] = (int64_t)e.n * L;
                nid[k] = lang->noise_id_sys[e.r];
                src[k] = make_int4(e.n, off[e.r], e.n, 0);
            }
            const int Nc = boff[ne];
            snapmd_batch sb{ne, boff.data(), boxes.data()};
            BatchDev bd;
            double mh2;
            SnapDev sd;
            LangevinDev ldv;
            if ((rc = prepare_batch(ctx, &sb, bd, mh2, st)) || (rc = prepare_snap(ctx, snap, mh2, sd, st)) ||
                (rc = prepare_langevin(ctx, lang, ne, T, step0, nid, ldv, st)))
                return rc;
            int4 *dsrc = ctx->m_src.p + cut[c];
            if ((rc = upload(ctx, dsrc, src.data(), (size_t)ne, st))) return rc;
            launch_entries_to_batch(Nc, ne, bd.off, dsrc, Nt, q_prev, ctx->pr_xf.p, st);
            launch_entries_to_batch(Nc, ne, bd.off, dsrc, Nt, p_prev, ctx->pr_pf.p, st);
            HIPCHK(hipMemcpyAsync(ctx->pr_xc.p, ctx->pr_xf.p, 3 * (size_t)Nc * sizeof(double), hipMemcpyDeviceToDevice,
                                  st));
            HIPCHK(hipMemcpyAsync(ctx->pr_pc.p, ctx->pr_pf.p, 3 * (size_t)Nc * sizeof(double), hipMemcpyDeviceToDevice,
                                  st));
            if ((rc = run_langevin_graph(ctx, ctx->w, ctx->d_f, SNAPMD_POT_FS_SNAP, bd, fp, sd, ldv, L, ctx->pr_xf.p,
                                         ctx->pr_pf.p, st)) ||
                (rc = run_langevin_graph(ctx, ctx->wc, ctx->d_fc, potC, bd, fpc, sdc, ldv, L, ctx->pr_xc.p,
                                         ctx->pr_pc.p, st)))
                return rc;
            launch_batch_jumps_to_slots(Nc, ne, bd.off, dsrc, Nt, ctx->pr_xf.p, ctx->pr_xc.p, jq, st);
            launch_batch_jumps_to_slots(Nc, ne, bd.off, dsrc, Nt, ctx->pr_pf.p, ctx->pr_pc.p, jp, st);
            if ((rc = check_launch(ctx))) return rc;
        }
    }
    // sweeps: the LDS-resident kernel for every system it takes, in one launch
    if (!dev_sys.empty()) {
        const int nd = (int)dev_sys.size();
        std::vector<unsigned char> tab(ab * nd);
        std::vector<double> out0(8 * (size_t)nd);
        int maxN = 0;
        for (int k = 0; k < nd; ++k) {
            const int r = dev_sys[k], Nr = off[r + 1] - off[r];
            const double *box = batch->box + 3 * r;
            maxN = std::max(maxN, Nr);
            SweepLaunch sw{};
            sw.N = Nr;
            for (int a = 0; a < 3; ++a) sw.box[a] = box[a];
            sw.fp = fpc;
            sw.skin = skin;
            sw.dt = lang->dt;
            sw.c1 = c1;
            sw.mass = lang->mass;
            sw.sig = std::sqrt((1.0 - c1 * c1) * lang->mass * kKB * lang->T_sys[r] / kMVV2E);
            sw.seed = lang->seed;
            sw.noise_id = (uint64_t)lang->noise_id_sys[r];
            sw.L = L;
            sw.n_in = n_in[r];
            sw.n_fi = n_fi[r];
            sw.mode = init ? 0 : 1;
            sw.n_win = n_in[r];
            int nc[3];
            for (int a = 0; a < 3; ++a) nc[a] = (int)std::floor(box[a] / (std::max(fpc.d, fpc.c) + skin));
            while ((long)nc[0] * nc[1] * nc[2] > 512) *std::max_element(nc, nc + 3) -= 1;
            if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) nc[0] = nc[1] = nc[2] = 0;
            sw.ncx = nc[0];
            sw.ncy = nc[1];
            sw.ncz = nc[2];
            sw.delta_expl = delta_expl;
            sw.q_cur = q_cur + off[r];
            sw.p_cur = p_cur + off[r];
            sw.q_prev = init ? nullptr : q_prev + off[r];
            sw.p_prev = init ? nullptr : p_prev + off[r];
            sw.jq = init ? nullptr : jq + (size_t)n_in[r] * 3 * Nt + off[r];
            sw.jp = init ? nullptr : jp + (size_t)n_in[r] * 3 * Nt + off[r];
            sw.out = ctx->m_out.p + 8 * (size_t)k;
            sw.noise = nullptr;
            fill_sweep_args(sw, (size_t)Nt, (size_t)Nt, 3 * (size_t)Nt, tab.data() + ab * k);
            const double o[8] = {0.0, (double)n_fi[r], -1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            std::copy(o, o + 8, out0.begin() + 8 * k);
        }
        if ((rc = upload(ctx, ctx->m_tab.p, tab.data(), tab.size(), st)) ||
            (rc = upload(ctx, ctx->m_out.p, out0.data(), out0.size(), st)))
            return rc;
        launch_coarse_sweep_multi(ctx->m_tab.p, nd, maxN, st);
        if ((rc = check_launch(ctx))) return rc;
        HIPCHK(hipMemcpyAsync(out0.data(), ctx->m_out.p, out0.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        if ((rc = snapmd_sync(ctx, stream))) return rc;
        for (int k = 0; k < nd; ++k) {
            const int r = dev_sys[k];
            const double *o = out0.data() + 8 * k;
            if (o[3] != 0.0)
                return fail(ctx, SNAPMD_EOVERFLOW, "an atom of the coarse sweep of system %d has more than its list "
                                                   "capacity of neighbours", r);
            if (o[2] >= 0.0)
                return fail(ctx, SNAPMD_ENONFINITE, "state of system %d became non-finite in slab %d", r, (int)o[2]);
            delta_out[r] = o[0];
            n_fi[r] = (int32_t)o[1];
        }
    }
    for (int r : host_sys) {
        const int Nr = off[r + 1] - off[r];
        const size_t jb = (size_t)n_in[r] * 3 * Nt + off[r];
        if ((rc = host_sweep(ctx, potC, fpc, sdc, lang, lang->T_sys[r], lang->noise_id_sys[r], Nr, batch->box + 3 * r, L,
                             n_in[r], n_fi + r, init, (size_t)Nt, q_cur + off[r], p_cur + off[r],
                             init ? nullptr : q_prev + off[r], init ? nullptr : jq + jb, init ? nullptr : jp + jb,
                             (size_t)Nt, 3 * (size_t)Nt, delta_expl, delta_out + r, st, stream)))
            return fail(ctx, rc, "system %d: %s", r, std::string(ctx->err).c_str());
    }
    return SNAPMD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free SNAP forces: every work buffer of snap_forces_noalloc lives in one
// file-scope device array.  Host code never uses the array's name as an address: the
// address on each device comes from hipGetSymbolAddress, taken once per device when a
// context is created on it.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)SNAPMD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch;  // device -> address of `scratch` on it

// the current device must be `device`
int scratch_setup(int device, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it == g_scratch.end()) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SNAPMD_EHIP;
        it = g_scratch.emplace(device, (unsigned char *)ptr).first;
    }
    *out = it->second;
    return SNAPMD_OK;
}

// Carves aligned regions out of the scratch array.
struct Carve {
    unsigned char *base;
    size_t used = 0;
    template <class T>
    T *take(size_t n) {
        used = (used + 255) & ~(size_t)255;
        T *p = (T *)(base + used);
        used += n * sizeof(T);
        return p;
    }
};

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
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
            ctx->n_cus = cus;
    }
    adjoint_init_attributes();
    sweep_init_attributes();
    neigh_init_attributes();
    if (scratch_setup(hip_device, &ctx->scratch) != SNAPMD_OK) {
        delete ctx;
        return SNAPMD_EHIP;
    }
    if (dalloc(ctx, &ctx->w.status, 1) != SNAPMD_OK || hipMemset(ctx->w.status, 0, sizeof(int)) != hipSuccess ||
        dalloc(ctx, &ctx->w.flag, 1) != SNAPMD_OK || hipMemset(ctx->w.flag, 0, sizeof(int)) != hipSuccess) {
        snapmd_destroy(ctx);
        return SNAPMD_ENOMEM;
    }
    *out = ctx;
    return SNAPMD_OK;
}

void snapmd_destroy(snapmd_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)drain(ctx);
    for (void *p : ctx->allocs) (void)hipFree(p);
    if (ctx->h_out) (void)hipHostFree(ctx->h_out);
    if (ctx->h_async) (void)hipHostFree(ctx->h_async);
    for (hipEvent_t e : ctx->async_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->sweep_chunk_ev) (void)hipEventDestroy(e);
    drop_graphs(ctx);
    for (hipStream_t c : ctx->cap_stream)
        if (c) (void)hipStreamDestroy(c);
    if (ctx->sweep_stream) (void)hipStreamDestroy(ctx->sweep_stream);
    if (ctx->coarse_stream) (void)hipStreamDestroy(ctx->coarse_stream);
    for (hipEvent_t e : ctx->pipe_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char *snapmd_last_error(const snapmd_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int snapmd_sync(snapmd_ctx *ctx, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
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
    if (const int rc_ = drain(ctx)) return rc_;
    if (!x || !f) return fail(ctx, SNAPMD_EINVAL, "x and f must be device pointers");
    BatchDev bd;
    double mh;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    if ((rc = neighbors(ctx, ctx->w, bd, x, snap->rcut, true, st))) return rc;
    launch_snap(sd.J, bd, x, sd, ctx->w, f, e_atom, (flags & SNAPMD_ACCUMULATE) ? 1 : 0, st, &ctx->prof);
    return check_launch(ctx);
}

int snap_forces_noalloc(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch, const double *x,
                        double *f, double *e_atom, uint32_t flags, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (!ctx->scratch) return fail(ctx, SNAPMD_EHIP, "the scratch array of this device is not set up");
    if (!x || !f) return fail(ctx, SNAPMD_EINVAL, "x and f must be device pointers");
    if (!batch || !batch->offset || !batch->box) return fail(ctx, SNAPMD_EINVAL, "batch, offset and box must be set");
    const int S = batch->n_sys;
    if (S < 1 || S > SNAPMD_NOALLOC_MAX_SYS)
        return fail(ctx, SNAPMD_EINVAL, "snap_forces_noalloc: need 1 <= n_sys <= %d (got %d)", SNAPMD_NOALLOC_MAX_SYS, S);
    if (batch->offset[0] != 0) return fail(ctx, SNAPMD_EINVAL, "batch.offset[0] must be 0");
    double mh = INFINITY;
    int max_sys = 0;
    for (int q = 0; q < S; ++q) {
        if (batch->offset[q + 1] < batch->offset[q])
            return fail(ctx, SNAPMD_EINVAL, "batch.offset must be nondecreasing (system %d)", q);
        max_sys = std::max(max_sys, batch->offset[q + 1] - batch->offset[q]);
        for (int a = 0; a < 3; ++a) {
            const double L = batch->box[3 * q + a];
            if (!(L > 0.0) || !std::isfinite(L))
                return fail(ctx, SNAPMD_EINVAL, "box edge %d of system %d must be finite and > 0", a, q);
            mh = std::min(mh, 0.5 * L);
        }
    }
    const int N = batch->offset[S];
    if (N > SNAPMD_NOALLOC_MAX_ATOMS)
        return fail(ctx, SNAPMD_EINVAL, "snap_forces_noalloc takes at most %d atoms (got %d); use snap_forces",
                    SNAPMD_NOALLOC_MAX_ATOMS, N);
    if (!snap) return fail(ctx, SNAPMD_EINVAL, "snap is NULL");
    const int J = snap->twojmax;
    if (J < 2 || J > kMaxJLds || (J & 1))
        return fail(ctx, SNAPMD_EUNSUPPORTED, "snap_forces_noalloc takes twojmax 2, 4, 6 or 8 (got %d)", J);
    const SnapTables &T = snap_tables(J);
    if (snap->n_coeff != T.K)
        return fail(ctx, SNAPMD_EINVAL, "n_coeff must be %d for twojmax %d (got %d)", T.K, J, snap->n_coeff);
    if (!snap->beta) return fail(ctx, SNAPMD_EINVAL, "snap.beta is NULL");
    if (!(snap->rcut > 0.0) || !(snap->rmin0 >= 0.0) || !(snap->rmin0 < snap->rcut))
        return fail(ctx, SNAPMD_EINVAL, "need 0 <= rmin0 < rcut (rcut %g, rmin0 %g)", snap->rcut, snap->rmin0);
    if (!(snap->rfac0 > 0.0 && snap->rfac0 < 1.0))
        return fail(ctx, SNAPMD_EINVAL, "need 0 < rfac0 < 1 (got %g)", snap->rfac0);
    if (!(snap->rcut < mh))
        return fail(ctx, SNAPMD_EINVAL, "rcut %g must be < half the smallest box edge %g", snap->rcut, mh);
    for (int k = 0; k <= T.K; ++k)
        if (!std::isfinite(snap->beta[k])) return fail(ctx, SNAPMD_EINVAL, "beta[%d] is not finite", k);
    if (N == 0) return SNAPMD_OK;
    AdjointHost &A = ctx->na_adj;
    adjoint_tables(J, snap->beta, A);
    // regions of the scratch array (nothing in them has to start at zero: every kernel
    // writes what it later reads, and the list build is forced)
    Carve cv{ctx->scratch};
    const size_t P = (size_t)N * kMaxNeigh;
    int *d_off = cv.take<int>(S + 1);
    double *d_box = cv.take<double>(3 * (size_t)S);
    int4 *d_cells = cv.take<int4>(S);
    double *d_nrm = cv.take<double>(T.nh), *d_ymult = cv.take<double>(T.nh);
    double *d_cgm = cv.take<double>(A.cgm.size()), *d_coef = cv.take<double>(A.coef.size());
    int *d_coef_off = cv.take<int>(A.coef_off.size()), *d_roles = cv.take<int>(A.roles.size());
    Work w{};
    w.Pcap = P;
    w.nbr = cv.take<int>(P);
    w.cnt = cv.take<int>(N);
    w.poff = cv.take<int>((size_t)N + 1);
    w.pair_i = cv.take<int>(P);
    w.pair_j = cv.take<int>(P);
    w.rev = cv.take<int>(P);
    w.ell = cv.take<double>(6 * P);
    w.nbr_t = cv.take<int>(P);
    w.dedr = cv.take<double>(3 * P);
    w.u = cv.take<double2>((size_t)T.nh * N);
    w.ytil = cv.take<double2>((size_t)T.nh * N);
    w.xref = cv.take<double>(3 * (size_t)N);
    w.status = ctx->w.status;  // overflow bits, reported by snapmd_sync
    w.flag = ctx->w.flag;
    if (cv.used > kNoAllocBytes)
        return fail(ctx, SNAPMD_EINVAL, "snap_forces_noalloc: %zu bytes of work space exceed the %zu of the array",
                    cv.used, kNoAllocBytes);
    // the cell grids the list build of snap_forces uses (same lists, same order)
    std::vector<int4> ci(S);
    int n_cells = 0;
    const double rl = snap->rcut + kSkin;
    for (int q = 0; q < S; ++q) {
        int n3[3];
        for (int a = 0; a < 3; ++a) n3[a] = (int)std::floor(batch->box[3 * q + a] / rl);
        if (n3[0] >= 3 && n3[1] >= 3 && n3[2] >= 3 && batch->offset[q + 1] - batch->offset[q] >= 500) {
            ci[q] = make_int4(n3[0], n3[1], n3[2], n_cells);
            n_cells += n3[0] * n3[1] * n3[2];
        } else {
            ci[q] = make_int4(0, 0, 0, n_cells);
        }
    }
    int rc;
    if ((rc = upload(ctx, d_off, batch->offset, (size_t)S + 1, st)) || (rc = upload(ctx, d_box, batch->box, 3 * (size_t)S, st)) ||
        (rc = upload(ctx, d_cells, ci.data(), (size_t)S, st)) ||
        (rc = upload(ctx, d_nrm, T.nrm.data(), (size_t)T.nh, st)) ||
        (rc = upload(ctx, d_ymult, T.ymult.data(), (size_t)T.nh, st)) ||
        (rc = upload(ctx, d_cgm, A.cgm.data(), A.cgm.size(), st)) ||
        (rc = upload(ctx, d_coef, A.coef.data(), A.coef.size(), st)) ||
        (rc = upload(ctx, d_coef_off, A.coef_off.data(), A.coef_off.size(), st)) ||
        (rc = upload(ctx, d_roles, A.roles.data(), A.roles.size(), st)))
        return rc;
    BatchDev bd;
    bd.N = N;
    bd.n_sys = S;
    bd.off = d_off;
    bd.box = d_box;
    bd.max_sys = max_sys;  // every system fits the one-workgroup list build (N <= 2048)
    bd.cells = d_cells;
    bd.n_cells = n_cells;
    SnapDev sd;
    sd.J = J;
    sd.K = T.K;
    sd.nh = T.nh;
    sd.gp = SnapGeoParams{snap->rcut, snap->rfac0, snap->rmin0};
    sd.beta0 = snap->beta[0];
    sd.nrm = d_nrm;
    sd.ymult = d_ymult;
    sd.adj = AdjointDev{d_cgm, d_coef, d_coef_off, d_roles, A.role_len};
    sd.shape.dens_parts = 1;  // the scratch array holds one density (no split)
    launch_neighbors(bd, x, snap->rcut, w, st, true, kSkin);
    launch_snap(J, bd, x, sd, w, f, e_atom, (flags & SNAPMD_ACCUMULATE) ? 1 : 0, st);
    return check_launch(ctx);
}

int eam_forces(snapmd_ctx *ctx, const snapmd_fs *fs, const snapmd_batch *batch, const double *x, double *f,
               double *e_atom, uint32_t flags, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (!x || !f) return fail(ctx, SNAPMD_EINVAL, "x and f must be device pointers");
    BatchDev bd;
    double mh;
    FsParams fp;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    if ((rc = neighbors(ctx, ctx->w, bd, x, std::max(fp.d, fp.c), true, st))) return rc;
    launch_fs(bd, x, fp, ctx->w, f, e_atom, (flags & SNAPMD_ACCUMULATE) ? 1 : 0, st);
    return check_launch(ctx);
}

int langevin_steps(snapmd_ctx *ctx, int potential, const snapmd_snap *snap, const snapmd_fs *fs,
                   const snapmd_batch *batch, const snapmd_langevin *lang, int32_t n_steps, double *x, double *p,
                   double *f_out, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (potential != SNAPMD_POT_FS && potential != SNAPMD_POT_FS_SNAP)
        return fail(ctx, SNAPMD_EINVAL, "potential must be SNAPMD_POT_FS or SNAPMD_POT_FS_SNAP");
    if (!x || !p) return fail(ctx, SNAPMD_EINVAL, "x and p must be device pointers");
    if (n_steps < 0) return fail(ctx, SNAPMD_EINVAL, "n_steps must be >= 0");
    int rc;
    if ((rc = check_lang(ctx, lang))) return rc;
    BatchDev bd;
    double mh;
    FsParams fp;
    SnapDev sd;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if (potential == SNAPMD_POT_FS_SNAP && (rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    const int S = bd.n_sys;
    std::vector<double> T(lang->T_sys, lang->T_sys + S);
    std::vector<int64_t> step0(lang->step0_sys, lang->step0_sys + S);
    std::vector<int> nid(lang->noise_id_sys, lang->noise_id_sys + S);
    for (int s = 0; s < S; ++s) {
        if (!(T[s] >= 0.0)) return fail(ctx, SNAPMD_EINVAL, "T_sys[%d] must be >= 0", s);
        if (nid[s] < 0) return fail(ctx, SNAPMD_EINVAL, "noise_id_sys[%d] must be >= 0", s);
    }
    LangevinDev ld;
    if ((rc = prepare_langevin(ctx, lang, S, T, step0, nid, ld, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    if ((rc = run_langevin_graph(ctx, ctx->w, ctx->d_f, potential, bd, fp, sd, ld, n_steps, x, p, st))) return rc;
    if (f_out)
        HIPCHK(hipMemcpyAsync(f_out, ctx->d_f, 3 * (size_t)bd.N * sizeof(double), hipMemcpyDeviceToDevice, st));
    return check_launch(ctx);
}

namespace {
int parareal_entry(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                   const snapmd_langevin *lang, int32_t L, const int32_t *n_in, int32_t *n_fi, int32_t n_slots,
                   double *q_prev, double *p_prev, double *q_cur, double *p_cur, double delta_expl,
                   double *delta_out, void *stream, bool async) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    int rc;
    if ((rc = check_lang(ctx, lang))) return rc;
    if (!batch || batch->n_sys < 1 || !batch->offset || !batch->box)
        return fail(ctx, SNAPMD_EINVAL, "parareal_iterate needs a batch of at least one system");
    if (!n_in || !n_fi || !delta_out) return fail(ctx, SNAPMD_EINVAL, "n_in, n_fi and delta_out must be host arrays");
    if (L < 1) return fail(ctx, SNAPMD_EINVAL, "L must be >= 1");
    if (!q_cur || !p_cur) return fail(ctx, SNAPMD_EINVAL, "q_cur and p_cur must be device pointers");
    if (q_prev && !p_prev) return fail(ctx, SNAPMD_EINVAL, "p_prev must be set with q_prev");
    if (!(delta_expl >= 0.0)) return fail(ctx, SNAPMD_EINVAL, "delta_expl must be >= 0");
    const int R = batch->n_sys;
    if (batch->offset[0] != 0) return fail(ctx, SNAPMD_EINVAL, "batch.offset[0] must be 0");
    for (int r = 0; r < R; ++r) {
        if (batch->offset[r + 1] < batch->offset[r])
            return fail(ctx, SNAPMD_EINVAL, "batch.offset must be nondecreasing (system %d)", r);
        for (int a = 0; a < 3; ++a)
            if (!(batch->box[3 * r + a] > 0.0) || !std::isfinite(batch->box[3 * r + a]))
                return fail(ctx, SNAPMD_EINVAL, "box edge %d of system %d must be finite and > 0", a, r);
        if (!(lang->T_sys[r] >= 0.0) || lang->noise_id_sys[r] < 0)
            return fail(ctx, SNAPMD_EINVAL, "need T_sys[%d] >= 0 and noise_id_sys[%d] >= 0", r, r);
        // a window of one system must lie in the state arrays; in a batch of several an
        // empty window (n_in = n_fi) leaves the system out
        if (n_in[r] < 0 || n_fi[r] < n_in[r] || (R == 1 && n_fi[r] == n_in[r]) || n_fi[r] > n_slots - 1)
            return fail(ctx, SNAPMD_EINVAL, "system %d: need 0 <= n_in < n_fi <= n_slots - 1 (got %d, %d, %d slots)", r,
                        n_in[r], n_fi[r], n_slots);
    }
    if (batch->offset[R] < 1) return fail(ctx, SNAPMD_EINVAL, "the batch needs at least one atom");
    if (R == 1)
        return parareal_one(ctx, snap, fs, batch, lang, L, n_in[0], n_fi, q_prev, p_prev, q_cur, p_cur, delta_expl,
                            delta_out, st, stream, async);
    if ((rc = drain(ctx))) return rc;
    return parareal_multi(ctx, snap, fs, batch, lang, L, n_in, n_fi, n_slots, q_prev, p_prev, q_cur, p_cur, delta_expl,
                          delta_out, st, stream);
}
}  // namespace

int parareal_iterate(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                     const snapmd_langevin *lang, int32_t L, const int32_t *n_in, int32_t *n_fi, int32_t n_slots,
                     double *q_prev, double *p_prev, double *q_cur, double *p_cur, double delta_expl,
                     double *delta_out, void *stream) {
    return parareal_entry(ctx, snap, fs, batch, lang, L, n_in, n_fi, n_slots, q_prev, p_prev, q_cur, p_cur, delta_expl,
                          delta_out, stream, false);
}

int parareal_iterate_async(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                           const snapmd_langevin *lang, int32_t L, int32_t n_in, int32_t n_fi, int32_t n_slots,
                           double *q_prev, double *p_prev, double *q_cur, double *p_cur, double delta_expl,
                           void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    if (!batch || batch->n_sys != 1)
        return fail(ctx, SNAPMD_EINVAL, "parareal_iterate_async takes a batch of one system");
    if ((int)ctx->async_q.size() >= snapmd_ctx::kAsyncSlots - 1)
        return fail(ctx, SNAPMD_EINVAL, "at most %d pipelined iterations may wait to be collected",
                    snapmd_ctx::kAsyncSlots - 1);
    const size_t queued = ctx->async_q.size();
    int32_t nf = n_fi;
    double delta = 0.0;
    const int rc = parareal_entry(ctx, snap, fs, batch, lang, L, &n_in, &nf, n_slots, q_prev, p_prev, q_cur, p_cur,
                                  delta_expl, &delta, stream, true);
    if (rc) return rc;
    // not pipelined (window initialisation, host-driven sweep): finished at the call
    if (ctx->async_q.size() == queued) ctx->async_q.push_back({-1, SNAPMD_OK, delta, nf});
    return SNAPMD_OK;
}

int snapmd_parareal_collect(snapmd_ctx *ctx, double *delta_out, int32_t *n_fi_out, void *stream) {
    if (!ctx || !delta_out || !n_fi_out) return SNAPMD_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->async_q.empty()) return fail(ctx, SNAPMD_EINVAL, "no pipelined parareal iteration to collect");
    const snapmd_ctx::AsyncIt it = ctx->async_q.front();
    ctx->async_q.pop_front();
    if (it.slot < 0) {
        *delta_out = it.delta;
        *n_fi_out = it.n_fi;
        return it.rc;
    }
    HIPCHK(hipEventSynchronize(ctx->async_ev[it.slot]));
    HIPCHK(hipStreamWaitEvent((hipStream_t)stream, ctx->async_ev[it.slot], 0));
    const double *h = ctx->h_async + snapmd_ctx::kAsyncStride * it.slot;
    const int status = *reinterpret_cast<const int *>(h + 16);
    if (status) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemset(ctx->w.status, 0, sizeof(int)));
        if (status & 1) return fail(ctx, SNAPMD_EOVERFLOW, "an atom has more than %d neighbours", kMaxNeigh);
        return fail(ctx, SNAPMD_EINVAL, "inconsistent neighbour list (status %d)", status);
    }
    if (h[3] != 0.0)
        return fail(ctx, SNAPMD_EOVERFLOW, "an atom of the coarse sweep has more than its list capacity of neighbours");
    if (h[7] != 0.0) return fail(ctx, SNAPMD_EHIP, "the workgroups of the coarse sweep did not meet at a barrier in time");
    if (h[2] >= 0.0) return fail(ctx, SNAPMD_ENONFINITE, "state became non-finite in slab %d", (int)h[2]);
    *delta_out = h[0];
    *n_fi_out = (int32_t)h[1];
    return SNAPMD_OK;
}

// Device-resident adaptive parareal over a batch of replicas (the paper's Algorithm
// "Adaptive parareal algorithm" for every replica at once).  The host enqueues rounds of a
// fixed launch sequence and synchronises only every rounds_per_check rounds; between
// checks every decision is taken on the device.
int parareal_adaptive(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs, const snapmd_batch *batch,
                      const snapmd_langevin *lang, int32_t L, int32_t N, int32_t max_window, double delta_conv,
                      double delta_expl, int32_t rounds_per_check, int32_t max_rounds, double *q, double *p,
                      snapmd_parareal_log *log, int32_t *rounds_out, int32_t *checks_out, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    int rc;
    if ((rc = drain(ctx))) return rc;
    if ((rc = check_lang(ctx, lang))) return rc;
    if (!batch || batch->n_sys < 1 || !batch->offset || !batch->box)
        return fail(ctx, SNAPMD_EINVAL, "parareal_adaptive needs a batch of at least one system");
    if (!q || !p) return fail(ctx, SNAPMD_EINVAL, "q and p must be device pointers");
    if (!log || !log->n_log || log->max_log < 0 ||
        (log->max_log > 0 && (!log->n_in || !log->n_fi || !log->n_fi_after || !log->delta)))
        return fail(ctx, SNAPMD_EINVAL, "log and its host arrays must be set");
    if (!rounds_out || !checks_out) return fail(ctx, SNAPMD_EINVAL, "rounds_out and checks_out must be host pointers");
    if (L < 1 || N < 1 || max_window < 1 || rounds_per_check < 1 || max_rounds < 1)
        return fail(ctx, SNAPMD_EINVAL, "need L, N, max_window, rounds_per_check, max_rounds >= 1");
    if (!(delta_conv >= 0.0) || !(delta_expl > delta_conv) || !std::isfinite(delta_expl))
        return fail(ctx, SNAPMD_EINVAL, "need 0 <= delta_conv < delta_expl < inf");
    if (lang->scheme != SNAPMD_SCHEME_BAOAB || ctx->coarse_snap_on)
        return fail(ctx, SNAPMD_EUNSUPPORTED, "parareal_adaptive runs BAOAB with a Finnis-Sinclair coarse potential");
    const int R = batch->n_sys;
    const int *off = batch->offset;
    if (off[0] != 0) return fail(ctx, SNAPMD_EINVAL, "batch.offset[0] must be 0");
    double mh = INFINITY;
    int maxN = 0;
    for (int r = 0; r < R; ++r) {
        const int Nr = off[r + 1] - off[r];
        if (Nr < 1) return fail(ctx, SNAPMD_EINVAL, "system %d has no atoms", r);
        if (!sweep_fits_lds(Nr))
            return fail(ctx, SNAPMD_EUNSUPPORTED, "system %d (%d atoms) is too large for the on-device sweep", r, Nr);
        if (!(lang->T_sys[r] >= 0.0) || lang->noise_id_sys[r] < 0)
            return fail(ctx, SNAPMD_EINVAL, "need T_sys[%d] >= 0 and noise_id_sys[%d] >= 0", r, r);
        maxN = std::max(maxN, Nr);
        for (int a = 0; a < 3; ++a) {
            const double b = batch->box[3 * r + a];
            if (!(b > 0.0) || !std::isfinite(b))
                return fail(ctx, SNAPMD_EINVAL, "box edge %d of system %d must be finite and > 0", a, r);
            mh = std::min(mh, 0.5 * b);
        }
    }
    const int Nt = off[R];
    FsParams fp, fpc;
    if ((rc = prepare_fs(ctx, fs, mh, fp)) || (rc = coarse_fs(ctx, fp, mh, fpc))) return rc;
    const double skin = kSweepSkin;
    if (!(std::max(fpc.d, fpc.c) + 2.0 * skin < mh))
        return fail(ctx, SNAPMD_EINVAL, "FS cutoff + %g A must be < half the smallest box edge", 2.0 * skin);
    SnapDev sd, sdc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    const int W = std::min(max_window, N);
    const size_t SS = (size_t)(N + 1) * 3 * Nt, RW = (size_t)R * W;
    const size_t ab = sweep_args_bytes();
    const int ML = log->max_log;
    // every buffer before the first round (an allocation drops the captured sequences)
    long max_chunk = 0;
    {
        long acc = 0;
        for (int r = 0; r < R; ++r)
            for (int s2 = 0; s2 < W; ++s2) {
                const long na = off[r + 1] - off[r];
                if (acc > 0 && acc + na > kMultiChunkAtoms) {
                    max_chunk = std::max(max_chunk, acc);
                    acc = 0;
                }
                acc += na;
            }
        max_chunk = std::max(max_chunk, acc);
    }
    const size_t M3 = 3 * (size_t)max_chunk;
    if ((rc = ensure(ctx, ctx->dr_qprev, SS)) || (rc = ensure(ctx, ctx->dr_pprev, SS)) ||
        (rc = ensure(ctx, ctx->m_jq, SS)) || (rc = ensure(ctx, ctx->m_jp, SS)) ||
        (rc = ensure(ctx, ctx->dr_st, (size_t)R)) || (rc = ensure(ctx, ctx->dr_act, (size_t)R)) ||
        (rc = ensure(ctx, ctx->dr_roff, (size_t)R + 1)) || (rc = ensure(ctx, ctx->m_win, (size_t)R)) ||
        (rc = ensure(ctx, ctx->dr_tab_init, ab * R)) || (rc = ensure(ctx, ctx->dr_tab_it, ab * R)) ||
        (rc = ensure(ctx, ctx->dr_out_init, 8 * (size_t)R)) || (rc = ensure(ctx, ctx->dr_out_it, 8 * (size_t)R)) ||
        (rc = ensure(ctx, ctx->dr_ent, RW)) || (rc = ensure(ctx, ctx->dr_step0, RW)) ||
        (rc = ensure(ctx, ctx->dr_sig, RW)) || (rc = ensure(ctx, ctx->dr_sb, RW)) ||
        (rc = ensure(ctx, ctx->dr_noise, RW)) || (rc = ensure(ctx, ctx->dr_eoff, RW + (size_t)R * W + 1)) ||
        (rc = ensure(ctx, ctx->dr_box, 3 * RW)) || (rc = ensure(ctx, ctx->dr_cells, RW)) ||
        (rc = ensure(ctx, ctx->dr_logi, (size_t)R * std::max(ML, 1))) ||
        (rc = ensure(ctx, ctx->dr_logd, (size_t)R * std::max(ML, 1))) || (rc = ensure(ctx, ctx->dr_err, 1)) ||
        (rc = ensure(ctx, ctx->pr_xf, M3)) || (rc = ensure(ctx, ctx->pr_pf, M3)) ||
        (rc = ensure(ctx, ctx->pr_xc, M3)) || (rc = ensure(ctx, ctx->pr_pc, M3)) ||
        (rc = ensure(ctx, ctx->seg_step0[0], RW)) || (rc = ensure(ctx, ctx->seg_step0[1], RW)))
        return rc;
    if ((rc = ensure_atoms(ctx, (size_t)max_chunk)) || (rc = ensure_atoms_coarse(ctx, (size_t)max_chunk, false)))
        return rc;
    // initial state of every replica: a new window starts at slab 0
    {
        std::vector<DrvState> s0(R);
        for (auto &v : s0) v = DrvState{DRV_NEW, 0, 0, 0, 0.0, 0, -1};
        const int zero = 0;
        if ((rc = upload(ctx, ctx->dr_st.p, s0.data(), (size_t)R, st)) || (rc = upload(ctx, ctx->dr_err.p, &zero, 1, st)) ||
            (rc = upload(ctx, ctx->dr_roff.p, off, (size_t)R + 1, st)))
            return rc;
    }
    const double c1 = std::exp(-lang->gamma * lang->dt);
    std::vector<DrvState> hs(R);
    std::vector<int> act;
    for (int r = 0; r < R; ++r) act.push_back(r);
    int rounds = 0, checks = 0;
    struct Chunk {
        BatchDev bd;
        LangevinDev ld;
        int e0, ne, Nc;
    };
    while (!act.empty()) {
        // tables of the replicas still running: their sweep arguments, and the W entries
        // of each in the batch, cut into chunks
        const int Ra = (int)act.size();
        std::vector<unsigned char> tin(ab * Ra), tit(ab * Ra);
        std::vector<int> eoff;
        std::vector<double> sig(Ra * (size_t)W), sb(Ra * (size_t)W, 0.0), bx(3 * (size_t)Ra * W);
        std::vector<int> nid(Ra * (size_t)W);
        std::vector<int4> cells(Ra * (size_t)W);
        std::vector<Chunk> chunks;
        const double rl = std::max(std::max(fp.d, fp.c), sd.gp.rcut) + kSkin;
        const double rlc = std::max(fpc.d, fpc.c) + kSkin;
        Chunk cur{};
        auto close_chunk = [&](int e_end) {
            if (cur.ne == 0) return;
            chunks.push_back(cur);
            (void)e_end;
            cur = Chunk{};
        };
        std::vector<int> chunk_first_off;  // start of each chunk's relative offsets in eoff
        for (int k = 0; k < Ra; ++k) {
            const int r = act[k], Nr = off[r + 1] - off[r];
            const double *box = batch->box + 3 * r;
            SweepLaunch sw{};
            sw.N = Nr;
            for (int a = 0; a < 3; ++a) sw.box[a] = box[a];
            sw.fp = fpc;
            sw.skin = skin;
            sw.dt = lang->dt;
            sw.c1 = c1;
            sw.mass = lang->mass;
            sw.sig = std::sqrt((1.0 - c1 * c1) * lang->mass * kKB * lang->T_sys[r] / kMVV2E);
            sw.seed = lang->seed;
            sw.noise_id = (uint64_t)lang->noise_id_sys[r];
            sw.L = L;
            sw.delta_expl = delta_expl;
            int nc[3];
            for (int a = 0; a < 3; ++a) nc[a] = (int)std::floor(box[a] / (std::max(fpc.d, fpc.c) + skin));
            while ((long)nc[0] * nc[1] * nc[2] > 512) *std::max_element(nc, nc + 3) -= 1;
            if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) nc[0] = nc[1] = nc[2] = 0;
            sw.ncx = nc[0];
            sw.ncy = nc[1];
            sw.ncz = nc[2];
            sw.q_cur = q + off[r];
            sw.p_cur = p + off[r];
            sw.noise = nullptr;
            sw.mode = 0;
            sw.out = ctx->dr_out_init.p + 8 * (size_t)k;
            fill_sweep_args(sw, (size_t)Nt, (size_t)Nt, 3 * (size_t)Nt, tin.data() + ab * k);
            sw.mode = 1;
            sw.q_prev = ctx->dr_qprev.p + off[r];
            sw.p_prev = ctx->dr_pprev.p + off[r];
            sw.out = ctx->dr_out_it.p + 8 * (size_t)k;
            fill_sweep_args(sw, (size_t)Nt, (size_t)Nt, 3 * (size_t)Nt, tit.data() + ab * k);
            // entries of replica r: k W .. k W + W - 1
            int n3[3];
            for (int a = 0; a < 3; ++a) n3[a] = (int)std::floor(box[a] / std::max(rl, rlc));
            const bool use_cells = n3[0] >= 3 && n3[1] >= 3 && n3[2] >= 3 && Nr >= 500;
            for (int s2 = 0; s2 < W; ++s2) {
                const int e = k * W + s2;
                if (cur.ne > 0 && (long)cur.Nc + Nr > kMultiChunkAtoms) close_chunk(e);
                if (cur.ne == 0) {
                    cur.e0 = e;
                    chunk_first_off.push_back((int)eoff.size());
                    eoff.push_back(0);
                }
                cur.ne += 1;
                cur.Nc += Nr;
                eoff.push_back(cur.Nc);
                cur.bd.max_sys = std::max(cur.bd.max_sys, Nr);
                sig[e] = sw.sig;
                nid[e] = lang->noise_id_sys[r];
                for (int a = 0; a < 3; ++a) bx[3 * (size_t)e + a] = box[a];
                cells[e] = use_cells ? make_int4(n3[0], n3[1], n3[2], 0) : make_int4(0, 0, 0, 0);
                if (use_cells) cur.bd.n_cells += n3[0] * n3[1] * n3[2];
            }
        }
        close_chunk(Ra * W);
        if ((rc = upload(ctx, ctx->dr_act.p, act.data(), (size_t)Ra, st)) ||
            (rc = upload(ctx, ctx->dr_tab_init.p, tin.data(), tin.size(), st)) ||
            (rc = upload(ctx, ctx->dr_tab_it.p, tit.data(), tit.size(), st)) ||
            (rc = upload(ctx, ctx->dr_eoff.p, eoff.data(), eoff.size(), st)) ||
            (rc = upload(ctx, ctx->dr_sig.p, sig.data(), sig.size(), st)) ||
            (rc = upload(ctx, ctx->dr_sb.p, sb.data(), sb.size(), st)) ||
            (rc = upload(ctx, ctx->dr_noise.p, nid.data(), nid.size(), st)) ||
            (rc = upload(ctx, ctx->dr_box.p, bx.data(), bx.size(), st)) ||
            (rc = upload(ctx, ctx->dr_cells.p, cells.data(), cells.size(), st)))
            return rc;
        for (size_t c = 0; c < chunks.size(); ++c) {
            Chunk &ch = chunks[c];
            BatchDev &b = ch.bd;
            b.N = ch.Nc;
            b.n_sys = ch.ne;
            b.off = ctx->dr_eoff.p + chunk_first_off[c];
            b.box = ctx->dr_box.p + 3 * (size_t)ch.e0;
            b.cells = ctx->dr_cells.p + ch.e0;
            b.cells_given = 1;
            LangevinDev &l = ch.ld;
            l.dt = lang->dt;
            l.c1 = c1;
            l.mass = lang->mass;
            l.seed = lang->seed;
            l.sig = ctx->dr_sig.p + ch.e0;
            l.step0 = ctx->dr_step0.p + ch.e0;
            l.noise_id = ctx->dr_noise.p + ch.e0;
            l.scheme = SNAPMD_SCHEME_BAOAB;
            l.gamma = lang->gamma;
            l.sb0 = l.sb1 = ctx->dr_sb.p + ch.e0;
        }
        for (int it = 0; it < rounds_per_check && rounds < max_rounds; ++it, ++rounds) {
            launch_drv_start(Ra, ctx->dr_act.p, ctx->dr_st.p, N, W, ctx->dr_tab_init.p, ctx->dr_out_init.p, st);
            launch_coarse_sweep_multi(ctx->dr_tab_init.p, Ra, maxN, st);
            launch_drv_iter(Ra, ctx->dr_act.p, R, ctx->dr_st.p, W, L, (size_t)Nt, ctx->dr_roff.p, ctx->dr_ent.p,
                            ctx->dr_step0.p, ctx->dr_tab_it.p, ctx->dr_out_it.p, ctx->m_win.p, ctx->m_jq.p, ctx->m_jp.p,
                            st);
            launch_copy_windows(N + 1, Nt, R, ctx->dr_roff.p, ctx->m_win.p, q, p, ctx->dr_qprev.p, ctx->dr_pprev.p, st);
            for (const Chunk &ch : chunks) {
                const int4 *ent = ctx->dr_ent.p + ch.e0;
                launch_entries_to_batch(ch.Nc, ch.ne, ch.bd.off, ent, Nt, ctx->dr_qprev.p, ctx->pr_xf.p, st);
                launch_entries_to_batch(ch.Nc, ch.ne, ch.bd.off, ent, Nt, ctx->dr_pprev.p, ctx->pr_pf.p, st);
                HIPCHK(hipMemcpyAsync(ctx->pr_xc.p, ctx->pr_xf.p, 3 * (size_t)ch.Nc * sizeof(double),
                                      hipMemcpyDeviceToDevice, st));
                HIPCHK(hipMemcpyAsync(ctx->pr_pc.p, ctx->pr_pf.p, 3 * (size_t)ch.Nc * sizeof(double),
                                      hipMemcpyDeviceToDevice, st));
                if ((rc = run_langevin_prepared(ctx, ctx->w, ctx->d_f, SNAPMD_POT_FS_SNAP, ch.bd, fp, sd, ch.ld, L,
                                                ctx->pr_xf.p, ctx->pr_pf.p, st)) ||
                    (rc = run_langevin_prepared(ctx, ctx->wc, ctx->d_fc, SNAPMD_POT_FS, ch.bd, fpc, sdc, ch.ld, L,
                                                ctx->pr_xc.p, ctx->pr_pc.p, st)))
                    return rc;
                launch_batch_jumps_to_slots(ch.Nc, ch.ne, ch.bd.off, ent, Nt, ctx->pr_xf.p, ctx->pr_xc.p, ctx->m_jq.p,
                                            st);
                launch_batch_jumps_to_slots(ch.Nc, ch.ne, ch.bd.off, ent, Nt, ctx->pr_pf.p, ctx->pr_pc.p, ctx->m_jp.p,
                                            st);
            }
            launch_coarse_sweep_multi(ctx->dr_tab_it.p, Ra, maxN, st);
            launch_drv_update(Ra, ctx->dr_act.p, ctx->dr_st.p, ctx->dr_out_it.p, delta_conv, delta_expl, N, ML,
                              ctx->dr_logi.p, ctx->dr_logd.p, ctx->dr_err.p, st);
            if ((rc = check_launch(ctx))) return rc;
        }
        // check: the replicas' states (one synchronisation per rounds_per_check rounds)
        HIPCHK(hipMemcpyAsync(hs.data(), ctx->dr_st.p, (size_t)R * sizeof(DrvState), hipMemcpyDeviceToHost, st));
        if ((rc = snapmd_sync(ctx, stream))) return rc;
        ++checks;
        for (int r = 0; r < R; ++r) {
            if (hs[r].err & 1)
                return fail(ctx, SNAPMD_EOVERFLOW, "system %d: an atom of the coarse sweep has more than its list "
                                                   "capacity of neighbours", r);
            if (hs[r].err & 2)
                return fail(ctx, SNAPMD_ENONFINITE, "state of system %d became non-finite in slab %d", r,
                            hs[r].bad_slab);
        }
        act.clear();
        for (int r = 0; r < R; ++r)
            if (hs[r].phase != DRV_DONE) act.push_back(r);
        if (!act.empty() && rounds >= max_rounds)
            return fail(ctx, SNAPMD_EINVAL, "parareal_adaptive: %zu systems not converged after %d rounds",
                        act.size(), rounds);
    }
    // the iteration logs
    if (ML > 0) {
        std::vector<int4> li((size_t)R * ML);
        std::vector<double> ld((size_t)R * ML);
        HIPCHK(hipMemcpy(li.data(), ctx->dr_logi.p, li.size() * sizeof(int4), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(ld.data(), ctx->dr_logd.p, ld.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t q2 = 0; q2 < li.size(); ++q2) {
            log->n_in[q2] = li[q2].x;
            log->n_fi[q2] = li[q2].y;
            log->n_fi_after[q2] = li[q2].z;
            log->delta[q2] = ld[q2];
        }
    }
    for (int r = 0; r < R; ++r) log->n_log[r] = hs[r].nlog;
    *rounds_out = rounds;
    *checks_out = checks;
    return SNAPMD_OK;
}

int snapmd_ws_sites(snapmd_ctx *ctx, const snapmd_batch *batch, const double *x, double a, int32_t *site,
                    int32_t *occ, int32_t n_occ, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (!x || !site || !occ) return fail(ctx, SNAPMD_EINVAL, "x, site and occ must be device pointers");
    if (!(a > 0.0)) return fail(ctx, SNAPMD_EINVAL, "the lattice constant must be > 0 (got %g)", a);
    BatchDev bd;
    double mh;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    std::vector<int4> ws(batch->n_sys);
    long total = 0;
    for (int s = 0; s < batch->n_sys; ++s) {
        int n[3];
        for (int al = 0; al < 3; ++al) {
            const double c = batch->box[3 * s + al] / a;
            n[al] = (int)std::lround(c);
            if (n[al] < 1 || std::fabs(c - n[al]) > 1e-9 * c)
                return fail(ctx, SNAPMD_EINVAL, "box edge %d of system %d is not a whole number of cells of %g A",
                            al, s, a);
        }
        ws[s] = make_int4(n[0], n[1], n[2], (int)total);
        total += 2L * n[0] * n[1] * n[2];
    }
    if (total > n_occ) return fail(ctx, SNAPMD_EINVAL, "occ holds %d sites, the batch has %ld", n_occ, total);
    if ((rc = ensure(ctx, ctx->d_ws, (size_t)batch->n_sys))) return rc;
    if ((rc = upload(ctx, ctx->d_ws.p, ws.data(), ws.size(), st))) return rc;
    launch_ws_sites(bd, ctx->d_ws.p, (int)total, a, x, site, occ, st);
    return check_launch(ctx);
}

int snapmd_relax(snapmd_ctx *ctx, int potential, const snapmd_snap *snap, const snapmd_fs *fs,
                 const snapmd_batch *batch, double *x, int32_t max_iter, double ftol, double alpha, double dmax,
                 double *fmax_out, int32_t *iters_out, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (potential != SNAPMD_POT_FS && potential != SNAPMD_POT_FS_SNAP)
        return fail(ctx, SNAPMD_EINVAL, "potential must be SNAPMD_POT_FS or SNAPMD_POT_FS_SNAP");
    if (!x) return fail(ctx, SNAPMD_EINVAL, "x must be a device pointer");
    if (!fmax_out || !iters_out) return fail(ctx, SNAPMD_EINVAL, "fmax_out and iters_out must be host pointers");
    if (max_iter < 0 || !(ftol > 0.0) || !(alpha > 0.0) || !(dmax > 0.0))
        return fail(ctx, SNAPMD_EINVAL, "need max_iter >= 0 and ftol, alpha, dmax > 0");
    BatchDev bd;
    double mh;
    FsParams fp;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_fs(ctx, fs, mh, fp))) return rc;
    if (potential == SNAPMD_POT_FS_SNAP && (rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    if ((rc = ensure(ctx, ctx->d_fmax, 1))) return rc;
    if (!ctx->h_out) HIPCHK(hipHostMalloc((void **)&ctx->h_out, 16 * sizeof(double), hipHostMallocDefault));
    const int N = bd.N;
    int it = 0;
    double fmax = 0.0;
    for (;;) {
        enqueue_forces(ctx, ctx->w, potential, bd, x, &fp, &sd, ctx->d_f, st);
        if (it % 20 == 0 || it == max_iter) {
            launch_fmax2(N, ctx->d_f, ctx->d_fmax.p, st);
            HIPCHK(hipMemcpyAsync(ctx->h_out, ctx->d_fmax.p, sizeof(double), hipMemcpyDeviceToHost, st));
            if ((rc = snapmd_sync(ctx, stream))) return rc;
            fmax = std::sqrt(ctx->h_out[0]);
            if (!std::isfinite(fmax)) return fail(ctx, SNAPMD_ENONFINITE, "forces became non-finite at step %d", it);
            if (fmax < ftol || it == max_iter) break;
        }
        launch_descent_step(N, x, ctx->d_f, alpha, dmax, st);
        ++it;
    }
    *fmax_out = fmax;
    *iters_out = it;
    return check_launch(ctx);
}

int snapmd_set_coarse_snap(snapmd_ctx *ctx, const snapmd_snap *coarse) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (!coarse) {
        ctx->coarse_snap_on = false;
        ctx->coarse_beta.clear();
        return SNAPMD_OK;
    }
    const int J = coarse->twojmax;
    if (J < 2 || J > kMaxJ || (J & 1))
        return fail(ctx, SNAPMD_EUNSUPPORTED, "coarse twojmax must be one of 2, 4, ..., 14 (got %d)", J);
    if (coarse->n_coeff != snap_tables(J).K)
        return fail(ctx, SNAPMD_EINVAL, "coarse n_coeff must be %d for twojmax %d (got %d)", snap_tables(J).K, J,
                    coarse->n_coeff);
    if (!coarse->beta) return fail(ctx, SNAPMD_EINVAL, "coarse beta is NULL");
    ctx->coarse_snap = *coarse;
    ctx->coarse_beta.assign(coarse->beta, coarse->beta + coarse->n_coeff + 1);
    ctx->coarse_snap.beta = nullptr;
    ctx->coarse_snap_on = true;
    return SNAPMD_OK;
}

int snapmd_set_kernel_shape(snapmd_ctx *ctx, int32_t twojmax, const snapmd_kernel_shape *shape) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (twojmax < 2 || twojmax > kMaxJLds || (twojmax & 1))
        return fail(ctx, SNAPMD_EINVAL, "kernel shapes are chosen for twojmax 2, 4, 6 or 8 (got %d)", twojmax);
    if (!shape) {
        ctx->shapes.erase(twojmax);
        return SNAPMD_OK;
    }
    const bool ok = (shape->density_acc == 45 || shape->density_acc == 28 || shape->density_acc == 21) &&
                    (shape->dedr_stage_atoms == 5 || shape->dedr_stage_atoms == 3 || shape->dedr_stage_atoms == 0) &&
                    (shape->adjoint_waves == 12 || shape->adjoint_waves == 8) &&
                    (shape->density_parts >= 0 && shape->density_parts <= 2);
    if (!ok)
        return fail(ctx, SNAPMD_EINVAL, "kernel shape (%d, %d, %d, %d) is not one of the compiled variants",
                    shape->density_acc, shape->dedr_stage_atoms, shape->adjoint_waves, shape->density_parts);
    ctx->shapes[twojmax] =
        KernelShape{shape->density_acc, shape->dedr_stage_atoms, shape->adjoint_waves, shape->density_parts};
    return SNAPMD_OK;
}

int snapmd_get_kernel_shape(snapmd_ctx *ctx, int32_t twojmax, snapmd_kernel_shape *shape) {
    if (!ctx || !shape) return SNAPMD_EINVAL;
    auto it = ctx->shapes.find(twojmax);
    KernelShape k = it != ctx->shapes.end() ? it->second : KernelShape{};
    if (twojmax > kMaxJLds) k = KernelShape{45, 0, 12, 1};
    *shape = snapmd_kernel_shape{k.dens_acc, k.dedr_atoms, k.adj_waves, k.dens_parts};
    return SNAPMD_OK;
}

int snapmd_set_coarse_fs(snapmd_ctx *ctx, const snapmd_fs *coarse) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (!coarse) {
        ctx->coarse_fs_on = false;
        return SNAPMD_OK;
    }
    if (!(coarse->d > 0.0) || !(coarse->c > 0.0) || !std::isfinite(coarse->A) || !std::isfinite(coarse->c0) ||
        !std::isfinite(coarse->c1) || !std::isfinite(coarse->c2))
        return fail(ctx, SNAPMD_EINVAL, "coarse FS: need d, c > 0 and finite coefficients");
    ctx->coarse_fs = *coarse;
    ctx->coarse_fs_on = true;
    return SNAPMD_OK;
}

int snapmd_set_chunk_plan(snapmd_ctx *ctx, const int32_t *sizes, int32_t n) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (n < 0 || n > 64) return fail(ctx, SNAPMD_EINVAL, "chunk plan: need 0 <= n <= 64 (got %d)", n);
    if (n > 0 && !sizes) return fail(ctx, SNAPMD_EINVAL, "chunk plan: sizes is null");
    for (int c = 0; c < n; ++c)
        if (sizes[c] < 1) return fail(ctx, SNAPMD_EINVAL, "chunk plan: size %d of chunk %d", sizes[c], c);
    ctx->chunk_override.assign(sizes, sizes + n);
    return SNAPMD_OK;
}

int snapmd_set_sweep_workgroups(snapmd_ctx *ctx, int32_t K) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (K < 0 || K > 64) return fail(ctx, SNAPMD_EINVAL, "sweep workgroups: need 0 <= K <= 64 (got %d)", K);
    ctx->sweep_k_override = K;
    return SNAPMD_OK;
}

int snapmd_set_fine_streams(snapmd_ctx *ctx, int32_t n) {
    if (!ctx) return SNAPMD_EINVAL;
    if (const int rc_ = drain(ctx)) return rc_;
    if (n != 1 && n != 2) return fail(ctx, SNAPMD_EINVAL, "fine streams: need 1 or 2 (got %d)", n);
    ctx->fine_streams = n;
    return SNAPMD_OK;
}

int snapmd_sweep_workgroups(snapmd_ctx *ctx, int32_t N, int32_t *K) {
    if (!ctx || !K) return SNAPMD_EINVAL;
    const bool one_wg = ctx->sweep_k_override == 1 && sweep_fits_lds(N);
    *K = one_wg ? 1 : sweep_mc_workgroups(N, ctx->sweep_k_override);
    if (*K == 0 && sweep_fits_lds(N)) *K = 1;
    return SNAPMD_OK;
}

int snapmd_chunk_plan(snapmd_ctx *ctx, int32_t S, int32_t N, int32_t *sizes, int32_t *n) {
    if (!ctx) return SNAPMD_EINVAL;
    if (S < 1 || N < 1 || !sizes || !n) return fail(ctx, SNAPMD_EINVAL, "chunk plan: need S, N >= 1 and outputs");
    const std::vector<int> plan = window_plan(ctx, S, N);
    if (plan.size() > 64) return fail(ctx, SNAPMD_EINVAL, "chunk plan: more than 64 chunks");
    for (size_t c = 0; c < plan.size(); ++c) sizes[c] = plan[c];
    *n = (int32_t)plan.size();
    return SNAPMD_OK;
}

int snapmd_use_graphs(snapmd_ctx *ctx, int enable) {
    if (!ctx) return SNAPMD_EINVAL;
    ctx->use_graphs = enable ? 1 : 0;
    return SNAPMD_OK;
}

int snapmd_profile(snapmd_ctx *ctx, int enable) {
    if (!ctx) return SNAPMD_EINVAL;
    if (enable < 0) return fail(ctx, SNAPMD_EINVAL, "profile: need enable >= 0 (got %d)", enable);
    ctx->prof.enabled = enable ? 1 : 0;
    ctx->prof.stride = enable ? enable : 1;
    ctx->prof.reset();
    return SNAPMD_OK;
}

int snapmd_profile_read(snapmd_ctx *ctx, int kernel, double *total_ms, int64_t *launches) {
    if (!ctx || !total_ms || !launches) return SNAPMD_EINVAL;
    if (kernel < 0 || kernel >= PROF_N) return fail(ctx, SNAPMD_EINVAL, "unknown kernel id %d", kernel);
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    double tot = 0.0;
    int64_t n = 0;
    // a pair the runtime cannot time (hipEventElapsedTime fails) is left out of the sample
    for (size_t q = 0; q < ctx->prof.ids.size() && q < ctx->prof.ev1.size(); ++q) {
        if (ctx->prof.ids[q] != kernel) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->prof.ev0[q], ctx->prof.ev1[q]) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return SNAPMD_OK;
}

int snapmd_pair_count(snapmd_ctx *ctx, int64_t *n_pairs) {
    if (!ctx || !n_pairs) return SNAPMD_EINVAL;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    HIPCHK(hipDeviceSynchronize());
    int v = 0;
    if (ctx->cap_atoms && !ctx->h_off.empty()) {
        const int N = ctx->h_off.back();
        HIPCHK(hipMemcpy(&v, ctx->w.poff + N, sizeof(int), hipMemcpyDeviceToHost));
    }
    *n_pairs = v;
    return SNAPMD_OK;
}

int snap_beta_grad(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch, const double *x,
                   const double *w, double *dEdbeta, double *gradF, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (!x || !w || !dEdbeta || !gradF) return fail(ctx, SNAPMD_EINVAL, "x, w, dEdbeta and gradF must be device pointers");
    if (snap && snap->twojmax > kMaxJLds)
        return fail(ctx, SNAPMD_EUNSUPPORTED, "snap_beta_grad takes twojmax up to %d (got %d)", kMaxJLds, snap->twojmax);
    BatchDev bd;
    double mh;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    const int N = bd.N, K = sd.K;
    launch_set_value(dEdbeta, (double)N, st);
    launch_set_value(gradF, 0.0, st);
    if (N == 0) {
        HIPCHK(hipMemsetAsync(dEdbeta + 1, 0, K * sizeof(double), st));
        HIPCHK(hipMemsetAsync(gradF + 1, 0, K * sizeof(double), st));
        return check_launch(ctx);
    }
    if ((rc = ensure(ctx, ctx->gB, (size_t)K * N))) return rc;
    if ((rc = neighbors(ctx, ctx->w, bd, x, snap->rcut, true, st))) return rc;
    launch_snap_density(sd.J, bd, x, sd, ctx->w, st);           // u (and the pair geometry)
    launch_bispectrum(bd, sd, ctx->w, ctx->gB.p, st);           // B[k][i]
    launch_reduce_rows(K, N, ctx->gB.p, 1.0, dEdbeta + 1, st);
    launch_jvp_density(sd.J, N, ctx->w, w, sd.nrm, ctx->w.ytil, st);  // du along w
    launch_bispectrum_jvp(N, sd, ctx->w.u, ctx->w.ytil, ctx->gB.p, st);
    launch_reduce_rows(K, N, ctx->gB.p, -1.0, gradF + 1, st);
    return check_launch(ctx);
}

// Bispectrum of every atom, B[t][i] (device, [K][n_atoms]); used by tests and the
// coefficient gradient.
int snapmd_bispectrum(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch, const double *x,
                      double *B, void *stream) {
    if (!ctx) return SNAPMD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if (const int rc_ = drain(ctx)) return rc_;
    if (!x || !B) return fail(ctx, SNAPMD_EINVAL, "x and B must be device pointers");
    BatchDev bd;
    double mh;
    SnapDev sd;
    int rc;
    if ((rc = prepare_batch(ctx, batch, bd, mh, st))) return rc;
    if ((rc = prepare_snap(ctx, snap, mh, sd, st))) return rc;
    if (bd.N == 0) return SNAPMD_OK;
    if ((rc = neighbors(ctx, ctx->w, bd, x, snap->rcut, true, st))) return rc;
    launch_snap_density(sd.J, bd, x, sd, ctx->w, st);
    launch_bispectrum(bd, sd, ctx->w, B, st);
    return check_launch(ctx);
}

}  // extern "C"
