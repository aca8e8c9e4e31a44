// Device-side argument bundles and kernel launchers of snapmd (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace snapmd {

// Ragged batch resident on the device.
struct BatchDev {
    int N = 0;              // total atoms
    int n_sys = 0;
    const int *off = nullptr;     // [n_sys + 1]
    const double *box = nullptr;  // [3 * n_sys]
    const int4 *cells = nullptr;  // [n_sys] (nx, ny, nz, first cell); nx = 0: brute force
    int n_cells = 0;
    int max_sys = 0;              // atoms of the largest system
    int cells_given = 0;          // cells / n_cells set by the caller (no grid set-up from the context)
};

struct FsParams {
    double A, d, c, c0, c1, c2;
};

// Finnis-Sinclair terms folded into the SNAP passes of a propagation step (on = 0: SNAP
// alone): phi(r) is stored beside a, b, f_c per list slot, the density pass sums rho_i and
// writes dF[i] = F'(rho_i), and the gather adds the pair force of the FS energy.
struct FsFuse {
    FsParams fp;
    double *dF;
    int on;
};

struct SnapGeoParams {
    double rcut, rfac0, rmin0;
};

// Tables of the LDS-staged adjoint kernel (host copies, built per twojmax / beta).
struct AdjointHost {
    int J = -1;
    std::vector<double> cgm;       // row-pair motif coupling constants (beta free)
    std::vector<double> coef;      // beta~ * C^{j m}_{j1 m1, j2 m2} per (2m, block, m1, j)
    std::vector<int> coef_off;     // [(2J+1) * n_blocks] start of each (2m, block) run
    std::vector<int> roles;        // [12][role_len] output rows 2m of each wave (> J ends)
    int role_len = 0;
    std::vector<int> roles8;       // the same for 8 waves
    int role_len8 = 0;
    std::vector<double> beta;
    bool coef_changed = false;
};
struct AdjointDev {
    const double *cgm = nullptr, *coef = nullptr;
    const int *coef_off = nullptr, *roles = nullptr;
    int role_len = 0;
    const int *roles8 = nullptr;
    int role_len8 = 0;
};

// Kernel shapes of the SNAP passes (tuning choices; forces do not depend on them, energies
// only through the order of the adjoint's partial sums):
//   dens_acc   density pass: most accumulated elements per lane (45, 28 or 21)
//   dedr_atoms dE/dr: atoms whose Y~ rows a wave stages in LDS (5, 3 or 0: from memory)
//   adj_waves  LDS-tiled adjoint: waves per 64-atom tile (12 or 8)
//   dens_parts density pass of a force evaluation: waves over which a tile's neighbour
//              slots are split (1 or 2); part p writes u + p nh N, the adjoint adds them;
//              0: 2 for a launch with fewer density waves than the device has SIMDs
//              (one wave per SIMD leaves the pass latency-bound), else 1
// Above twojmax 8 the passes have one shape each (45, 0, -, 1).
struct KernelShape {
    int dens_acc = 45;
    int dedr_atoms = 0;
    int adj_waves = 12;
    int dens_parts = 0;
};

// SNAP coefficient-dependent tables on the device.
struct SnapDev {
    int J = 0, K = 0, nh = 0;
    int simds = 1024;  // SIMDs of the device (4 per CU): the automatic density split
    SnapGeoParams gp{};
    double beta0 = 0.0;
    const double *nrm = nullptr, *ymult = nullptr;
    const int *ystart = nullptr;
    const int *ychunk = nullptr;    // [n_ychunk + 1] output-element chunks of the coupling program
    int n_ychunk = 0;
    const uint32_t *yidx = nullptr;
    const double *ycoef = nullptr;  // CG product * beta tilde
    const int *bstart = nullptr, *bel = nullptr;
    const uint32_t *bidx = nullptr;
    const double *bcg = nullptr;
    AdjointDev adj;
    KernelShape shape;
};

struct LangevinDev {
    double dt, c1, mass;
    uint64_t seed;
    const double *sig = nullptr;       // [n_sys] sqrt((1 - c1^2) m kB T / mvv2e)
    const int64_t *step0 = nullptr;    // [n_sys]
    const int *noise_id = nullptr;     // [n_sys]
    int scheme = 0;                    // 0 BAOAB, 1 the paper's modified BBK
    double gamma = 0.0;
    const double *sb0 = nullptr;       // [n_sys] BBK noise amplitude of G_0: (1/2) sqrt(2 gamma m kB C_0 T dt / mvv2e)
    const double *sb1 = nullptr;       // [n_sys] the same with C_l (l >= 1)
};

// Per-evaluation scratch (owned by the context).
struct Work {
    size_t Pcap = 0;        // pair capacity (N * kMaxNeigh)
    int *nbr = nullptr, *cnt = nullptr, *poff = nullptr, *pair_i = nullptr, *pair_j = nullptr, *rev = nullptr;
    int *status = nullptr;  // device error bits: 1 neighbour overflow, 4 asymmetric list
    int *flag = nullptr;    // rebuild request of the Verlet list
    int *cell_of = nullptr, *cell_cnt = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *cell_atoms = nullptr;
    size_t cap_cells = 0;
    double *xref = nullptr; // [3][N] positions at the last build
    double *rho = nullptr;
    double *geo = nullptr;  // [20][Pcap]
    double *ell = nullptr;  // [6][kMaxNeigh][N] a, b, f_c (and the FS phi) by (list slot, atom)
    int *nbr_t = nullptr;   // [kMaxNeigh][N] neighbour j by (list slot, atom)
    double *ph = nullptr;   // [3][N] BBK: p_{l-1/2} of the running call
    double *dedr = nullptr; // [3][Pcap]
    double2 *u = nullptr, *ytil = nullptr;  // [nh][N]
    double *epart = nullptr;                // [kMaxYChunks][N] energy parts of the chunked adjoint
};
constexpr int kMaxYChunks = 64;

// Optional per-kernel timing with HIP events on the launch stream (for the roofline).
enum { PROF_DEDR = 0, PROF_ADJOINT = 1, PROF_DENSITY = 2, PROF_NEIGH = 3, PROF_N = 4 };
// HIP events around a sample of the launches: every stride-th launch of each kernel id
// (an event record leaves the device idle for a few microseconds, so recording around
// every launch would slow the run being measured).
struct KernelProf {
    int enabled = 0;
    int stride = 1;
    long long calls[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool open = false;
    // nonzero on a thread that must not record (graph capture, or a thread launching
    // beside the one being timed)
    static inline thread_local int suppress = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> ids;
    std::vector<hipEvent_t> ev0, ev1;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int id, hipStream_t st) {
        if (!enabled || suppress) return;
        if (calls[id & 7]++ % stride != 0) return;
        hipEvent_t e = get();
        (void)hipEventRecord(e, st);
        ids.push_back(id);
        ev0.push_back(e);
        open = true;
    }
    void end(hipStream_t st) {
        if (!open) return;
        open = false;
        hipEvent_t e = get();
        (void)hipEventRecord(e, st);
        ev1.push_back(e);
    }
    void reset() {
        open = false;
        for (long long &c : calls) c = 0;
        used = 0;
        ids.clear();
        ev0.clear();
        ev1.clear();
    }
};

// Arguments of the persistent coarse sweep of a parareal iteration.
struct SweepLaunch {
    int N;
    double box[3];
    FsParams fp;
    double skin;
    double dt, c1, mass, sig;
    uint64_t seed, noise_id;
    int L, n_in, n_fi, mode, n_win;
    int ncx, ncy, ncz;  // cell grid of the sweep's list build (0: all pairs)
    int K, A;           // multi-workgroup sweep: K workgroups of A atoms (K = 0: one workgroup)
    unsigned long long *gx, *gdfe, *gpart;  // exchange words: 12 N, 4 N and 16 K, zeroed before launch
    int *abort;
    double delta_expl;
    double *q_cur, *p_cur;
    const double *q_prev, *p_prev, *jq, *jp;
    double *out;
    const double *noise;  // [S][L][3][N], S = n_fi - n_in
};
void launch_slabs_to_batch(int S, int N, const double *slots, double *out, hipStream_t st);
void launch_jumps(size_t n, double *a, const double *b, hipStream_t st);
void launch_coarse_sweep(const SweepLaunch &s, hipStream_t st);
void sweep_init_attributes();
void neigh_init_attributes();
bool sweep_fits_lds(int N);
int sweep_mc_workgroups(int N, int want = 0);
void launch_slab_end(int N, int mode, size_t jsa, size_t jss, size_t s, double *xs, double *ps, const double *jq,
                     const double *jp, size_t ld, const double *qprev_next, double *qcur_next, double *pcur_next,
                     double *part, hipStream_t st);
// batches of systems with windows of their own (slot layout [slot][3][ld])
void launch_copy_windows(int n_slots, int ld, int n_sys, const int *off, const int2 *win, const double *q,
                         const double *p, double *qd, double *pd, hipStream_t st);
void launch_entries_to_batch(int Nc, int n_ent, const int *off, const int4 *src, int ld, const double *state,
                             double *out, hipStream_t st);
void launch_batch_jumps_to_slots(int Nc, int n_ent, const int *off, const int4 *src, int ld, const double *f,
                                 const double *c, double *jump, hipStream_t st);
// device-resident adaptive driver: per-replica state of the adaptive algorithm
enum { DRV_NEW = 0, DRV_ITER = 1, DRV_DONE = 2 };
struct DrvState {
    int phase, n_in, n_fi, nlog;
    double delta;
    int err, bad_slab;
};
void launch_drv_start(int Ra, const int *act, DrvState *st, int N, int W, void *tab, double *out, hipStream_t s);
void launch_drv_iter(int Ra, const int *act, int R_all, const DrvState *st, int W, int L, size_t ld, const int *roff,
                     int4 *ent, int64_t *step0, void *tab, double *out, int2 *win, const double *jq, const double *jp,
                     hipStream_t s);
void launch_drv_update(int Ra, const int *act, DrvState *st, const double *out, double dconv, double dexpl, int N,
                       int max_log, int4 *logi, double *logd, int *err, hipStream_t s);
// the sweep arguments of one system of a batch, in the layout the multi-system sweep reads
size_t sweep_args_bytes();
void fill_sweep_args(const SweepLaunch &s, size_t ld, size_t jsa, size_t jss, void *dst);
void launch_coarse_sweep_multi(const void *tab, int n, int max_atoms, hipStream_t st);
void launch_noise_table(int S, int L, int N, int n_in, uint64_t seed, uint64_t noise_id, double *noise,
                        hipStream_t st);

// force: rebuild now; checked: the displacement test was done by k_baoab_pre (else a
// check kernel runs); clear_in_fs: the rebuild flag is cleared by the next k_fs_rho
// (launch_fs with clear_flag) instead of a kernel of its own
void launch_neighbors(const BatchDev &bd, const double *x, double rc, Work &w, hipStream_t st, bool force,
                      double skin, bool checked = false, bool clear_in_fs = false);
// p_kick (nullable): momenta that receive the closing half kick p += (dt/2) f of a BAOAB
// step from the force pass
void launch_fs(const BatchDev &bd, const double *x, const FsParams &fp, Work &w, double *f, double *e_atom,
               int accumulate, hipStream_t st, bool clear_flag = false, double *p_kick = nullptr, double dt = 0.0);
// join (nullable): an event the gather waits for (the Finnis-Sinclair force written into f
// on another stream); p_kick (nullable): momenta that receive the closing half kick
// p += (dt/2) f of a BAOAB step from the gather
// analysis.hip
void launch_ws_sites(const BatchDev &bd, const int4 *ws, int n_sites, double a, const double *x, int *site,
                     int *occ, hipStream_t st);
void launch_descent_step(int N, double *x, const double *f, double alpha, double dmax, hipStream_t st);
void launch_fmax2(int N, const double *f, unsigned long long *out, hipStream_t st);

// The opening B A O A of the next BAOAB step, done by the gather after the closing kick
// (open_step < 0: none): x and p of the batch, the Langevin parameters, the step index and
// the Verlet-list displacement test of k_baoab_pre.
struct StepOpen {
    int open_step = -1;
    double *x = nullptr;
    LangevinDev ld{};
    const int *off = nullptr;
    int n_sys = 0;
    const double *xref = nullptr;
    double lim2 = 0.0;
    int *flag = nullptr;
};
void launch_snap(int J, const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, double *f,
                 double *e_atom, int accumulate, hipStream_t st, KernelProf *prof = nullptr,
                 hipEvent_t join = nullptr, double *p_kick = nullptr, double dt = 0.0, const FsParams *fuse = nullptr,
                 const StepOpen *open = nullptr);
void launch_snap_density(int J, const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, hipStream_t st);
void adjoint_tables(int J, const double *beta, AdjointHost &A);
void adjoint_init_attributes();
// u2: the second part of the density (null: u is whole)
void launch_adjoint(int J, const AdjointDev &ad, int N, const double2 *u, const double2 *u2, const double *nrm,
                    const double *ymult, double beta0, double2 *ytil, double *e_atom, int accumulate, hipStream_t st,
                    int waves = 12);
void launch_bispectrum(const BatchDev &bd, const SnapDev &sd, Work &w, double *B, hipStream_t st);
void launch_jvp_density(int J, int N, const Work &w, const double *wf, const double *nrm, double2 *du,
                        hipStream_t st);
void launch_bispectrum_jvp(int N, const SnapDev &sd, const double2 *u, const double2 *du, double *dB,
                           hipStream_t st);
void launch_reduce_rows(int rows, int N, const double *in, double scale, double *out, hipStream_t st);
void launch_set_value(double *p, double v, hipStream_t st);
void launch_baoab_pre(const BatchDev &bd, double *x, double *p, const double *f, const LangevinDev &ld, int s_step,
                      const Work &w, double skin, hipStream_t st);
void launch_bbk_pre(const BatchDev &bd, double *x, double *p, const double *f, const LangevinDev &ld, int s_step,
                    const Work &w, double skin, hipStream_t st);
void launch_add_i64(int n, int64_t *v, int64_t delta, hipStream_t st);
// s1 = l + 1 (1 .. n_steps)
void launch_bbk_post(const BatchDev &bd, double *p, const double *f, const LangevinDev &ld, int s1, int n_steps,
                     hipStream_t st);

}  // namespace snapmd
