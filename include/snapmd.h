/*
 * snapmd -- batched SNAP + Finnis-Sinclair Langevin propagation for adaptive parareal,
 * hand-written HIP for MI355X (gfx950), FP64 throughout.
 *
 * The method (Gorynina, Legoll, Lelievre, Perez, "Combining machine-learned and
 * empirical force fields with the parareal algorithm") integrates the Langevin
 * equation of its "Algorithm" section with a fine propagator F (L steps on the
 * fine potential) and a coarse propagator C (L steps on the coarse potential) that
 * share their Gaussian increments, and corrects a coarse sweep with the jumps
 * F - C ("Parareal method", "Adaptive parareal method").  This library provides:
 *
 *   snap_forces       SNAP forces (fine potential of the "MD settings" section)
 *   eam_forces        Finnis-Sinclair EAM forces (coarse potential)
 *   langevin_steps    BAOAB Langevin steps for a ragged batch of systems
 *   parareal_iterate  one corrected iteration of adaptive parareal, every system on
 *                     a window of its own
 *   parareal_adaptive the whole adaptive algorithm for many replicas, decided on the device
 *   snap_beta_grad    dE/dbeta and d(force loss)/dbeta (SNAP coefficient gradients)
 *
 * Conventions (every entry point):
 *   - Units: metal (A, ps, eV, amu, K).  Momenta are p = m v (amu A / ps).
 *   - Per-atom arrays are DEVICE pointers, SoA: x[3][n_atoms] (x row, y row, z row),
 *     likewise p and f.  Positions may be unwrapped; periodic boundaries are applied
 *     by minimum image in each system's orthorhombic box.
 *   - Parameter structs and the batch descriptor hold small HOST arrays; they are
 *     copied (and validated) at each call, and need not outlive it.
 *   - The caller owns every array it passes; the library never frees or retains a
 *     caller pointer past the call.  The library owns its context workspace.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and is
 *     asynchronous, except where a function says it synchronises.
 *   - Return value: SNAPMD_OK (0) or a negative SNAPMD_E* code; snapmd_last_error()
 *     then describes the failure.  No C++ exception crosses this boundary.
 *     Errors detected on the device (neighbour overflow, non-finite state) are
 *     latched in the context and reported by the next synchronising call
 *     (parareal_iterate, snapmd_sync).
 *   - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef SNAPMD_H
#define SNAPMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snapmd_ctx snapmd_ctx;

enum {
    SNAPMD_OK = 0,
    SNAPMD_EINVAL = -1,       /* invalid argument (message names it)            */
    SNAPMD_ENOMEM = -2,       /* device allocation failed                       */
    SNAPMD_EHIP = -3,         /* HIP runtime error                              */
    SNAPMD_EUNSUPPORTED = -4, /* twojmax outside {2, ..., 14}, or a feature's limit */
    SNAPMD_ENONFINITE = -5,   /* NaN/Inf in a propagated state (message: slab)  */
    SNAPMD_EOVERFLOW = -6     /* an atom has more than SNAPMD_MAX_NEIGH neighbours */
};

#define SNAPMD_MAX_NEIGH 64   /* neighbours per atom within the cutoff           */
#define SNAPMD_ACCUMULATE 1u  /* flags: add into f / e_atom instead of overwriting */

/* Create a context on HIP device `hip_device`.  Returns SNAPMD_OK and *out, or an
 * error (then *out is NULL). */
int snapmd_create(snapmd_ctx **out, int hip_device);
/* Release the context and its device workspace (NULL is a no-op). */
void snapmd_destroy(snapmd_ctx *ctx);
/* Message of the last error on this context ("" if none).  Owned by the context. */
const char *snapmd_last_error(const snapmd_ctx *ctx);
/* Synchronise `stream` and report any error latched by device-side checks. */
int snapmd_sync(snapmd_ctx *ctx, void *stream);

/* Ragged batch of independent periodic systems stored back to back.
 * offset[s] .. offset[s+1]-1 are the atoms of system s (offset[0] = 0,
 * nondecreasing); box[3*s + 0..2] are its orthorhombic edges. */
typedef struct {
    int32_t n_sys;
    const int32_t *offset; /* host [n_sys + 1] */
    const double *box;     /* host [3 * n_sys] */
} snapmd_batch;

/* SNAP (spectral neighbour analysis potential; the paper's fine force field,
 * "MD settings" section, defined by Thompson et al.):
 *   E_i = beta[0] + sum_k beta[k] B_k(i),  k over the canonical (j1, j2, j) triples
 *   0 <= 2j2 <= 2j1 <= 2j <= twojmax (lexicographic order), B_k the bispectrum of
 *   the neighbour density of atom i within rcut (switching function
 *   (cos(pi (r - rmin0)/(rcut - rmin0)) + 1)/2, self term and unit weights).
 * Requirements: twojmax in {2, 4, ..., 14} (14: the paper's SNAP-205 size); n_coeff =
 * number of canonical triples (5, 14, 30, 55, 91, 140, 204); 0 < rfac0 < 1;
 * 0 <= rmin0 < rcut; rcut < min(box)/2.  Above twojmax 8 the adjoint pass reads the
 * densities from device memory (a 64-atom tile no longer fits the local memory), so the
 * cost per atom grows faster than the operation count; snap_beta_grad and
 * snap_forces_noalloc take twojmax <= 8. */
typedef struct {
    int32_t twojmax;
    double rcut, rfac0, rmin0;
    int32_t n_coeff;
    const double *beta; /* host [n_coeff + 1]; beta[0] = constant term */
} snapmd_snap;

/* Finnis-Sinclair EAM (the coarse potential; the paper's EAM of its "MD settings"
 * section is replaced by this tungsten parameterisation):
 *   E = sum_i [ -A sqrt(rho_i) + 1/2 sum_j V(r_ij) ],  rho_i = sum_j phi(r_ij),
 *   phi(r) = (r - d)^2 for r < d,  V(r) = (r - c)^2 (c0 + c1 r + c2 r^2) for r < c.
 * Requirements: d > 0, c > 0, max(d, c) < min(box)/2. */
typedef struct {
    double A, d, c, c0, c1, c2;
} snapmd_fs;

/* Langevin integration (the equation of the paper's "Algorithm" section with masses:
 * dq = p/m dt, dp = -grad V dt - gamma p dt + sqrt(2 gamma m kB T) dW), one force
 * evaluation per step, by one of two schemes:
 *
 * SNAPMD_SCHEME_BAOAB: half kick, half drift, exact Ornstein-Uhlenbeck step, half
 *   drift, force, half kick.  The Gaussian increment of atom i (local index within its
 *   system) at global step n is drawn from Philox4x64-10 with key (seed, 0) and counter
 *   (noise_id[s], n, i, 0) through Box-Muller, so a fine and a coarse run of the same
 *   slab see identical noise (paper, "Parareal method").  Splitting a run into several
 *   calls gives the same trajectory.
 *
 * SNAPMD_SCHEME_BBK: the paper's modified BBK scheme (eq:scheme_debut, eq:scheme) with
 *   the temperature schedule of eq:scheme_corrected_debut / eq:scheme_corrected.  ONE
 *   call is one application of L = n_steps iterates: iterate 0 uses p_0 in place of
 *   p_{-1/2}; the Gaussians G_0 .. G_L of the call are drawn with counters
 *   (noise_id[s], step0 + l, i, 1) for l < L and (noise_id[s], step0 + L, i, 2) for G_L
 *   (so G_L of one call and G_0 of the call starting at step0 + L differ), G_l with
 *   temperature C_l T: C_0 = bbk_c0, C_l = bbk_c1 for l >= 1.  bbk_c0 = bbk_c1 = 1 is
 *   the uncorrected scheme, (3, 1) the schedule valid for every L (eq:robust), (2, 2)
 *   the one for L = 1 (eq:choix_L_egal_1).  Unlike BAOAB, two calls of L/2 steps are
 *   not one call of L steps (the first iterate differs; the paper's point). */
enum { SNAPMD_SCHEME_BAOAB = 0, SNAPMD_SCHEME_BBK = 1 };

typedef struct {
    double dt;                     /* ps, > 0                           */
    double gamma;                  /* 1/ps, >= 0                        */
    double mass;                   /* amu, > 0 (one species)            */
    const double *T_sys;           /* host [n_sys] temperatures, K >= 0 */
    uint64_t seed;
    const int64_t *step0_sys;      /* host [n_sys] global step of the first step */
    const int32_t *noise_id_sys;   /* host [n_sys] noise stream ids (>= 0)       */
    int32_t scheme;                /* SNAPMD_SCHEME_BAOAB or SNAPMD_SCHEME_BBK   */
    double bbk_c0;                 /* BBK: temperature factor C_0 of G_0 (> 0)   */
    double bbk_c1;                 /* BBK: temperature factor C_l, l >= 1 (> 0)  */
} snapmd_langevin;

enum { SNAPMD_POT_FS = 0, SNAPMD_POT_FS_SNAP = 1 };

/* SNAP forces of every system of the batch.
 * x: device [3][n_atoms] positions.  f: device [3][n_atoms] forces (eV/A), overwritten
 * (or added to with SNAPMD_ACCUMULATE).  e_atom: device [n_atoms] SNAP energies (eV)
 * or NULL.  Asynchronous on `stream`. */
int snap_forces(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch,
                const double *x, double *f, double *e_atom, uint32_t flags, void *stream);

/* Allocation-free variant of snap_forces, for callers that cannot allocate device memory
 * (work captured into a graph, tight serving loops, harnesses that forbid allocation).
 * Same arguments and asynchrony as snap_forces; it runs the kernel shape (45, 0, 12, 1)
 * whatever shape the context holds, so its results are bitwise those of snap_forces in
 * that shape and equal to rounding otherwise.  Every buffer its kernels use
 * besides x, f and e_atom (neighbour lists, pair tables, SNAP densities and adjoints, the
 * batch description, the coefficient tables) lives in one fixed device array of
 * SNAPMD_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends (its address on a device is taken when a context is first created there);
 * the call allocates nothing.  Limits: at most SNAPMD_NOALLOC_MAX_ATOMS atoms and
 * SNAPMD_NOALLOC_MAX_SYS systems per call, else SNAPMD_EINVAL with a message (larger
 * batches: snap_forces).  The array keeps the last call's contents; nothing in it has to
 * start at zero.  All calls on one GPU share the array: calls that overlap on one GPU (on
 * other streams, contexts or threads) race, and the caller must serialise them.  A
 * neighbour overflow is latched in the context like snap_forces' and reported by the next
 * snapmd_sync. */
#define SNAPMD_NOALLOC_MAX_ATOMS 2048
#define SNAPMD_NOALLOC_MAX_SYS 256
#define SNAPMD_NOALLOC_SCRATCH_BYTES (24u << 20) /* 24 MiB */
int snap_forces_noalloc(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch,
                        const double *x, double *f, double *e_atom, uint32_t flags, void *stream);

/* Finnis-Sinclair forces of every system (same layout and flags as snap_forces). */
int eam_forces(snapmd_ctx *ctx, const snapmd_fs *fs, const snapmd_batch *batch, const double *x,
               double *f, double *e_atom, uint32_t flags, void *stream);

/* Advance every system of the batch by n_steps BAOAB steps in place.
 * potential: SNAPMD_POT_FS (coarse: FS only; snap may be NULL) or SNAPMD_POT_FS_SNAP
 * (fine: FS + SNAP).  The force is evaluated from x at the start (the propagators of
 * the paper's "Parareal method" section restart at every slab).  x, p: device
 * [3][n_atoms], updated.  f_out: device [3][n_atoms] force at the final positions,
 * or NULL.  Asynchronous on `stream`. */
int langevin_steps(snapmd_ctx *ctx, int potential, const snapmd_snap *snap, const snapmd_fs *fs,
                   const snapmd_batch *batch, const snapmd_langevin *lang, int32_t n_steps,
                   double *x, double *p, double *f_out, void *stream);

/* One corrected iteration of (adaptive) parareal ("Adaptive parareal method": the body
 * of the inner while loop of its Algorithm "Adaptive parareal algorithm", equation
 * eq:parareal) for EVERY system r of the batch, each on its own window
 * [n_in[r], n_fi[r]] of slabs:
 *   prev_n := cur_n for n_in <= n <= n_fi;
 *   J_n := F(prev_n) - C(prev_n) for n_in <= n < n_fi, all slabs of all systems at once;
 *   for n = n_in .. n_fi - 1:  cur_{n+1} := C(cur_n) + J_n;
 *       delta := sum_{m=n_in+1}^{n+1} |cur_m - prev_m| / sum_{m=n_in+1}^{n+1} |prev_m|
 *       (Euclidean norms of the 3 n_atoms position vector of the system; the sums start
 *       after the window's first slab, so that at n_in = 0 this is def:rel-Err);
 *       if delta > delta_expl: n_fi := max(n, n_in + 1); stop.
 * Slab n of system r covers global steps n*L .. n*L + L - 1 of noise stream
 * lang->noise_id_sys[r] at temperature lang->T_sys[r] (lang->step0_sys is ignored).
 * State layout: q_cur, p_cur, q_prev, p_prev are device [n_slots][3][n_atoms] (n_atoms =
 * offset[n_sys]); slot n holds every system's state at slab boundary n, system r in
 * columns offset[r] .. offset[r+1]-1 of each row.  cur is read on [n_in[r], n_fi[r]] and
 * written on (n_in[r], n_fi[r]]; prev receives cur on [n_in[r], n_fi[r]]; nothing else
 * is touched.
 * n_in: host [n_sys]; n_fi: host [n_sys], updated; delta_out: host [n_sys], receives
 * delta.  Need 0 <= n_in[r] <= n_fi[r] <= n_slots - 1; with more than one system an
 * empty window (n_in[r] = n_fi[r]) leaves system r out (delta_out[r] = 0), with one
 * system the window must not be empty.
 * delta_expl = +inf gives the classical algorithm.  Synchronises `stream` once (plus once
 * per slab of a sweep driven from the host); returns SNAPMD_ENONFINITE if a state became
 * non-finite (the message names the system and the slab).
 * Initialisation of new time windows (the coarse propagation that starts each window of
 * the adaptive algorithm): pass q_prev = p_prev = NULL; then only cur_{n+1} := C(cur_n)
 * for n_in[r] <= n < n_fi[r] is done, delta_out = 0, snap may be NULL.
 * The coarse sweep keeps a Verlet list with a 0.5 A skin and stores each listed pair's
 * periodic image: max(d, c) + 1.0 must be below half the smallest box edge.
 * Schedules: one system runs the pipelined path (slab chunks of the fine propagation
 * overlapping the on-device sweep); several systems run their fine and coarse
 * propagations as ragged batches of (system, slab) entries, then the sweeps of all
 * systems of at most ~1,500 atoms in one launch (one workgroup each), larger ones from
 * the host.  With SNAPMD_SCHEME_BBK, or a SNAP coarse potential, every sweep runs slab by
 * slab from the host (one small synchronisation per slab) instead of in one persistent
 * kernel.  Results do not depend on the schedule beyond the rounding of the relative
 * error's partial sums. */
int parareal_iterate(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs,
                     const snapmd_batch *batch, const snapmd_langevin *lang, int32_t L,
                     const int32_t *n_in, int32_t *n_fi, int32_t n_slots, double *q_prev,
                     double *p_prev, double *q_cur, double *p_cur, double delta_expl,
                     double *delta_out, void *stream);

/* Pipelined corrected iterations of one system ("Parareal method": iterations of
 * eq:parareal run back to back).  parareal_iterate_async does what parareal_iterate does
 * for a batch of one system with the window [n_in, n_fi], but returns once the work is
 * enqueued on `stream`; snapmd_parareal_collect returns the results of the iterations in
 * the order they were enqueued: delta_out and n_fi_out (host) as parareal_iterate's
 * delta_out[0] and n_fi[0], and the status codes parareal_iterate would return (an error
 * found while enqueueing is returned by parareal_iterate_async itself).  At most 3
 * iterations may wait to be collected (SNAPMD_EINVAL beyond).
 * Overlap: a corrected iteration that follows a pipelined one with the same window,
 * state buffers, box, potentials, Langevin parameters, slab chunks, sweep width and
 * stream copies prev := cur chunk by chunk, each as soon as the previous iteration's
 * on-device sweep has passed that chunk, so its fine propagation starts while the
 * previous sweep finishes its last chunks.  The results are bitwise those of the same
 * parareal_iterate calls.  cur and prev of an iteration are complete when its result has
 * been collected (the collect makes `stream` wait for them).  Any other call (another
 * window, parameter set or stream, and every other entry point of the library except the
 * getters, snapmd_profile, snapmd_use_graphs and snapmd_parareal_collect) first waits on
 * the host for the pipelined iterations in flight; their results stay queued.  Window
 * initialisations and sweeps driven from the host are not pipelined: they complete at the
 * call and queue their result.  The caller owns the speculation: an iteration enqueued
 * before the previous result was collected used the window given at its call. */
int parareal_iterate_async(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs,
                           const snapmd_batch *batch, const snapmd_langevin *lang, int32_t L, int32_t n_in,
                           int32_t n_fi, int32_t n_slots, double *q_prev, double *p_prev, double *q_cur,
                           double *p_cur, double delta_expl, void *stream);
int snapmd_parareal_collect(snapmd_ctx *ctx, double *delta_out, int32_t *n_fi_out, void *stream);

/* Iteration log of parareal_adaptive (host arrays owned by the caller): entry t of system
 * r (index r * max_log + t) describes its t-th corrected iteration: the window
 * [n_in, n_fi] it ran on, the window end after it (shorter when the relative error passed
 * delta_expl) and the relative error delta at its end.  n_log[r] receives the number of
 * iterations of system r (entries beyond max_log are counted but not stored). */
typedef struct {
    int32_t max_log;
    int32_t *n_log;                         /* host [n_sys]            */
    int32_t *n_in, *n_fi, *n_fi_after;      /* host [n_sys * max_log]  */
    double *delta;                          /* host [n_sys * max_log]  */
} snapmd_parareal_log;

/* The whole adaptive parareal algorithm ("Adaptive parareal method", Algorithm "Adaptive
 * parareal algorithm") for every system of the batch at once, with its branch logic and
 * window bookkeeping on the device: each system r runs the algorithm on its own sequence
 * of windows (tentative window [n_in, min(N, n_in + max_window)], initialised by a coarse
 * sweep, corrected until delta < delta_conv, shortened when delta > delta_expl, as
 * parareal_iterate does one iteration) over N slabs of L steps, with noise stream
 * lang->noise_id_sys[r] at temperature lang->T_sys[r].
 * q, p: device [N+1][3][n_atoms] (the slot layout of parareal_iterate); slot 0 holds the
 * initial states on entry; on return every slot holds the converged trajectory.
 * The call enqueues rounds of one fixed launch sequence (start of new windows,
 * initialisation sweeps, the corrected iteration of every running system with max_window
 * slabs per system in the batched propagation (slabs beyond a shortened window are
 * propagated and discarded, keeping the launch shapes fixed), the sweeps, the
 * algorithm's decisions) and synchronises only every rounds_per_check rounds to see which
 * systems are done (those leave the batch) and to report errors; it returns when every
 * system has reached slab N, or fails after max_rounds rounds.  *rounds_out and
 * *checks_out receive the rounds enqueued and the synchronisations made.
 * Needs BAOAB, a Finnis-Sinclair coarse potential (snapmd_set_coarse_fs applies) and
 * systems that fit the on-device sweep (else SNAPMD_EUNSUPPORTED); 0 <= delta_conv <
 * delta_expl < inf.  Errors: SNAPMD_EINVAL, SNAPMD_ENONFINITE (names the system and
 * slab), SNAPMD_EOVERFLOW. */
int parareal_adaptive(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_fs *fs,
                      const snapmd_batch *batch, const snapmd_langevin *lang, int32_t L, int32_t N,
                      int32_t max_window, double delta_conv, double delta_expl,
                      int32_t rounds_per_check, int32_t max_rounds, double *q, double *p,
                      snapmd_parareal_log *log, int32_t *rounds_out, int32_t *checks_out,
                      void *stream);

/* Coarse propagator of parareal_iterate.  By default it is Finnis-Sinclair alone (the
 * paper's strategy II: an EAM coarse potential).  snapmd_set_coarse_snap(ctx, coarse)
 * makes it Finnis-Sinclair + the SNAP model `coarse`, a low-twojmax SNAP beside the
 * fine one: the paper's strategy I (section "Numerical results", SNAP-6 as the coarse
 * potential for a larger SNAP fine one).  coarse is copied (beta included);
 * coarse = NULL restores Finnis-Sinclair alone.  Its twojmax must be in {2, 4, ..., 14},
 * n_coeff must match, and parareal_iterate refuses (SNAPMD_EINVAL) a coarse twojmax equal
 * to the fine one.  With a SNAP coarse potential the coarse propagation of the slabs is
 * batched like the fine one, and the sequential sweep is driven from the host (one
 * launch sequence and one small synchronisation per slab).  Errors: SNAPMD_EINVAL,
 * SNAPMD_EUNSUPPORTED. */
int snapmd_set_coarse_snap(snapmd_ctx *ctx, const snapmd_snap *coarse);

/* Finnis-Sinclair parameters of the coarse propagator of parareal_iterate.  By default the
 * coarse propagator uses the `fs` passed to parareal_iterate, which is also the
 * Finnis-Sinclair part of the fine potential.  snapmd_set_coarse_fs(ctx, coarse) gives the
 * coarse propagator parameters of its own (copied), e.g. an empirical potential fitted
 * apart from the fine one, as the paper's strategy II has it; NULL restores the default.
 * Combines with snapmd_set_coarse_snap.  Errors: SNAPMD_EINVAL (d, c not > 0 or a
 * coefficient not finite). */
int snapmd_set_coarse_fs(snapmd_ctx *ctx, const snapmd_fs *coarse);

/* Gradients of the SNAP model with respect to its coefficients beta (for a
 * force-matching fit; the loss is the caller's):
 *   dEdbeta[k]  = sum_i B_k(i)                    (k = 1..K; dEdbeta[0] = n_atoms)
 *   gradF[k]    = sum_i w_i . dF_i/dbeta_k = -sum_i w_i . d(sum_j B_k(j))/dx_i
 * for a per-atom weight field w (e.g. the loss gradient dLoss/dF).
 * x, w: device [3][n_atoms]; dEdbeta, gradF: device [n_coeff + 1], overwritten
 * (per system totals are summed over the batch).  Asynchronous on `stream`. */
int snap_beta_grad(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch,
                   const double *x, const double *w, double *dEdbeta, double *gradF,
                   void *stream);

/* Bispectrum components of every atom (the features E_i is linear in):
 * B: device [n_coeff][n_atoms], B[k-1][i] = B_k(i) for k = 1..n_coeff (same order as
 * beta[1..]).  Asynchronous on `stream`. */
int snapmd_bispectrum(snapmd_ctx *ctx, const snapmd_snap *snap, const snapmd_batch *batch,
                      const double *x, double *B, void *stream);

/* Launch mode of langevin_steps and of the fine and coarse propagation of
 * parareal_iterate.  enable = 1 (the default): the n_steps launch sequence is captured
 * once into a hipGraph, cached per context (keyed by sizes, parameters and device
 * pointers; at most 256 kept per workspace, least recently used dropped; every cached graph is dropped
 * when the context reallocates a work buffer) and replayed on the caller's stream.
 * enable = 0: kernels are launched one by one.  A call of more than 1000 steps is replayed
 * as captured segments of 250 steps (the step offsets of the systems are advanced on the
 * device between segments), so no captured chain holds more than about 4,000 kernels.
 * Results are identical either way.
 * While snapmd_profile is on, SNAP propagation is launched one by one. */
int snapmd_use_graphs(snapmd_ctx *ctx, int enable);

/* Wigner-Seitz analysis of a bcc lattice (to follow the interstitial between its
 * metastable states; stands in for the Voronoi analysis the paper runs with OVITO,
 * section "Numerical results").  Every box edge of every system must be a whole number
 * n of cubic cells of edge a (lattice constant, A).  The sites of system s are the cube
 * corners and centres of its cells, numbered first_s + 2 (ix ny nz + iy nz + iz) + b
 * (b = 0 corner (ix, iy, iz) a, b = 1 centre), first_s = sum over earlier systems of
 * 2 nx ny nz.  site[i] (device, [N]) receives the site nearest to atom i (positions may
 * be unwrapped; of two equally near sites the corner wins) and occ (device, [n_occ],
 * n_occ >= total number of sites) the number of atoms of each site: a site holding two
 * atoms is an interstitial dumbbell, an empty one a vacancy.  Asynchronous on stream.
 * Errors: SNAPMD_EINVAL (a box edge not a whole number of cells, occ too small). */
int snapmd_ws_sites(snapmd_ctx *ctx, const snapmd_batch *batch, const double *x, double a, int32_t *site,
                    int32_t *occ, int32_t n_occ, void *stream);

/* Energy minimisation by steepest descent (the first step of the paper's equilibration,
 * section "Numerical results": insert the interstitial, minimise the energy, then
 * thermalise): x <- x + F_i min(alpha, dmax / |F_i|) per atom (alpha in A^2/eV, dmax in
 * A), with the forces of `potential` (SNAPMD_POT_FS, or SNAPMD_POT_FS_SNAP with snap).
 * Stops when max_i |F_i| < ftol (eV/A), tested every 20 steps, or after max_iter steps.
 * x (device, [3][N]) is updated in place; *fmax_out (host) receives max_i |F_i| at the
 * last test and *iters_out the steps taken.  Synchronises the stream.  Errors:
 * SNAPMD_EINVAL, SNAPMD_ENONFINITE (forces became non-finite). */
int snapmd_relax(snapmd_ctx *ctx, int potential, const snapmd_snap *snap, const snapmd_fs *fs,
                 const snapmd_batch *batch, double *x, int32_t max_iter, double ftol, double alpha, double dmax,
                 double *fmax_out, int32_t *iters_out, void *stream);

/* Kernel shapes of the SNAP force passes (tuning, not part of the method), chosen per
 * twojmax (2, 4, 6 or 8; above 8 each pass has a single shape):
 *   density_acc       density pass: the most density elements one lane accumulates
 *                     (45, 28 or 21; smaller: more waves of fewer registers, each
 *                     recomputing the lower levels of its column chain);
 *   dedr_stage_atoms  dE/dr: a wave whose 64 pairs belong to at most this many atoms copies
 *                     their adjoint rows into local memory first (5, 3, or 0: never);
 *   adjoint_waves     LDS-tiled adjoint: waves per 64-atom tile (12 or 8);
 *   density_parts     density pass of a force evaluation: the neighbour slots of a tile are
 *                     split over this many waves (1 or 2), whose partial densities the
 *                     adjoint adds as it loads them (more, shorter waves); 0: split (2)
 *                     a launch whose density pass has fewer waves than the device has
 *                     SIMDs (a small chunk, where one wave per SIMD leaves the pass
 *                     latency-bound), else 1.
 * With the same split, forces do not depend on the shape and per-atom energies only
 * through the order in which the adjoint's partial sums are added; the two splits differ
 * by the rounding of the density sum (so with density_parts 0 the rounding depends on how
 * many atoms a call propagates at once).
 * snapmd_set_kernel_shape(ctx, J, NULL) restores the built-in shape (45, 0, 12, 0); any
 * other value is SNAPMD_EINVAL.  snapmd_get_kernel_shape writes the shape in use for J. */
typedef struct {
    int32_t density_acc;
    int32_t dedr_stage_atoms;
    int32_t adjoint_waves;
    int32_t density_parts;
} snapmd_kernel_shape;
int snapmd_set_kernel_shape(snapmd_ctx *ctx, int32_t twojmax, const snapmd_kernel_shape *shape);
int snapmd_get_kernel_shape(snapmd_ctx *ctx, int32_t twojmax, snapmd_kernel_shape *shape);

/* Slab chunks of parareal_iterate (tuning, not part of the method).  The pipelined path
 * of parareal_iterate (systems the on-device sweep handles, BAOAB) propagates the S slabs
 * of a window in chunks of consecutive slabs: the SNAP propagation of chunk c runs while
 * the sweep works through chunk c - 1.  snapmd_set_chunk_plan(ctx, sizes, n) makes every
 * later window of exactly sizes[0] + .. + sizes[n-1] slabs use those chunks, in order;
 * windows of other lengths, and n = 0 (sizes ignored), use the built-in plan (chunks of
 * whole adjoint rounds).  1 <= n <= 64 and every size >= 1, else SNAPMD_EINVAL.
 * snapmd_chunk_plan writes the plan that a window of S slabs of N atoms would use into
 * sizes[0 .. *n) (sizes holds at least 64 entries).  The results of parareal_iterate do
 * not depend on the plan as long as every launch takes the same density split (kernel
 * shape density_parts 1 or 2, or systems so small that every launch splits; tested).
 * With the automatic split (density_parts 0, the built-in shape) a launch of few atoms
 * sums each density in two parts, so a slab that lands in such a chunk under one plan and
 * in a larger chunk under another gets results that differ in the last bits (tested at 64
 * slabs of 1025 atoms: within 1e-9 relative).  The run time depends on the plan. */
int snapmd_set_chunk_plan(snapmd_ctx *ctx, const int32_t *sizes, int32_t n);
int snapmd_chunk_plan(snapmd_ctx *ctx, int32_t S, int32_t N, int32_t *sizes, int32_t *n);

/* Width of the on-device coarse sweep (tuning, not part of the method).  Systems of 512 to
 * 65,535 atoms are swept by K workgroups (one compute unit each) that exchange positions
 * and embedding derivatives every step; K trades the compute per workgroup against the
 * cost of the exchanges and against compute units taken from the SNAP propagation running
 * beside it.  snapmd_set_sweep_workgroups(ctx, K) asks for K workgroups in later calls of
 * parareal_iterate (0: the built-in choice, the fewest from 8 up with at most 64 atoms
 * each, else with at most 128); K = 1 asks for the one-workgroup sweep (positions,
 * embedding derivatives and lists in the local memory of one compute unit, no exchanges),
 * which fits systems of up to about 1,500 atoms; a K that the system cannot use (more than
 * 128 atoms per workgroup, or a local-memory tile over 160 KB) falls back to the built-in
 * choice.  0 <= K <= 64, else SNAPMD_EINVAL.  snapmd_sweep_workgroups writes the width a
 * system of N atoms would get into *K (1: one workgroup, 0: driven from the host).
 * Results do not depend on K beyond the rounding order of the partial sums of the adaptive
 * criterion, which every K combines in a fixed order. */
int snapmd_set_sweep_workgroups(snapmd_ctx *ctx, int32_t K);
int snapmd_sweep_workgroups(snapmd_ctx *ctx, int32_t N, int32_t *K);

/* SNAP streams of a parareal iteration of one system (tuning, not part of the method):
 * with 2 (the built-in value) the odd slab chunks run their SNAP propagation on a stream
 * of their own, with a second workspace, beside the even ones, so that one chunk's small
 * kernels and partial rounds fill the compute units the other leaves idle; with 1 every
 * chunk runs on the caller's stream.  An iteration that does not follow a pipelined one
 * (every synchronous call) runs its chunks one after another on the two streams, since
 * its sweep waits for each chunk in turn.  Kernel timing (snapmd_profile) runs iterations
 * on one stream.  n in {1, 2}, else SNAPMD_EINVAL.  Results do not depend on n (every chunk
 * starts from a freshly built neighbour list in either workspace). */
int snapmd_set_fine_streams(snapmd_ctx *ctx, int32_t n);

/* Measurement support (not part of the propagation):
 * snapmd_profile(ctx, s) with s >= 1 starts recording HIP events around every s-th launch
 * of each of the SNAP kernels and the neighbour build, on the stream they are launched on
 * (clears earlier records; 0 stops; s < 0: SNAPMD_EINVAL).  Every event record leaves the
 * device idle for a few microseconds, so a sample (s > 1) disturbs the measured run less.
 * snapmd_profile_read synchronises the device and returns, for kernel id
 * 0 = SNAP dE/dr, 1 = SNAP adjoint, 2 = SNAP density, 3 = neighbour build,
 * the summed duration (ms) and the number of launches recorded (a pair of events the
 * runtime cannot time is left out).  Neighbour builds
 * replayed from a captured graph (FS-only propagation) are not recorded. */
int snapmd_profile(snapmd_ctx *ctx, int enable);
int snapmd_profile_read(snapmd_ctx *ctx, int kernel, double *total_ms, int64_t *launches);
/* Number of neighbour pairs (both directions) of the last neighbour build, after a
 * device synchronisation. */
int snapmd_pair_count(snapmd_ctx *ctx, int64_t *n_pairs);

#ifdef __cplusplus
}
#endif
#endif /* SNAPMD_H */
