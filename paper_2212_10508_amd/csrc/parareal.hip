// Parareal pieces of snapmd (gfx950, FP64).
//
//   k_slabs_to_batch : slab states [slot][3][N] -> batch layout [3][S*N] (S slabs)
//   k_jumps          : J = F(prev) - C(prev) in batch layout (in place into the fine copy)
//   k_coarse_sweep_lds : the sequential part of a parareal iteration in ONE persistent
//                      workgroup: for n = n_in .. n_fi-1, cur_{n+1} = C(cur_n) + J_n with
//                      C = L BAOAB steps on the Finnis-Sinclair potential (force at the
//                      slab start, same noise counters as the batched propagators), the
//                      relative error delta = sum |cur - prev| / sum |prev| accumulated
//                      over the slabs done so far, and the early stop of the adaptive
//                      algorithm when delta exceeds the explosion threshold.  In its
//                      initialisation mode it only propagates (cur_{n+1} = C(cur_n)).
// The sweep keeps a Verlet list with a skin, rebuilt when an atom has moved more than
// half the skin since the last build; forces use the exact cutoffs, so the list only
// decides which pairs are examined.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_util.h"
#include "kernels.h"
#include "snapmd_internal.h"

namespace snapmd {

#define SW_MVV2E 1.0364269652680506e-4
constexpr int kSweepThreads = 1024;

__device__ __forceinline__ double mimg_s(double d, double L, double iL) { return d - L * rint(d * iL); }

__global__ void k_slabs_to_batch(int S, int N, const double *__restrict__ slots, double *__restrict__ out) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t tot = (size_t)3 * S * N;
    if (q >= tot) return;
    // out[al][s*N + i] = slots[s][al][i]
    const size_t al = q / ((size_t)S * N), r = q % ((size_t)S * N);
    const size_t s = r / N, i = r % N;
    out[q] = slots[(s * 3 + al) * N + i];
}

__global__ void k_jumps(size_t n, double *__restrict__ a, const double *__restrict__ b) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) a[q] = a[q] - b[q];
}

struct SweepArgs {
    int N;
    double Lx, Ly, Lz, iLx, iLy, iLz;
    FsParams fp;
    double skin;
    double dt, c1, mass, sig;
    uint64_t seed, noise_id;
    int L, n_in, n_fi, mode;  // slabs n_in .. n_fi-1; mode 0: initialise (no jumps), 1: corrected
    int n_win;                // first slab of the window (the early stop keeps at least n_win + 1)
    int ncx, ncy, ncz;        // cell grid of the list build (edges >= list radius), 0: all pairs
    // multi-workgroup sweep: K workgroups own A consecutive atoms each and exchange
    // positions and F'(rho) every step through device memory
    int K, A;
    // (tagged words, two per value, cleared before the launch)
    unsigned long long *gx;       // [2][3][N][2] positions by step parity
    unsigned long long *gdfe;     // [2][N][2] F'(rho) by step parity
    unsigned long long *gpart;    // [2][4][K][2] per-workgroup partials by parity
    int *abort;                   // set when a wait runs out (zero at launch)
    double delta_expl;
    double *q_cur, *p_cur;                 // [slot][3][ld] (this system's atoms at 0 .. N-1)
    const double *q_prev, *p_prev;         // [slot][3][ld] (mode 1)
    const double *jq, *jp;                 // jump of slab n_in + s, row al, atom i at al jsa + s jss + i (mode 1)
    size_t ld, jsa, jss;
    // [0] delta, [1] n_fi after, [2] bad slab (-1 none), [3] overflow, [4] sum |cur - prev|,
    // [5] sum |prev|, [6] stopped: carried from one launch to the next over the slabs of a
    // window, initialised by the host
    double *out;
    const double *noise;                   // [S][L][3][N] Gaussians of slabs n_in .. n_fi-1 (or drawn in place)
};

__device__ __forceinline__ void sweep_gauss3(uint64_t seed, uint64_t noise_id, uint64_t step, uint64_t atom,
                                             double &g0, double &g1, double &g2) {
    uint64_t c[4] = {noise_id, step, atom, 0};
    uint64_t k0 = seed, k1 = 0;
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    const double two53 = 1.0 / 9007199254740992.0;
    const double u1 = 1.0 - (double)(c[0] >> 11) * two53, u2 = (double)(c[1] >> 11) * two53;
    const double u3 = 1.0 - (double)(c[2] >> 11) * two53, u4 = (double)(c[3] >> 11) * two53;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    double s2, c2, s4, c4;
    sincos(2.0 * M_PI * u2, &s2, &c2);
    sincos(2.0 * M_PI * u4, &s4, &c4);
    g0 = r1 * c2;
    g1 = r1 * s2;
    g2 = r2 * c4;
}

// ---------------------------------------------------------------------------
// LDS-resident sweep (N <= kSweepLdsMaxAtoms): positions, F'(rho) and a uint16 Verlet
// list live in LDS; momenta, forces and reference positions of the atoms a thread owns
// live in its registers.  Thread t owns atom t.  Atoms beyond the first 1024 are owned
// by a second round of threads (t + 1024) or, when there are at most 16 of them, one
// per wave, the wave's lanes then sharing that atom's neighbour list.
// The rho pass marks the list entries within the force cutoff; the force pass of the
// same step visits only those.
// ---------------------------------------------------------------------------
constexpr int kSweepLdsNeigh = 48;
constexpr int kSweepNbRows = kSweepLdsNeigh + 3;  // a thread's list is padded to a multiple of 4
constexpr int kSweepLdsMaxAtoms = 2048;
constexpr int kSpillMax = kSweepThreads / 64;
constexpr int kSweepMaxCells = 512;

// positions, F'(rho), list, the momenta / forces / reference positions of the atoms
// beyond the first 1024 (their owners keep them in LDS), reduction partials, cell grid
// (counts / fill pointers, starts, atoms by cell, cell of each atom)
size_t sweep_lds_bytes(int N) {
    const size_t NS = N > kSweepThreads ? (size_t)(N - kSweepThreads) : 0;
    return (size_t)N * (3 * sizeof(double) + sizeof(double) + kSweepNbRows * sizeof(uint16_t)) +
           NS * 9 * sizeof(double) + kSpillMax * sizeof(double) + (2 * kSweepMaxCells + 1) * sizeof(int) +
           (size_t)N * 2 * sizeof(uint16_t) + 8;
}

struct SwCells {
    int *cnt, *start;             // [kSweepMaxCells], [kSweepMaxCells + 1]
    uint16_t *atom, *cid;         // [N] atoms by cell (ascending in each cell), cell of each atom
};

__device__ __forceinline__ int swl_cell_index(double v, double iL, int n) {
    double f = v * iL;
    f -= floor(f);
    const int c = (int)(f * n);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}
__device__ __forceinline__ int swl_cell_of(const SweepArgs &a, double x, double y, double z) {
    return (swl_cell_index(x, a.iLx, a.ncx) * a.ncy + swl_cell_index(y, a.iLy, a.ncy)) * a.ncz +
           swl_cell_index(z, a.iLz, a.ncz);
}
// cell cc of the 27-cell stencil (o = 0..26) around cell c (periodic)
__device__ __forceinline__ int swl_stencil(const SweepArgs &a, int c, int o) {
    const int cz = c % a.ncz, cy = (c / a.ncz) % a.ncy, cx = c / (a.ncz * a.ncy);
    const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
    return (((cx + ox + a.ncx) % a.ncx) * a.ncy + (cy + oy + a.ncy) % a.ncy) * a.ncz + (cz + oz + a.ncz) % a.ncz;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
// workgroup reductions through kSpillMax wave partials (fixed order, every thread gets the result)
__device__ __forceinline__ double wg_sum(double v, double *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kSpillMax; ++w) r += red[w];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double wg_max(double v, double *red) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kSpillMax; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

// separation x_j - x_i (minimum image) of list entry j
__device__ __forceinline__ void swl_sep(const SweepArgs &a, const double *__restrict__ xs, int N, int j, double xi,
                                        double yi, double zi, double &dx, double &dy, double &dz) {
    dx = mimg_s(xs[j] - xi, a.Lx, a.iLx);
    dy = mimg_s(xs[N + j] - yi, a.Ly, a.iLy);
    dz = mimg_s(xs[2 * N + j] - zi, a.Lz, a.iLz);
}

// list test of the pair (i, j): within the list radius
__device__ __forceinline__ bool swl_pair(const SweepArgs &a, const double *__restrict__ xs, int N, int j, double xi,
                                         double yi, double zi, double rcl2) {
    double dx, dy, dz;
    swl_sep(a, xs, N, j, xi, yi, zi, dx, dy, dz);
    return dx * dx + dy * dy + dz * dz < rcl2;
}

// list of atom i by one thread (j ascending); returns the count (capped, overflow flagged)
// (list entries of atom i: col[t * ns], t = 0, 1, ..)
__device__ __forceinline__ int swl_build_thread(const SweepArgs &a, const double *__restrict__ xs,
                                                uint16_t *__restrict__ col, int ns, const SwCells &cl, int i,
                                                double rcl2, int &overflow, int h = 0, int H = 1) {
    const int N = a.N;
    const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
    int c = 0;
    if (a.ncx > 0) {  // the 27 cells around i's cell, atoms of a cell in ascending order
        const int ci = cl.cid[i];
        for (int o = h; o < 27; o += H) {
            const int cc = swl_stencil(a, ci, o);
            for (int q = cl.start[cc]; q < cl.start[cc + 1]; ++q) {
                const int j = cl.atom[q];
                if (j != i && swl_pair(a, xs, N, j, xi, yi, zi, rcl2)) {
                    if (c < kSweepLdsNeigh) col[c * ns] = (uint16_t)j;
                    ++c;
                }
            }
        }
    } else {
        for (int j = h * N / H; j < (h + 1) * N / H; ++j) {
            if (j != i && swl_pair(a, xs, N, j, xi, yi, zi, rcl2)) {
                if (c < kSweepLdsNeigh) col[c * ns] = (uint16_t)j;
                ++c;
            }
        }
    }
    if (c > kSweepLdsNeigh) {
        overflow = 1;
        c = kSweepLdsNeigh;
    }
    // rows c .. c+2 repeat the last entry (read, never counted, by the unrolled passes)
    const uint16_t last = c > 0 ? col[(c - 1) * ns] : (uint16_t)i;
#pragma unroll
    for (int t = 0; t < 3; ++t) col[(c + t) * ns] = last;
    return c;
}

// list of atom i by a whole wave (lanes scan 64 j at a time, ballot compaction keeps j ascending)
__device__ __forceinline__ int swl_build_wave(const SweepArgs &a, const double *__restrict__ xs,
                                              uint16_t *__restrict__ col, int ns, const SwCells &cl, int i,
                                              double rcl2, int &overflow) {
    const int N = a.N, lane = threadIdx.x & 63;
    const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
    const uint64_t below = (1ull << lane) - 1ull;
    int c = 0;
    // candidates in the order of the thread build: stencil cells, ascending in each
    const int no = a.ncx > 0 ? 27 : 1;
    for (int o = 0; o < no; ++o) {
        int q0 = 0, q1 = N;
        if (a.ncx > 0) {
            const int cc = swl_stencil(a, cl.cid[i], o);
            q0 = cl.start[cc];
            q1 = cl.start[cc + 1];
        }
        for (int base = q0; base < q1; base += 64) {
            const int q = base + lane;
            const int j = q < q1 ? (a.ncx > 0 ? (int)cl.atom[q] : q) : i;
            const int hit = (j != i) ? (int)swl_pair(a, xs, N, j, xi, yi, zi, rcl2) : 0;
            const uint64_t m = __ballot(hit);
            const int pos = c + __popcll(m & below);
            if (hit && pos < kSweepLdsNeigh) col[pos * ns] = (uint16_t)j;
            c += __popcll(m);
        }
    }
    if (c > kSweepLdsNeigh) {
        overflow = 1;
        c = kSweepLdsNeigh;
    }
    return c;
}

// rho pass of atom i by one thread: F'(rho_i) into dfe[i]; mask of the entries within
// the force cutoff (positions do not change before the force pass of the same step).
// The unrolled body is branch-free (entries past the count repeat the last one and
// add nothing) so that the LDS reads of four neighbours are in flight together.
__device__ __forceinline__ uint64_t swl_rho_acc(const SweepArgs &a, const double *__restrict__ xs,
                                                const uint16_t *__restrict__ col, int ns, int i, int c,
                                                double &acc_out) {
    const int N = a.N;
    const FsParams fp = a.fp;
    const double d2c = fp.d * fp.d, rc2f = fmax(fp.d, fp.c) * fmax(fp.d, fp.c);
    const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
    double acc = 0.0;
    uint64_t mk = 0;
    for (int t0 = 0; t0 < c; t0 += 4) {
        int e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = (int)col[__umul24(t0 + u, ns)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool valid = t0 + u < c;
            double dx, dy, dz;
            swl_sep(a, xs, N, e[u], xi, yi, zi, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            mk |= (valid && r2 < rc2f) ? (1ull << (t0 + u)) : 0ull;
            const double r = r2 * rsqrt_nr(r2);
            acc += (valid && r2 < d2c) ? (r - fp.d) * (r - fp.d) : 0.0;
        }
    }
    acc_out = acc;
    return mk;
}
__device__ __forceinline__ double swl_dfe(const FsParams &fp, double acc) {
    return acc > 0.0 ? -fp.A / (2.0 * sqrt(acc)) : 0.0;
}
__device__ __forceinline__ uint64_t swl_rho_thread(const SweepArgs &a, const double *__restrict__ xs,
                                                   double *__restrict__ dfe, const uint16_t *__restrict__ col, int ns,
                                                   int i, int c) {
    double acc;
    const uint64_t mk = swl_rho_acc(a, xs, col, ns, i, c, acc);
    dfe[i] = swl_dfe(a.fp, acc);
    return mk;
}

// pair force term w = (dE/dr) / r of a pair at distance r (ir = 1/r)
__device__ __forceinline__ double swl_w(const FsParams &fp, double r, double ir, double dFi, double dFj) {
    const double tt = r - fp.c, poly = fp.c0 + r * (fp.c1 + r * fp.c2);
    const double pc = r < fp.c ? 2.0 * tt * poly + tt * tt * (fp.c1 + 2.0 * fp.c2 * r) : 0.0;
    const double pd = r < fp.d ? (dFi + dFj) * 2.0 * (r - fp.d) : 0.0;
    return (pc + pd) * ir;
}

// force pass of atom i by one thread over the masked entries (branch-free groups of 4)
__device__ __forceinline__ void swl_force_thread(const SweepArgs &a, const double *__restrict__ xs,
                                                 const double *__restrict__ dfe, const uint16_t *__restrict__ col,
                                                 int ns, int i, uint64_t m, double (&f)[3]) {
    const int N = a.N;
    const FsParams fp = a.fp;
    const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
    const double dFi = dfe[i];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    while (m) {
        int e[4];
        bool v[4];
        int t = __builtin_ctzll(m);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = m != 0;
            t = v[u] ? __builtin_ctzll(m) : t;
            m &= m - 1ull;
            e[u] = (int)col[__umul24(t, ns)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double dx, dy, dz;
            const int j = e[u];
            swl_sep(a, xs, N, j, xi, yi, zi, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt_nr(r2), r = r2 * ir;
            const double w = swl_w(fp, r, ir, dFi, dfe[j]);
            fx += v[u] ? w * dx : 0.0;
            fy += v[u] ? w * dy : 0.0;
            fz += v[u] ? w * dz : 0.0;
        }
    }
    f[0] = fx;
    f[1] = fy;
    f[2] = fz;
}

// rho pass of atom i by a whole wave (lane t takes entry t, c <= 64); returns the mask
__device__ __forceinline__ uint64_t swl_rho_wave(const SweepArgs &a, const double *__restrict__ xs,
                                                 double *__restrict__ dfe, const uint16_t *__restrict__ col, int ns,
                                                 int i, int c) {
    const int N = a.N, lane = threadIdx.x & 63;
    const FsParams fp = a.fp;
    const double d2c = fp.d * fp.d, rc2f = fmax(fp.d, fp.c) * fmax(fp.d, fp.c);
    double v = 0.0;
    int in = 0;
    if (lane < c) {
        double dx, dy, dz;
        swl_sep(a, xs, N, (int)col[lane * ns], xs[i], xs[N + i], xs[2 * N + i], dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        in = r2 < rc2f;
        if (r2 < d2c) {
            const double r = r2 * rsqrt_nr(r2);
            v = (r - fp.d) * (r - fp.d);
        }
    }
    const uint64_t mk = __ballot(in);
    const double acc = wave_sum(v);
    if (lane == 0) dfe[i] = acc > 0.0 ? -fp.A / (2.0 * sqrt(acc)) : 0.0;
    return mk;
}

// force pass of atom i by a whole wave; every lane receives the force
__device__ __forceinline__ void swl_force_wave(const SweepArgs &a, const double *__restrict__ xs,
                                               const double *__restrict__ dfe, const uint16_t *__restrict__ col,
                                               int ns, int i, uint64_t mk, double (&f)[3]) {
    const int N = a.N, lane = threadIdx.x & 63;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if ((mk >> lane) & 1ull) {
        double dx, dy, dz;
        const int j = (int)col[lane * ns];
        swl_sep(a, xs, N, j, xs[i], xs[N + i], xs[2 * N + i], dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ir = rsqrt_nr(r2), r = r2 * ir;
        const double w = swl_w(a.fp, r, ir, dfe[i], dfe[j]);
        fx = w * dx;
        fy = w * dy;
        fz = w * dz;
    }
    f[0] = wave_sum(fx);
    f[1] = wave_sum(fy);
    f[2] = wave_sum(fz);
}

// Body of the LDS-resident sweep of one system.  Drawn = true: the Gaussians are drawn in
// place (counter (noise_id, n L + l, atom)) instead of read from a window table.
template <bool Drawn>
__device__ __forceinline__ void sweep_lds_body(const SweepArgs &a) {
    extern __shared__ double sm[];
    if (a.out[6] != 0.0) return;  // an earlier launch of the window stopped early
    const int N = a.N;
    const int NS = N > kSweepThreads ? N - kSweepThreads : 0;
    double *red = sm;                                      // [kSpillMax]
    double *xs = red + kSpillMax;                          // [3][N]
    double *dfe = xs + 3 * N;                              // [N]  F'(rho)
    double *s1 = dfe + N;                                  // [9][NS] p, f, reference x of atoms >= 1024
    uint16_t *nb = reinterpret_cast<uint16_t *>(s1 + 9 * NS);  // [kSweepNbRows][N]
    SwCells cl;
    cl.cnt = reinterpret_cast<int *>(nb + (size_t)kSweepNbRows * N + ((kSweepNbRows * N) & 1));
    cl.start = cl.cnt + kSweepMaxCells;
    cl.atom = reinterpret_cast<uint16_t *>(cl.start + kSweepMaxCells + 1);
    cl.cid = cl.atom + N;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // second slot: the spill atom of this wave (lane 0 owns it) or atom tid + 1024
    const bool spill = NS > 0 && NS <= kSpillMax;
    const int is = kSweepThreads + wv;                     // spill atom of the wave
    const bool has_s = spill && is < N;                    // wave-uniform
    const int i1 = spill ? (lane == 0 ? is : N) : tid + kSweepThreads;
    const bool own0 = tid < N, own1 = i1 < N;
    double *p1 = s1 + (i1 - kSweepThreads), *f1 = p1 + 3 * NS, *r1 = p1 + 6 * NS;  // [al * NS] (own1 only)
    const double rcl = fmax(a.fp.d, a.fp.c) + a.skin, rcl2 = rcl * rcl;
    double pr[3], fr[3], xr[3];
    int cn0 = 0, cn1 = 0;
    uint64_t mk0 = 0, mk1 = 0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        fr[al] = 0.0;
        xr[al] = 0.0;
        pr[al] = 0.0;
        if (own0) {
            xs[al * N + tid] = a.q_cur[((size_t)a.n_in * 3 + al) * a.ld + tid];
            pr[al] = a.p_cur[((size_t)a.n_in * 3 + al) * a.ld + tid];
        }
        if (own1) {
            xs[al * N + i1] = a.q_cur[((size_t)a.n_in * 3 + al) * a.ld + i1];
            p1[al * NS] = a.p_cur[((size_t)a.n_in * 3 + al) * a.ld + i1];
            f1[al * NS] = 0.0;
        }
    }
    __syncthreads();
    int overflow = 0;
    // thread-owned atoms of this thread: tid, and i1 outside the spill mode (one inlined
    // copy of the per-thread passes, looped over the two slots)
    const int nslot = (!spill && own1) ? 2 : 1;
    const int NC = a.ncx * a.ncy * a.ncz;
    auto build = [&]() {
        if (NC > 0) {
            // cell grid: counts, starts (wave 0), fill, ascending order inside each cell
            for (int c = tid; c < NC; c += kSweepThreads) cl.cnt[c] = 0;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int i = q ? i1 : tid;
                if (i < N) {
                    const int c = swl_cell_of(a, xs[i], xs[N + i], xs[2 * N + i]);
                    cl.cid[i] = (uint16_t)c;
                    atomicAdd(&cl.cnt[c], 1);
                }
            }
            __syncthreads();
            if (tid < 64) {
                constexpr int per = kSweepMaxCells / 64;
                int loc[per], sum = 0;
#pragma unroll
                for (int k = 0; k < per; ++k) {
                    const int c = tid * per + k;
                    loc[k] = c < NC ? cl.cnt[c] : 0;
                    sum += loc[k];
                }
                int incl = sum;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int v = __shfl_up(incl, o, 64);
                    if (tid >= o) incl += v;
                }
                int run = incl - sum;
#pragma unroll
                for (int k = 0; k < per; ++k) {
                    const int c = tid * per + k;
                    if (c < NC) {
                        cl.start[c] = run;
                        cl.cnt[c] = run;  // fill pointer
                    }
                    run += loc[k];
                }
                if (tid == 63) cl.start[NC] = incl;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int i = q ? i1 : tid;
                if (i < N) cl.atom[atomicAdd(&cl.cnt[cl.cid[i]], 1)] = (uint16_t)i;
            }
            __syncthreads();
            for (int c = tid; c < NC; c += kSweepThreads) {
                const int b = cl.start[c], e = cl.start[c + 1];
                for (int q = b + 1; q < e; ++q) {
                    const uint16_t v = cl.atom[q];
                    int r = q - 1;
                    while (r >= b && cl.atom[r] > v) {
                        cl.atom[r + 1] = cl.atom[r];
                        --r;
                    }
                    cl.atom[r + 1] = v;
                }
            }
            __syncthreads();
        }
#pragma unroll 1
        for (int q = 0; q < nslot; ++q) {
            const int i = q ? i1 : tid;
            if (i < N) {
                const int c = swl_build_thread(a, xs, nb + i, N, cl, i, rcl2, overflow);
                if (q) cn1 = c;
                else cn0 = c;
            }
        }
        if (has_s) cn1 = swl_build_wave(a, xs, nb + is, N, cl, is, rcl2, overflow);
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            if (own0) xr[al] = xs[al * N + tid];
            if (own1) r1[al * NS] = xs[al * N + i1];
        }
        __syncthreads();
    };
    auto forces = [&]() {
#pragma unroll 1
        for (int q = 0; q < nslot; ++q) {
            const int i = q ? i1 : tid;
            if (i < N) {
                const uint64_t m = swl_rho_thread(a, xs, dfe, nb + i, N, i, q ? cn1 : cn0);
                if (q) mk1 = m;
                else mk0 = m;
            }
        }
        if (has_s) mk1 = swl_rho_wave(a, xs, dfe, nb + is, N, is, cn1);
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < nslot; ++q) {
            const int i = q ? i1 : tid;
            if (i < N) {
                double g[3];
                swl_force_thread(a, xs, dfe, nb + i, N, i, q ? mk1 : mk0, g);
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    if (q) f1[al * NS] = g[al];
                    else fr[al] = g[al];
                }
            }
        }
        if (has_s) {
            double g[3];
            swl_force_wave(a, xs, dfe, nb + is, N, is, mk1, g);
            if (own1)
#pragma unroll
                for (int al = 0; al < 3; ++al) f1[al * NS] = g[al];
        }
        __syncthreads();
    };
    double num = a.out[4], den = a.out[5], delta = a.out[0];
    int nfi_new = -1, bad = -1;
    const double hk = 0.5 * a.dt / SW_MVV2E, hd = 0.5 * a.dt / a.mass;
    bool built = false;
    for (int n = a.n_in; n < a.n_fi; ++n) {
        // l = -1: force at the slab start (slab states may have jumped); then L BAOAB steps.
        // The list is rebuilt only if some atom moved more than skin/2 since the last build.
        for (int l = -1; l < a.L; ++l) {
            double d0 = 0.0, d1 = 0.0;
            const double *gz = Drawn ? nullptr : a.noise + ((size_t)((n - a.n_in) * a.L + max(l, 0)) * 3) * N;
            double gd0[3] = {0.0, 0.0, 0.0}, gd1[3] = {0.0, 0.0, 0.0};
            if (Drawn && l >= 0) {
                const uint64_t gs = (uint64_t)n * (uint64_t)a.L + (uint64_t)l;
                if (own0) sweep_gauss3(a.seed, a.noise_id, gs, (uint64_t)tid, gd0[0], gd0[1], gd0[2]);
                if (own1) sweep_gauss3(a.seed, a.noise_id, gs, (uint64_t)i1, gd1[0], gd1[1], gd1[2]);
            }
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                if (own0) {
                    double xx = xs[al * N + tid];
                    if (l >= 0) {
                        double pp = pr[al] + hk * fr[al];
                        xx = xx + hd * pp;
                        pp = a.c1 * pp + a.sig * (Drawn ? gd0[al] : gz[al * N + tid]);
                        xx = xx + hd * pp;
                        pr[al] = pp;
                        xs[al * N + tid] = xx;
                    }
                    d0 += (xx - xr[al]) * (xx - xr[al]);
                }
                if (own1) {
                    double xx = xs[al * N + i1];
                    if (l >= 0) {
                        double pp = p1[al * NS] + hk * f1[al * NS];
                        xx = xx + hd * pp;
                        pp = a.c1 * pp + a.sig * (Drawn ? gd1[al] : gz[al * N + i1]);
                        xx = xx + hd * pp;
                        p1[al * NS] = pp;
                        xs[al * N + i1] = xx;
                    }
                    d1 += (xx - r1[al * NS]) * (xx - r1[al * NS]);
                }
            }
            const double m = wg_max(fmax(d0, d1), red);
            if (!built || !(4.0 * m <= a.skin * a.skin)) {
                build();
                built = true;
            }
            forces();
            if (l >= 0) {
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    pr[al] = pr[al] + hk * fr[al];
                    if (own1) p1[al * NS] = p1[al * NS] + hk * f1[al * NS];
                }
            }
        }
        const size_t s = (size_t)(n - a.n_in);
        double d2 = 0.0, p2 = 0.0, fin = 0.0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = q == 0 ? tid : i1;
            if (i >= N) continue;
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                double xq = xs[al * N + i], pq = q == 0 ? pr[al] : p1[al * NS];
                if (a.mode == 1) {
                    xq += a.jq[al * a.jsa + s * a.jss + i];
                    pq += a.jp[al * a.jsa + s * a.jss + i];
                    const double pv = a.q_prev[((size_t)(n + 1) * 3 + al) * a.ld + i];
                    d2 += (xq - pv) * (xq - pv);
                    p2 += pv * pv;
                }
                fin += xq * 0.0 + pq * 0.0;  // NaN/Inf propagate into fin
                xs[al * N + i] = xq;
                if (q == 0) pr[al] = pq;
                else p1[al * NS] = pq;
                a.q_cur[((size_t)(n + 1) * 3 + al) * a.ld + i] = xq;
                a.p_cur[((size_t)(n + 1) * 3 + al) * a.ld + i] = pq;
            }
        }
        const double sfin = wg_sum(fin, red);
        if (!isfinite(sfin)) {
            bad = n;
            break;
        }
        if (a.mode == 1) {
            const double sd = wg_sum(d2, red), sp = wg_sum(p2, red);
            num += sqrt(sd);
            den += sqrt(sp);
            delta = den > 0.0 ? num / den : 0.0;
            if (delta > a.delta_expl) {
                nfi_new = max(n, a.n_win + 1);
                break;
            }
        }
    }
    if (overflow) a.out[3] = 1.0;
    if (tid == 0) {
        a.out[0] = delta;
        a.out[4] = num;
        a.out[5] = den;
        if (nfi_new >= 0) a.out[1] = (double)nfi_new;
        if (bad >= 0) a.out[2] = (double)bad;
        if (nfi_new >= 0 || bad >= 0) a.out[6] = 1.0;
    }
}

__global__ void __launch_bounds__(1024) k_coarse_sweep_lds(SweepArgs a) { sweep_lds_body<false>(a); }

// The sweeps of several independent systems at once, one workgroup each (tab[blockIdx.x]);
// the Gaussians are drawn in place.
__global__ void __launch_bounds__(1024) k_coarse_sweep_lds_multi(const SweepArgs *__restrict__ tab) {
    const SweepArgs a = tab[blockIdx.x];
    sweep_lds_body<true>(a);
}

// ---------------------------------------------------------------------------
// Multi-workgroup sweep: the same propagation with the atoms split over K workgroups
// (one CU each; consecutive workgroups land on different chiplets, so the CUs taken from
// the batched kernels running beside the sweep are spread evenly).  Every
// step each workgroup publishes its atoms' positions, waits at a grid barrier, copies all
// positions into LDS, does the rho pass for its atoms, publishes F'(rho), waits again and
// does the force pass.  Shared data are written and read with device-scope accesses
// (coherent at the device level, so no cache-wide write-back or invalidation is
// needed); each wave waits for its stores to complete before the workgroup arrives at
// the barrier, one arrival slot per workgroup whose wait is bounded (a wait that runs
// out sets `abort` and every workgroup leaves).  Per-workgroup partial sums are combined in a fixed
// order, so every workgroup takes the same decisions.
// ---------------------------------------------------------------------------
constexpr int kMcSpin = 1 << 22;
// static LDS of the multi-workgroup sweep (the partial values, 3 x 64 doubles, and the
// workgroup vote of __syncthreads_or: 1,792 bytes), rounded up
constexpr size_t kMcStaticLds = 2048;

// Tagged words: a published double v of exchange b travels as two 64-bit words
// (b + 1) << 32 | low half and (b + 1) << 32 | high half, each written with one
// device-scope store, so a word holds either its old or its new contents and a reader
// recognises the value of exchange b by the tags.  The buffers are cleared before every
// launch (no word carries a live tag) and alternate by step parity (a workgroup cannot
// run two exchanges ahead of a reader, since it needs that reader's next values first).
__device__ __forceinline__ void put_tagged(unsigned long long *p, double v, unsigned long long b) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v), t = (b + 1) << 32;
    __hip_atomic_store(p, t | (u & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, t | (u >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_word(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the two words at p carry tag b + 1 and returns the double they hold;
// false (ok) when the caller's spin budget ran out or another workgroup gave up.
__device__ __forceinline__ double get_tagged(const unsigned long long *p, unsigned long long lo,
                                             unsigned long long hi, unsigned long long b, const SweepArgs &a,
                                             int &spins, bool &ok) {
    const unsigned long long t = b + 1;
    while (ok && ((lo >> 32) != t || (hi >> 32) != t)) {
        ++spins;
        if (spins > kMcSpin || ((spins & 255) == 0 && __hip_atomic_load(a.abort, __ATOMIC_RELAXED,
                                                                       __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        lo = ld_word(p);
        hi = ld_word(p + 1);
    }
    return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}

// Exchange b: the workgroup copies the np partial values parts[q] (tagged words) into pdst
// and n doubles of src (tagged words) into dst in LDS, 8 values per thread in flight (16
// were slower, measured); the words of the eight not yet tagged b are reloaded together
// until all are.  Ends with a workgroup barrier; returns
// false in every thread when some wait ran out or another workgroup gave up.
__device__ bool mc_get(double *__restrict__ dst, const unsigned long long *__restrict__ src, int n,
                       const unsigned long long *__restrict__ parts, int np, double *__restrict__ pdst,
                       unsigned long long b, const SweepArgs &a) {
    const int T = blockDim.x, tid = threadIdx.x;
    int spins = 0;
    bool ok = true;
    for (int q = tid; q < np && ok; q += T)
        pdst[q] = get_tagged(parts + 2 * q, ld_word(parts + 2 * q), ld_word(parts + 2 * q + 1), b, a, spins, ok);
    const unsigned long long tg = b + 1;
    for (int base = tid; base < n && ok; base += 8 * T) {
        unsigned long long lo[8], hi[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = base + k * T;
            lo[k] = q < n ? ld_word(src + 2 * q) : tg << 32;
            hi[k] = q < n ? ld_word(src + 2 * q + 1) : tg << 32;
        }
        // words not yet carrying the tag are loaded again together (one round trip per
        // retry for all eight, not one per word)
        while (true) {
            bool ready = true;
#pragma unroll
            for (int k = 0; k < 8; ++k) ready = ready && (lo[k] >> 32) == tg && (hi[k] >> 32) == tg;
            if (ready) break;
            ++spins;
            if (spins > kMcSpin ||
                ((spins & 255) == 0 && __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int q = base + k * T;
                if ((lo[k] >> 32) != tg) lo[k] = ld_word(src + 2 * q);
                if ((hi[k] >> 32) != tg) hi[k] = ld_word(src + 2 * q + 1);
            }
        }
        if (!ok) break;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = base + k * T;
            if (q < n) dst[q] = __longlong_as_double((long long)((hi[k] << 32) | (lo[k] & 0xffffffffull)));
        }
    }
    return __syncthreads_or(ok ? 0 : 1) == 0;
}

// kMcLanes lanes per atom: at most 512 / kMcLanes atoms per workgroup of at most 512 threads
constexpr int kMcLanes = 4;
constexpr int kMcMaxAtoms = 512 / kMcLanes;

// sum over the kMcLanes lanes of an atom (every lane gets the same value)
__device__ __forceinline__ double mc_lane_sum(double v) {
#pragma unroll
    for (int o = 1; o < kMcLanes; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(512) k_coarse_sweep_mc(SweepArgs a) {
    extern __shared__ double sm[];
    if (a.out[6] != 0.0) return;  // an earlier launch of the window stopped early
    const int N = a.N, K = a.K, A = a.A;
    const int w = blockIdx.x, a0 = w * A, na = min(N, a0 + A) - a0;
    const int tid = threadIdx.x;
    // kMcLanes lanes per atom: lane kMcLanes k + h holds atom a0 + k (state kept
    // identically in all of them) and the part of its list built from stencil cells
    // o = h, h + kMcLanes, .. (the short per-lane lists keep the passes' dependent chains
    // short; with one or two waves per SIMD nothing else hides their latency)
    const int k = tid / kMcLanes, h = tid % kMcLanes;
    const bool own = k < na, lead = own && h == 0;
    const int i = a0 + k;
    double *xs = sm;                                       // [3][N]
    double *dfe = xs + 3 * N;                              // [N]
    int *flag = reinterpret_cast<int *>(dfe + N);          // [2] (spare)
    uint16_t *nb = reinterpret_cast<uint16_t *>(flag + 2); // [kSweepNbRows][A]
    SwCells cl;
    cl.cnt = reinterpret_cast<int *>(nb + (size_t)kSweepNbRows * kMcLanes * A);
    cl.start = cl.cnt + kSweepMaxCells;
    cl.atom = reinterpret_cast<uint16_t *>(cl.start + kSweepMaxCells + 1);
    cl.cid = cl.atom + N;
    uint16_t *col = nb + tid;  // rows of stride kMcLanes A
    const int NC = a.ncx * a.ncy * a.ncz;
    const double rcl = fmax(a.fp.d, a.fp.c) + a.skin, rcl2 = rcl * rcl;
    const size_t SN = (size_t)(a.n_fi - a.n_in) * N;
    const double hk = 0.5 * a.dt / SW_MVV2E, hd = 0.5 * a.dt / a.mass;
    double pr[3] = {0.0, 0.0, 0.0}, fr[3] = {0.0, 0.0, 0.0}, xr[3] = {0.0, 0.0, 0.0}, xo[3] = {0.0, 0.0, 0.0};
    int cn = 0, overflow = 0, bad = -1, nfi_new = -1;
    uint64_t mk = 0;
    if (own)
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            xo[al] = a.q_cur[((size_t)a.n_in * 3 + al) * N + i];
            pr[al] = a.p_cur[((size_t)a.n_in * 3 + al) * N + i];
        }
    double num = a.out[4], den = a.out[5], delta = a.out[0];
    unsigned long long b = 0;
    int par = 0;
    bool built = false, alive = true;
    // partial values of the workgroups: gpart[parity][slot][K] tagged words (slot 0 the
    // displacement maximum, 1..3 the slab-end sums), received into pv
    __shared__ double pv[3 * 64];
    auto gpart = [&](int slot) { return a.gpart + 2 * ((size_t)(par * 4 + slot) * K); };
    // exchange: publish own positions and displacement maximum, gather all of them
    auto exchange_x = [&](double wmax) -> bool {
        if (lead)
#pragma unroll
            for (int al = 0; al < 3; ++al) put_tagged(a.gx + 2 * (((size_t)par * 3 + al) * N + i), xo[al], b);
        if (tid == 0) put_tagged(gpart(0) + 2 * w, wmax, b);
        const bool r = mc_get(xs, a.gx + 2 * (size_t)par * 3 * N, 3 * N, gpart(0), K, pv, b, a);
        ++b;
        return r;
    };
    auto partial = [&](int k) {  // sum over workgroups (fixed order) of slab-end partial k
        double s = 0.0;
        for (int v = 0; v < K; ++v) s += pv[(k - 1) * K + v];
        return s;
    };
    // the Gaussians of step l of slab n, loaded one step ahead (the load is off the
    // sequential chain of steps)
    auto noise_of = [&](int n, int l, double (&z)[3]) {
        const double *gz = a.noise + ((size_t)((n - a.n_in) * a.L + l) * 3) * N;
#pragma unroll
        for (int al = 0; al < 3; ++al) z[al] = gz[al * N + i];
    };
    double nz[3] = {0.0, 0.0, 0.0};
    for (int n = a.n_in; n < a.n_fi && alive; ++n) {
        if (own) noise_of(n, 0, nz);
        for (int l = -1; l < a.L; ++l) {
            double d2m = 0.0;
            if (own) {
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    if (l >= 0) {
                        double pp = pr[al] + hk * fr[al];
                        double xx = xo[al] + hd * pp;
                        pp = a.c1 * pp + a.sig * nz[al];
                        xx = xx + hd * pp;
                        pr[al] = pp;
                        xo[al] = xx;
                    }
                    d2m += (xo[al] - xr[al]) * (xo[al] - xr[al]);
                }
                if (l >= 0 && l + 1 < a.L) noise_of(n, l + 1, nz);
            }
            const double m = wave_max(d2m);
            double wmax = 0.0;
            {
                // workgroup max of the displacement (wave partials through dfe, free here)
                if ((tid & 63) == 0) dfe[tid >> 6] = m;
                __syncthreads();
                for (int v = 0; v < (int)(blockDim.x >> 6); ++v) wmax = fmax(wmax, dfe[v]);
            }
            if (!exchange_x(wmax)) { alive = false; break; }
            double gmax = 0.0;
            for (int v = 0; v < K; ++v) gmax = fmax(gmax, pv[v]);
            if (!built || !(4.0 * gmax <= a.skin * a.skin)) {
                if (NC > 0) {
                    for (int c = tid; c < NC; c += blockDim.x) cl.cnt[c] = 0;
                    __syncthreads();
                    for (int q = tid; q < N; q += blockDim.x) {
                        const int c = swl_cell_of(a, xs[q], xs[N + q], xs[2 * N + q]);
                        cl.cid[q] = (uint16_t)c;
                        atomicAdd(&cl.cnt[c], 1);
                    }
                    __syncthreads();
                    if (tid < 64) {
                        constexpr int per = kSweepMaxCells / 64;
                        int loc[per], sum = 0;
#pragma unroll
                        for (int k = 0; k < per; ++k) {
                            const int c = tid * per + k;
                            loc[k] = c < NC ? cl.cnt[c] : 0;
                            sum += loc[k];
                        }
                        int incl = sum;
#pragma unroll
                        for (int o = 1; o < 64; o <<= 1) {
                            const int v = __shfl_up(incl, o, 64);
                            if (tid >= o) incl += v;
                        }
                        int run = incl - sum;
#pragma unroll
                        for (int k = 0; k < per; ++k) {
                            const int c = tid * per + k;
                            if (c < NC) {
                                cl.start[c] = run;
                                cl.cnt[c] = run;
                            }
                            run += loc[k];
                        }
                        if (tid == 63) cl.start[NC] = incl;
                    }
                    __syncthreads();
                    for (int q = tid; q < N; q += blockDim.x) cl.atom[atomicAdd(&cl.cnt[cl.cid[q]], 1)] = (uint16_t)q;
                    __syncthreads();
                    for (int c = tid; c < NC; c += blockDim.x) {
                        const int bb = cl.start[c], e = cl.start[c + 1];
                        for (int q = bb + 1; q < e; ++q) {
                            const uint16_t v = cl.atom[q];
                            int r = q - 1;
                            while (r >= bb && cl.atom[r] > v) {
                                cl.atom[r + 1] = cl.atom[r];
                                --r;
                            }
                            cl.atom[r + 1] = v;
                        }
                    }
                    __syncthreads();
                }
                if (own) {
                    cn = swl_build_thread(a, xs, col, kMcLanes * A, cl, i, rcl2, overflow, h, kMcLanes);
#pragma unroll
                    for (int al = 0; al < 3; ++al) xr[al] = xo[al];
                }
                built = true;
                __syncthreads();
            }
            double acc = 0.0;
            if (own) mk = swl_rho_acc(a, xs, col, kMcLanes * A, i, cn, acc);
            acc = mc_lane_sum(acc);  // all parts of the list (the same sum in every lane)
            if (lead) put_tagged(a.gdfe + 2 * ((size_t)par * N + i), swl_dfe(a.fp, acc), b);
            if (!mc_get(dfe, a.gdfe + 2 * (size_t)par * N, N, nullptr, 0, pv, b, a)) { alive = false; break; }
            ++b;
            double fh[3] = {0.0, 0.0, 0.0};
            if (own) swl_force_thread(a, xs, dfe, col, kMcLanes * A, i, mk, fh);
#pragma unroll
            for (int al = 0; al < 3; ++al) fr[al] = mc_lane_sum(fh[al]);
            if (l >= 0)
#pragma unroll
                for (int al = 0; al < 3; ++al) pr[al] = pr[al] + hk * fr[al];
            par ^= 1;
            __syncthreads();  // xs / dfe reads done before the next step overwrites them
        }
        if (!alive) break;
        // slab end: cur_{n+1} = C(cur_n) (+ J_n) for own atoms; partial sums exchanged
        const size_t s = (size_t)(n - a.n_in);
        double d2 = 0.0, p2 = 0.0, fin = 0.0;
        if (own)
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                double xq = xo[al], pq = pr[al];
                if (a.mode == 1) {
                    xq += a.jq[al * SN + s * N + i];
                    pq += a.jp[al * SN + s * N + i];
                    const double pv = a.q_prev[((size_t)(n + 1) * 3 + al) * N + i];
                    if (lead) {
                        d2 += (xq - pv) * (xq - pv);
                        p2 += pv * pv;
                    }
                }
                if (lead) fin += xq * 0.0 + pq * 0.0;  // NaN/Inf propagate into fin
                xo[al] = xq;
                pr[al] = pq;
                if (lead) {
                    a.q_cur[((size_t)(n + 1) * 3 + al) * N + i] = xq;
                    a.p_cur[((size_t)(n + 1) * 3 + al) * N + i] = pq;
                }
            }
        {
            const double v0 = wave_sum(d2), v1 = wave_sum(p2), v2 = wave_sum(fin);
            if ((tid & 63) == 0) {
                dfe[3 * (tid >> 6)] = v0;
                dfe[3 * (tid >> 6) + 1] = v1;
                dfe[3 * (tid >> 6) + 2] = v2;
            }
            __syncthreads();
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
                s0 += dfe[3 * v];
                s1 += dfe[3 * v + 1];
                s2 += dfe[3 * v + 2];
            }
            if (tid == 0) {
                put_tagged(gpart(1) + 2 * w, s0, b);
                put_tagged(gpart(2) + 2 * w, s1, b);
                put_tagged(gpart(3) + 2 * w, s2, b);
            }
        }
        if (!mc_get(nullptr, nullptr, 0, gpart(1), 3 * K, pv, b, a)) { alive = false; break; }
        ++b;
        const double sfin = partial(3);
        if (!isfinite(sfin)) {
            bad = n;
            break;
        }
        if (a.mode == 1) {
            num += sqrt(partial(1));
            den += sqrt(partial(2));
            delta = den > 0.0 ? num / den : 0.0;
            if (delta > a.delta_expl) {
                nfi_new = max(n, a.n_win + 1);
                break;
            }
        }
        par ^= 1;
        __syncthreads();
    }
    if (overflow) a.out[3] = 1.0;
    if (w == 0 && tid == 0) {
        if (!alive) a.out[7] = 1.0;
        a.out[0] = delta;
        a.out[4] = num;
        a.out[5] = den;
        if (nfi_new >= 0) a.out[1] = (double)nfi_new;
        if (bad >= 0) a.out[2] = (double)bad;
        if (nfi_new >= 0 || bad >= 0 || !alive) a.out[6] = 1.0;
    }
}

size_t sweep_mc_lds_bytes(int N, int A) {
    return (size_t)N * 4 * sizeof(double) + 2 * sizeof(int) + (size_t)kSweepNbRows * kMcLanes * A * sizeof(uint16_t) + 4 +
           (2 * kSweepMaxCells + 1) * sizeof(int) + (size_t)N * 2 * sizeof(uint16_t) + 8;
}

// Gaussians of every (slab, step, atom) of a window: noise[s][l][al][i] for global step
// (n_in + s) L + l, drawn exactly as the batched propagators draw them.
__global__ void k_noise_table(int S, int L, int N, int n_in, uint64_t seed, uint64_t noise_id,
                              double *__restrict__ noise) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)S * L * N) return;
    const int i = (int)(q % N);
    const size_t sl = q / N;  // s * L + l
    const uint64_t gstep = (uint64_t)n_in * (uint64_t)L + (uint64_t)sl;
    double g0, g1, g2;
    sweep_gauss3(seed, noise_id, gstep, (uint64_t)i, g0, g1, g2);
    double *o = noise + sl * 3 * N + i;
    o[0] = g0;
    o[N] = g1;
    o[2 * N] = g2;
}

void launch_noise_table(int S, int L, int N, int n_in, uint64_t seed, uint64_t noise_id, double *noise,
                        hipStream_t st) {
    const size_t tot = (size_t)S * L * N;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_noise_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, L, N, n_in, seed,
                       noise_id, noise);
}

// End of slab n for the host-driven sweep of large systems: cur_{n+1} = state (+ J_n),
// written to the slab slot and back into the running state; partial sums of
// |cur - prev|^2, |prev|^2 and a non-finite probe into part[0..2] (one workgroup, fixed
// reduction order).  The running state xs, ps is [3][N]; the slot rows (qprev_next,
// qcur_next, pcur_next) have stride ld; the jump of row al is at jq[al jsa + s jss + i].
__global__ void __launch_bounds__(1024) k_slab_end(int N, int mode, size_t jsa, size_t jss, size_t s,
                                                   double *__restrict__ xs, double *__restrict__ ps,
                                                   const double *__restrict__ jq, const double *__restrict__ jp,
                                                   size_t ld, const double *__restrict__ qprev_next,
                                                   double *__restrict__ qcur_next, double *__restrict__ pcur_next,
                                                   double *__restrict__ part) {
    __shared__ double red[kSpillMax];
    double d2 = 0.0, p2 = 0.0, fin = 0.0;
    for (int i = threadIdx.x; i < N; i += kSweepThreads)
        for (int al = 0; al < 3; ++al) {
            double xq = xs[al * N + i], pq = ps[al * N + i];
            if (mode == 1) {
                xq += jq[al * jsa + s * jss + i];
                pq += jp[al * jsa + s * jss + i];
                const double pv = qprev_next[al * ld + i];
                d2 += (xq - pv) * (xq - pv);
                p2 += pv * pv;
            }
            fin += xq * 0.0 + pq * 0.0;
            xs[al * N + i] = xq;
            ps[al * N + i] = pq;
            qcur_next[al * ld + i] = xq;
            pcur_next[al * ld + i] = pq;
        }
    const double a = wg_sum(d2, red), b = wg_sum(p2, red), c = wg_sum(fin, red);
    if (threadIdx.x == 0) {
        part[0] = a;
        part[1] = b;
        part[2] = c;
    }
}

void launch_slab_end(int N, int mode, size_t jsa, size_t jss, size_t s, double *xs, double *ps, const double *jq,
                     const double *jp, size_t ld, const double *qprev_next, double *qcur_next, double *pcur_next,
                     double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_slab_end, dim3(1), dim3(kSweepThreads), 0, st, N, mode, jsa, jss, s, xs, ps, jq, jp, ld,
                       qprev_next, qcur_next, pcur_next, part);
}

// ---------------------------------------------------------------------------
// Batches of several systems, each with its own window [n_in_r, n_fi_r] of slabs.  The
// states of all systems share one slot layout [slot][3][ld] (system r's atoms at columns
// off[r] .. off[r+1]-1); the batched propagators see entry e = (system r_e, slab n_e) as
// a system of their own, entries back to back in the chunk's SoA arrays [3][Nc].
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_seg(const int *__restrict__ off, int n, int i) {
    int lo = 0, hi = n;  // largest s with off[s] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// prev := cur on the slots n_in_r .. n_fi_r of every system r (win[r] = (n_in, n_fi);
// an empty window, n_in = n_fi, copies nothing)
__global__ void k_copy_windows(int n_slots, int ld, int n_sys, const int *__restrict__ off,
                               const int2 *__restrict__ win, const double *__restrict__ q, const double *__restrict__ p,
                               double *__restrict__ qd, double *__restrict__ pd) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n_slots * 3 * ld) return;
    const int col = (int)(e % ld);
    const int slot = (int)(e / ((size_t)3 * ld));
    const int r = find_seg(off, n_sys, col);
    const int2 w = win[r];
    if (w.x < w.y && slot >= w.x && slot <= w.y) {
        qd[e] = q[e];
        pd[e] = p[e];
    }
}

// entries -> batch: out[al][j] = state[slot_e][al][col_e + j - off[e]] for the Nc atoms of
// a chunk of entries (src[e] = (slot_e, col_e, slot its jump goes to or -1, -), off = the
// chunk's atom offsets)
__global__ void k_entries_to_batch(int Nc, int n_ent, const int *__restrict__ off, const int4 *__restrict__ src,
                                   int ld, const double *__restrict__ state, double *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nc) return;
    const int e = find_seg(off, n_ent, j);
    const int4 sc = src[e];
    const size_t base = (size_t)sc.x * 3 * ld + sc.y + (j - off[e]);
#pragma unroll
    for (int al = 0; al < 3; ++al) out[(size_t)al * Nc + j] = state[base + (size_t)al * ld];
}

// jumps of a chunk into the slot layout: jump[dst_e][al][col_e + i] = f[al][j] - c[al][j]
// (entries with dst_e < 0 were propagated only to keep the launch shape fixed)
__global__ void k_batch_jumps_to_slots(int Nc, int n_ent, const int *__restrict__ off, const int4 *__restrict__ src,
                                       int ld, const double *__restrict__ f, const double *__restrict__ c,
                                       double *__restrict__ jump) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nc) return;
    const int e = find_seg(off, n_ent, j);
    const int4 sc = src[e];
    if (sc.z < 0) return;
    const size_t base = (size_t)sc.z * 3 * ld + sc.y + (j - off[e]);
#pragma unroll
    for (int al = 0; al < 3; ++al) jump[base + (size_t)al * ld] = f[(size_t)al * Nc + j] - c[(size_t)al * Nc + j];
}

void launch_copy_windows(int n_slots, int ld, int n_sys, const int *off, const int2 *win, const double *q,
                         const double *p, double *qd, double *pd, hipStream_t st) {
    const size_t tot = (size_t)n_slots * 3 * ld;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_copy_windows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_slots, ld, n_sys, off,
                       win, q, p, qd, pd);
}

void launch_entries_to_batch(int Nc, int n_ent, const int *off, const int4 *src, int ld, const double *state,
                             double *out, hipStream_t st) {
    if (Nc <= 0) return;
    hipLaunchKernelGGL(k_entries_to_batch, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, st, Nc, n_ent, off, src,
                       ld, state, out);
}

void launch_batch_jumps_to_slots(int Nc, int n_ent, const int *off, const int4 *src, int ld, const double *f,
                                 const double *c, double *jump, hipStream_t st) {
    if (Nc <= 0) return;
    hipLaunchKernelGGL(k_batch_jumps_to_slots, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, st, Nc, n_ent, off,
                       src, ld, f, c, jump);
}

// ---------------------------------------------------------------------------
// Device-resident adaptive driver: the branch logic and window bookkeeping of the
// adaptive algorithm for every replica, in device memory, between the launches of a
// round (start windows -> initialisation sweeps -> entries and windows of the corrected
// iteration -> ... -> corrected sweeps -> update).  act[k] is the replica of active slot
// k; tab_* and out_* are indexed by k, the state by replica.
// ---------------------------------------------------------------------------
// Window starts: a replica that needs a new time window gets [n_fi, min(N, n_fi + W)] and
// an initialisation sweep over it; the others get an empty sweep.
__global__ void k_drv_start(int Ra, const int *__restrict__ act, DrvState *__restrict__ st, int N, int W,
                            SweepArgs *__restrict__ tab, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ra) return;
    const int r = act[k];
    DrvState s = st[r];
    SweepArgs &a = tab[k];
    if (s.phase == DRV_NEW) {
        s.n_in = s.n_fi;
        s.n_fi = min(N, s.n_in + W);
        s.phase = DRV_ITER;
        st[r] = s;
        a.n_in = s.n_in;
        a.n_fi = s.n_fi;
    } else {
        a.n_in = a.n_fi = s.n_in;
    }
    a.n_win = a.n_in;
    double *o = out + 8 * (size_t)k;
    o[0] = 0.0;
    o[1] = (double)a.n_fi;
    o[2] = -1.0;
    for (int q = 3; q < 8; ++q) o[q] = 0.0;
}

// Corrected iteration of every iterating replica: its window (for the prev := cur copy),
// its sweep arguments, and the W entries (replica, slab) of its slot in the batch: slab
// n_in + s for s < n_fi - n_in, else a filler (slab n_in, jump discarded) that keeps the
// batch's shape fixed.  Threads: Ra * W entries, then R_all windows.
__global__ void k_drv_iter(int Ra, const int *__restrict__ act, int R_all, const DrvState *__restrict__ st, int W,
                           int L, size_t ld, const int *__restrict__ roff, int4 *__restrict__ ent,
                           int64_t *__restrict__ step0, SweepArgs *__restrict__ tab, double *__restrict__ out,
                           int2 *__restrict__ win, const double *__restrict__ jq, const double *__restrict__ jp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < Ra * W) {
        const int k = t / W, sl = t % W, r = act[k];
        const DrvState s = st[r];
        const bool live = s.phase == DRV_ITER && s.n_in + sl < s.n_fi;
        const int slab = live ? s.n_in + sl : s.n_in;
        ent[t] = make_int4(slab, roff[r], live ? slab : -1, 0);
        step0[t] = (int64_t)slab * L;
        if (sl == 0) {
            SweepArgs &a = tab[k];
            a.n_in = s.n_in;
            a.n_fi = s.phase == DRV_ITER ? s.n_fi : s.n_in;
            a.n_win = s.n_in;
            a.jq = jq + (size_t)s.n_in * 3 * ld + roff[r];
            a.jp = jp + (size_t)s.n_in * 3 * ld + roff[r];
            double *o = out + 8 * (size_t)k;
            o[0] = 0.0;
            o[1] = (double)a.n_fi;
            o[2] = -1.0;
            for (int q = 3; q < 8; ++q) o[q] = 0.0;
        }
    } else if (t < Ra * W + R_all) {
        const int r = t - Ra * W;
        const DrvState s = st[r];
        win[r] = s.phase == DRV_ITER ? make_int2(s.n_in, s.n_fi) : make_int2(0, 0);
    }
}

// After the corrected sweeps: log the iteration and take the adaptive algorithm's next
// step (stay on the window while delta_conv <= delta <= delta_expl; otherwise the run is
// over at n_fi = N, a converged window starts the next one, and an exploded one was
// shortened by the sweep and is iterated again).  A non-finite state or a list overflow
// stops the replica and is recorded in err (bit 1 overflow, bit 2 non-finite).
__global__ void k_drv_update(int Ra, const int *__restrict__ act, DrvState *__restrict__ st,
                             const double *__restrict__ out, double dconv, double dexpl, int N, int max_log,
                             int4 *__restrict__ logi, double *__restrict__ logd, int *__restrict__ err) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ra) return;
    const int r = act[k];
    DrvState s = st[r];
    if (s.phase != DRV_ITER) return;
    const double *o = out + 8 * (size_t)k;
    if (o[3] != 0.0 || o[2] >= 0.0) {
        s.err = o[3] != 0.0 ? 1 : 2;
        s.bad_slab = o[2] >= 0.0 ? (int)o[2] : -1;
        s.phase = DRV_DONE;
        atomicOr(err, s.err);
        st[r] = s;
        return;
    }
    const double delta = o[0];
    const int window = s.n_fi, after = (int)o[1];
    if (s.nlog < max_log) {
        logi[(size_t)r * max_log + s.nlog] = make_int4(s.n_in, window, after, 0);
        logd[(size_t)r * max_log + s.nlog] = delta;
    }
    ++s.nlog;
    s.n_fi = after;
    s.delta = delta;
    if (!(dconv <= delta && delta <= dexpl)) {
        if (s.n_fi >= N) s.phase = DRV_DONE;
        else if (delta < dexpl) s.phase = DRV_NEW;
        // else: the window was shortened; iterate on it again
    }
    st[r] = s;
}

void launch_drv_start(int Ra, const int *act, DrvState *st, int N, int W, void *tab, double *out, hipStream_t st_) {
    if (Ra <= 0) return;
    hipLaunchKernelGGL(k_drv_start, dim3((Ra + 63) / 64), dim3(64), 0, st_, Ra, act, st, N, W, (SweepArgs *)tab, out);
}

void launch_drv_iter(int Ra, const int *act, int R_all, const DrvState *st, int W, int L, size_t ld, const int *roff,
                     int4 *ent, int64_t *step0, void *tab, double *out, int2 *win, const double *jq, const double *jp,
                     hipStream_t s_) {
    const int tot = Ra * W + R_all;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_drv_iter, dim3((tot + 255) / 256), dim3(256), 0, s_, Ra, act, R_all, st, W, L, ld, roff, ent,
                       step0, (SweepArgs *)tab, out, win, jq, jp);
}

void launch_drv_update(int Ra, const int *act, DrvState *st, const double *out, double dconv, double dexpl, int N,
                       int max_log, int4 *logi, double *logd, int *err, hipStream_t s_) {
    if (Ra <= 0) return;
    hipLaunchKernelGGL(k_drv_update, dim3((Ra + 63) / 64), dim3(64), 0, s_, Ra, act, st, out, dconv, dexpl, N,
                       max_log, logi, logd, err);
}

// LDS sweeps of n systems at once (tab: device [n] arguments, one workgroup each; every
// system fits the LDS-resident sweep, max_atoms the largest)
void launch_coarse_sweep_multi(const void *tab, int n, int max_atoms, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_coarse_sweep_lds_multi, dim3(n), dim3(kSweepThreads), sweep_lds_bytes(max_atoms), st,
                       (const SweepArgs *)tab);
}

bool sweep_fits_lds(int N) { return N <= kSweepLdsMaxAtoms && sweep_lds_bytes(N) <= 160 * 1024; }

// workgroups of the multi-workgroup sweep for N atoms (0: not used); want > 0 asks for
// that many, granted when they fit (at most 64, at most kMcMaxAtoms atoms per workgroup);
// built in: the fewest from 8 up that fit
int sweep_mc_workgroups(int N, int want) {
    if (N < 512 || N > 65535) return 0;
    auto fits = [N](int K) {
        const int A = (N + K - 1) / K;
        return K <= 64 && A <= kMcMaxAtoms && sweep_mc_lds_bytes(N, A) + kMcStaticLds <= 160 * 1024;
    };
    if (want > 0 && fits(want)) return want;
    // built in: the fewest from 8 up with at most 64 atoms each (pipelined iterations of
    // 64 slabs of 1025 atoms, where the sweep sets the pace: 2.7 % faster with 17
    // workgroups than with 9 of up to 128 atoms, widths 17 to 20 within 0.5 %), else
    // with at most 128 atoms each
    for (int K = 8; K <= 64; ++K)
        if (fits(K) && (N + K - 1) / K <= 64) return K;
    for (int K = 8; K <= 64; ++K)
        if (fits(K)) return K;
    return 0;
}

// ---------------------------------------------------------------------------
void launch_slabs_to_batch(int S, int N, const double *slots, double *out, hipStream_t st) {
    const size_t tot = (size_t)3 * S * N;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_slabs_to_batch, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, N, slots, out);
}

void launch_jumps(size_t n, double *a, const double *b, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_jumps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b);
}

static SweepArgs sweep_args(const SweepLaunch &s) {
    SweepArgs a;
    a.N = s.N;
    a.Lx = s.box[0];
    a.Ly = s.box[1];
    a.Lz = s.box[2];
    a.iLx = 1.0 / s.box[0];
    a.iLy = 1.0 / s.box[1];
    a.iLz = 1.0 / s.box[2];
    a.noise = s.noise;
    a.fp = s.fp;
    a.skin = s.skin;
    a.dt = s.dt;
    a.c1 = s.c1;
    a.mass = s.mass;
    a.sig = s.sig;
    a.seed = s.seed;
    a.noise_id = s.noise_id;
    a.L = s.L;
    a.n_in = s.n_in;
    a.n_fi = s.n_fi;
    a.n_win = s.n_win;
    a.ncx = s.ncx;
    a.ncy = s.ncy;
    a.ncz = s.ncz;
    a.K = s.K;
    a.A = s.A;
    a.gx = s.gx;
    a.gdfe = s.gdfe;
    a.gpart = s.gpart;
    a.abort = s.abort;
    a.mode = s.mode;
    a.delta_expl = s.delta_expl;
    a.q_cur = s.q_cur;
    a.p_cur = s.p_cur;
    a.q_prev = s.q_prev;
    a.p_prev = s.p_prev;
    a.jq = s.jq;
    a.jp = s.jp;
    // one system: slots [slot][3][N], jumps [3][S N]
    a.ld = (size_t)s.N;
    a.jsa = (size_t)(s.n_fi - s.n_in) * s.N;
    a.jss = (size_t)s.N;
    a.out = s.out;
    return a;
}

size_t sweep_args_bytes() { return sizeof(SweepArgs); }

void fill_sweep_args(const SweepLaunch &s, size_t ld, size_t jsa, size_t jss, void *dst) {
    SweepArgs a = sweep_args(s);
    a.ld = ld;
    a.jsa = jsa;
    a.jss = jss;
    *(SweepArgs *)dst = a;
}

void launch_coarse_sweep(const SweepLaunch &s, hipStream_t st) {
    const SweepArgs a = sweep_args(s);
    if (s.K > 0) {
        // at least 81 KB of LDS so that no two of the workgroups share a CU
        const size_t lds = std::max<size_t>(sweep_mc_lds_bytes(s.N, s.A), 81 * 1024);
        const int T = (kMcLanes * s.A + 63) / 64 * 64;
        hipLaunchKernelGGL(k_coarse_sweep_mc, dim3(s.K), dim3(T), lds, st, a);
    } else {
        hipLaunchKernelGGL(k_coarse_sweep_lds, dim3(1), dim3(kSweepThreads), sweep_lds_bytes(s.N), st, a);
    }
}

void sweep_init_attributes() {
    (void)hipFuncSetAttribute((const void *)k_coarse_sweep_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_coarse_sweep_mc, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - kMcStaticLds);
    (void)hipFuncSetAttribute((const void *)k_coarse_sweep_lds_multi, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

}  // namespace snapmd
