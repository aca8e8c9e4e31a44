// Parareal pieces of snapmd (gfx950, FP64).
//
//   k_slabs_to_batch : slab states [slot][3][N] -> batch layout [3][S*N] (S slabs)
//   k_jumps          : J = F(prev) - C(prev) in batch layout (in place into the fine copy)
//   k_coarse_sweep   : the sequential part of a parareal iteration in ONE persistent
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

// block-wide reduction helpers (1024 threads, red has 1024 doubles)
__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kSweepThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_max(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kSweepThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

struct SweepArgs {
    int N;
    double Lx, Ly, Lz, iLx, iLy, iLz;
    FsParams fp;
    double skin;
    double dt, c1, mass, sig;
    uint64_t seed, noise_id;
    int L, n_in, n_fi, mode;  // mode 0: initialise (no jumps), 1: corrected sweep
    double delta_expl;
    double *q_cur, *p_cur;                 // [slot][3][N]
    const double *q_prev, *p_prev;         // [slot][3][N] (mode 1)
    const double *jq, *jp;                 // [3][S*N], S = n_fi - n_in (mode 1)
    double *wx, *wp, *wf, *wrho, *xref;    // [3N], [3N], [3N], [N], [3N]
    int *nbr, *cnt;                        // [N][kMaxNeigh], [N]
    double *out;                           // [0] delta, [1] n_fi after, [2] bad slab (-1 none), [3] overflow
    const double *noise;                   // [S][L][3][N] Gaussians of the window's slabs
};

__device__ void sweep_build(const SweepArgs &a) {
    const int N = a.N;
    const double rc = fmax(a.fp.d, a.fp.c) + a.skin, rc2 = rc * rc;
    for (int i = threadIdx.x; i < N; i += kSweepThreads) {
        const double xi = a.wx[i], yi = a.wx[N + i], zi = a.wx[2 * N + i];
        int c = 0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            const double dx = mimg_s(a.wx[j] - xi, a.Lx, a.iLx), dy = mimg_s(a.wx[N + j] - yi, a.Ly, a.iLy),
                         dz = mimg_s(a.wx[2 * N + j] - zi, a.Lz, a.iLz);
            if (dx * dx + dy * dy + dz * dz < rc2) {
                if (c < kMaxNeigh) a.nbr[(size_t)i * kMaxNeigh + c] = j;
                ++c;
            }
        }
        if (c > kMaxNeigh) { a.out[3] = 1.0; c = kMaxNeigh; }
        a.cnt[i] = c;
        a.xref[i] = xi; a.xref[N + i] = yi; a.xref[2 * N + i] = zi;
    }
}

// Finnis-Sinclair force on every atom into wf (same expressions as the batched kernels).
__device__ void sweep_force(const SweepArgs &a) {
    const int N = a.N;
    const FsParams fp = a.fp;
    const double d2c = fp.d * fp.d, rc2f = fmax(fp.d, fp.c) * fmax(fp.d, fp.c);
    for (int i = threadIdx.x; i < N; i += kSweepThreads) {
        const double xi = a.wx[i], yi = a.wx[N + i], zi = a.wx[2 * N + i];
        double acc = 0.0;
        for (int t = 0; t < a.cnt[i]; ++t) {
            const int j = a.nbr[(size_t)i * kMaxNeigh + t];
            const double dx = mimg_s(a.wx[j] - xi, a.Lx, a.iLx), dy = mimg_s(a.wx[N + j] - yi, a.Ly, a.iLy),
                         dz = mimg_s(a.wx[2 * N + j] - zi, a.Lz, a.iLz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= d2c) continue;
            const double r = sqrt(r2);
            if (r < fp.d) acc += (r - fp.d) * (r - fp.d);
        }
        a.wrho[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += kSweepThreads) {
        const double xi = a.wx[i], yi = a.wx[N + i], zi = a.wx[2 * N + i];
        const double ri = a.wrho[i];
        const double dFi = ri > 0.0 ? -fp.A / (2.0 * sqrt(ri)) : 0.0;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int t = 0; t < a.cnt[i]; ++t) {
            const int j = a.nbr[(size_t)i * kMaxNeigh + t];
            const double dx = mimg_s(a.wx[j] - xi, a.Lx, a.iLx), dy = mimg_s(a.wx[N + j] - yi, a.Ly, a.iLy),
                         dz = mimg_s(a.wx[2 * N + j] - zi, a.Lz, a.iLz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= rc2f) continue;
            const double r = sqrt(r2);
            double dEdr = 0.0;
            if (r < fp.c) {
                const double tt = r - fp.c, poly = fp.c0 + r * (fp.c1 + r * fp.c2);
                dEdr += 2.0 * tt * poly + tt * tt * (fp.c1 + 2.0 * fp.c2 * r);
            }
            if (r < fp.d) {
                const double rj = a.wrho[j];
                const double dFj = rj > 0.0 ? -fp.A / (2.0 * sqrt(rj)) : 0.0;
                dEdr += (dFi + dFj) * 2.0 * (r - fp.d);
            }
            if (r < fp.c || r < fp.d) {
                const double w = dEdr / r;
                fx += w * dx;
                fy += w * dy;
                fz += w * dz;
            }
        }
        a.wf[i] = fx;
        a.wf[N + i] = fy;
        a.wf[2 * N + i] = fz;
    }
    __syncthreads();
}

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

__global__ void __launch_bounds__(1024) k_coarse_sweep(SweepArgs a) {
    __shared__ double red[kSweepThreads];
    const int N = a.N;
    const size_t SN = (size_t)(a.n_fi - a.n_in) * N;
    for (int i = threadIdx.x; i < N; i += kSweepThreads)
        for (int al = 0; al < 3; ++al) {
            a.wx[al * N + i] = a.q_cur[((size_t)a.n_in * 3 + al) * N + i];
            a.wp[al * N + i] = a.p_cur[((size_t)a.n_in * 3 + al) * N + i];
        }
    __syncthreads();
    double num = 0.0, den = 0.0, delta = 0.0;
    int nfi_new = a.n_fi, bad = -1;
    const double hk = 0.5 * a.dt / SW_MVV2E, hd = 0.5 * a.dt / a.mass;
    for (int n = a.n_in; n < a.n_fi; ++n) {
        sweep_build(a);
        __syncthreads();
        sweep_force(a);
        for (int l = 0; l < a.L; ++l) {
            double dmax = 0.0;
            for (int i = threadIdx.x; i < N; i += kSweepThreads) {
                double g[3];
                const double *gz = a.noise + ((size_t)((n - a.n_in) * a.L + l) * 3) * N + i;
                g[0] = gz[0];
                g[1] = gz[N];
                g[2] = gz[2 * N];
                double d2 = 0.0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    double pp = a.wp[al * N + i] + hk * a.wf[al * N + i];
                    double xx = a.wx[al * N + i] + hd * pp;
                    pp = a.c1 * pp + a.sig * g[al];
                    xx = xx + hd * pp;
                    a.wp[al * N + i] = pp;
                    a.wx[al * N + i] = xx;
                    const double dd = xx - a.xref[al * N + i];
                    d2 += dd * dd;
                }
                dmax = fmax(dmax, d2);
            }
            const double m = block_max(dmax, red);  // includes the barrier before the list is read
            if (4.0 * m > a.skin * a.skin) {
                sweep_build(a);
                __syncthreads();
            }
            sweep_force(a);
            for (int q = threadIdx.x; q < 3 * N; q += kSweepThreads) a.wp[q] = a.wp[q] + hk * a.wf[q];
            __syncthreads();
        }
        // slab end: cur_{n+1} = C(cur_n) (+ J_n)
        const size_t s = (size_t)(n - a.n_in);
        double d2 = 0.0, p2 = 0.0, fin = 0.0;
        for (int i = threadIdx.x; i < N; i += kSweepThreads)
            for (int al = 0; al < 3; ++al) {
                double xq = a.wx[al * N + i], pq = a.wp[al * N + i];
                if (a.mode == 1) {
                    xq += a.jq[al * SN + s * N + i];
                    pq += a.jp[al * SN + s * N + i];
                    const double pv = a.q_prev[((size_t)(n + 1) * 3 + al) * N + i];
                    d2 += (xq - pv) * (xq - pv);
                    p2 += pv * pv;
                }
                fin += xq * 0.0 + pq * 0.0;  // NaN/Inf propagate into fin
                a.wx[al * N + i] = xq;
                a.wp[al * N + i] = pq;
                a.q_cur[((size_t)(n + 1) * 3 + al) * N + i] = xq;
                a.p_cur[((size_t)(n + 1) * 3 + al) * N + i] = pq;
            }
        const double sfin = block_sum(fin, red);
        if (!isfinite(sfin)) {
            bad = n;
            break;
        }
        if (a.mode == 1) {
            const double sd = block_sum(d2, red), sp = block_sum(p2, red);
            num += sqrt(sd);
            den += sqrt(sp);
            delta = den > 0.0 ? num / den : 0.0;
            if (delta > a.delta_expl) {
                nfi_new = max(n, a.n_in + 1);
                break;
            }
        }
    }
    if (threadIdx.x == 0) {
        a.out[0] = delta;
        a.out[1] = (double)nfi_new;
        a.out[2] = (double)bad;
    }
}

// ---------------------------------------------------------------------------
// LDS-resident sweep for small systems (N <= kSweepLdsMaxAtoms): positions, rho and a
// uint16 Verlet list live in LDS, momenta / forces / reference positions of the (at
// most kSweepAtomsPerThread) atoms a thread owns live in its registers.
// ---------------------------------------------------------------------------
constexpr int kSweepLdsNeigh = 40;
constexpr int kSweepAtomsPerThread = 2;
constexpr int kSweepLdsMaxAtoms = kSweepThreads * kSweepAtomsPerThread;

size_t sweep_lds_bytes(int N) {
    return (size_t)N * (3 * sizeof(double) + sizeof(double) + kSweepLdsNeigh * sizeof(uint16_t)) +
           kSweepThreads * sizeof(double);
}

using SwReg = double[kSweepAtomsPerThread][3];

__device__ __forceinline__ void swl_build(const SweepArgs &a, const double *__restrict__ xs, uint16_t *__restrict__ nb,
                                          int (&cn)[kSweepAtomsPerThread], SwReg &xr, int &overflow) {
    const int N = a.N, tid = threadIdx.x;
    const double rcl = fmax(a.fp.d, a.fp.c) + a.skin, rcl2 = rcl * rcl;
#pragma unroll
    for (int q = 0; q < kSweepAtomsPerThread; ++q) {
        const int i = tid + q * kSweepThreads;
        if (i >= N) continue;
        const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
        int c = 0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            const double dx = mimg_s(xs[j] - xi, a.Lx, a.iLx), dy = mimg_s(xs[N + j] - yi, a.Ly, a.iLy),
                         dz = mimg_s(xs[2 * N + j] - zi, a.Lz, a.iLz);
            if (dx * dx + dy * dy + dz * dz < rcl2) {
                if (c < kSweepLdsNeigh) nb[c * N + i] = (uint16_t)j;
                ++c;
            }
        }
        if (c > kSweepLdsNeigh) {
            overflow = 1;
            c = kSweepLdsNeigh;
        }
        cn[q] = c;
        xr[q][0] = xi;
        xr[q][1] = yi;
        xr[q][2] = zi;
    }
}

// Embedding derivative F'(rho) = -A / (2 sqrt(rho)) of every atom into LDS, barrier,
// forces into registers, barrier.  Neighbour loops are unrolled by 4 so that the LDS
// reads of independent neighbours overlap.
__device__ __forceinline__ void swl_force(const SweepArgs &a, const double *__restrict__ xs, double *__restrict__ dfe,
                                          const uint16_t *__restrict__ nb, const int (&cn)[kSweepAtomsPerThread],
                                          SwReg &fr) {
    const int N = a.N, tid = threadIdx.x;
    const FsParams fp = a.fp;
    const double d2c = fp.d * fp.d, rc2f = fmax(fp.d, fp.c) * fmax(fp.d, fp.c);
#pragma unroll
    for (int q = 0; q < kSweepAtomsPerThread; ++q) {
        const int i = tid + q * kSweepThreads;
        if (i >= N) continue;
        const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
        double acc = 0.0;
        const int c = cn[q];
        for (int t0 = 0; t0 < c; t0 += 4) {
            int jj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) jj[u] = (t0 + u < c) ? (int)nb[(t0 + u) * N + i] : i;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = jj[u];
                const double dx = mimg_s(xs[j] - xi, a.Lx, a.iLx), dy = mimg_s(xs[N + j] - yi, a.Ly, a.iLy),
                             dz = mimg_s(xs[2 * N + j] - zi, a.Lz, a.iLz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (j == i || r2 >= d2c) continue;
                const double r = sqrt(r2);
                acc += (r - fp.d) * (r - fp.d);
            }
        }
        dfe[i] = acc > 0.0 ? -fp.A / (2.0 * sqrt(acc)) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSweepAtomsPerThread; ++q) {
        const int i = tid + q * kSweepThreads;
        if (i >= N) continue;
        const double xi = xs[i], yi = xs[N + i], zi = xs[2 * N + i];
        const double dFi = dfe[i];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        const int c = cn[q];
        for (int t0 = 0; t0 < c; t0 += 4) {
            int jj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) jj[u] = (t0 + u < c) ? (int)nb[(t0 + u) * N + i] : i;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = jj[u];
                const double dx = mimg_s(xs[j] - xi, a.Lx, a.iLx), dy = mimg_s(xs[N + j] - yi, a.Ly, a.iLy),
                             dz = mimg_s(xs[2 * N + j] - zi, a.Lz, a.iLz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (j == i || r2 >= rc2f) continue;
                const double r = sqrt(r2);
                double dEdr = 0.0;
                if (r < fp.c) {
                    const double tt = r - fp.c, poly = fp.c0 + r * (fp.c1 + r * fp.c2);
                    dEdr += 2.0 * tt * poly + tt * tt * (fp.c1 + 2.0 * fp.c2 * r);
                }
                if (r < fp.d) dEdr += (dFi + dfe[j]) * 2.0 * (r - fp.d);
                const double w = dEdr / r;
                fx += w * dx;
                fy += w * dy;
                fz += w * dz;
            }
        }
        fr[q][0] = fx;
        fr[q][1] = fy;
        fr[q][2] = fz;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_coarse_sweep_lds(SweepArgs a) {
    extern __shared__ double sm[];
    const int N = a.N;
    double *red = sm;                                      // [1024]
    double *xs = sm + kSweepThreads;                       // [3][N]
    double *rho = xs + 3 * N;                              // [N]
    uint16_t *nb = reinterpret_cast<uint16_t *>(rho + N);  // [kSweepLdsNeigh][N]
    const int tid = threadIdx.x;
    const size_t SN = (size_t)(a.n_fi - a.n_in) * N;
    double pr[kSweepAtomsPerThread][3], fr[kSweepAtomsPerThread][3], xr[kSweepAtomsPerThread][3];
    int cn[kSweepAtomsPerThread];
#pragma unroll
    for (int q = 0; q < kSweepAtomsPerThread; ++q) {
        const int i = tid + q * kSweepThreads;
        cn[q] = 0;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            fr[q][al] = 0.0;
            xr[q][al] = 0.0;
            pr[q][al] = 0.0;
            if (i < N) {
                xs[al * N + i] = a.q_cur[((size_t)a.n_in * 3 + al) * N + i];
                pr[q][al] = a.p_cur[((size_t)a.n_in * 3 + al) * N + i];
            }
        }
    }
    __syncthreads();
    int overflow = 0;
    double num = 0.0, den = 0.0, delta = 0.0;
    int nfi_new = a.n_fi, bad = -1;
    const double hk = 0.5 * a.dt / SW_MVV2E, hd = 0.5 * a.dt / a.mass;
    bool built = false;
    for (int n = a.n_in; n < a.n_fi; ++n) {
        // the list is rebuilt only if some atom moved more than skin/2 since the last build
        double dmax0 = 0.0;
#pragma unroll
        for (int q = 0; q < kSweepAtomsPerThread; ++q) {
            const int i = tid + q * kSweepThreads;
            if (i >= N) continue;
            double d2 = 0.0;
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const double dd = xs[al * N + i] - xr[q][al];
                d2 += dd * dd;
            }
            dmax0 = fmax(dmax0, d2);
        }
        const double m0 = block_max(dmax0, red);
        if (!built || !(4.0 * m0 <= a.skin * a.skin)) {
            swl_build(a, xs, nb, cn, xr, overflow);
            __syncthreads();
            built = true;
        }
        swl_force(a, xs, rho, nb, cn, fr);
        for (int l = 0; l < a.L; ++l) {
            double dmax = 0.0;
#pragma unroll
            for (int q = 0; q < kSweepAtomsPerThread; ++q) {
                const int i = tid + q * kSweepThreads;
                if (i >= N) continue;
                double g[3];
                const double *gz = a.noise + ((size_t)((n - a.n_in) * a.L + l) * 3) * N + i;
                g[0] = gz[0];
                g[1] = gz[N];
                g[2] = gz[2 * N];
                double d2 = 0.0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    double pp = pr[q][al] + hk * fr[q][al];
                    double xx = xs[al * N + i] + hd * pp;
                    pp = a.c1 * pp + a.sig * g[al];
                    xx = xx + hd * pp;
                    pr[q][al] = pp;
                    xs[al * N + i] = xx;
                    const double dd = xx - xr[q][al];
                    d2 += dd * dd;
                }
                dmax = fmax(dmax, d2);
            }
            const double m = block_max(dmax, red);
            if (4.0 * m > a.skin * a.skin) {
                swl_build(a, xs, nb, cn, xr, overflow);
                __syncthreads();
            }
            swl_force(a, xs, rho, nb, cn, fr);
#pragma unroll
            for (int q = 0; q < kSweepAtomsPerThread; ++q)
#pragma unroll
                for (int al = 0; al < 3; ++al) pr[q][al] = pr[q][al] + hk * fr[q][al];
        }
        const size_t s = (size_t)(n - a.n_in);
        double d2 = 0.0, p2 = 0.0, fin = 0.0;
#pragma unroll
        for (int q = 0; q < kSweepAtomsPerThread; ++q) {
            const int i = tid + q * kSweepThreads;
            if (i >= N) continue;
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                double xq = xs[al * N + i], pq = pr[q][al];
                if (a.mode == 1) {
                    xq += a.jq[al * SN + s * N + i];
                    pq += a.jp[al * SN + s * N + i];
                    const double pv = a.q_prev[((size_t)(n + 1) * 3 + al) * N + i];
                    d2 += (xq - pv) * (xq - pv);
                    p2 += pv * pv;
                }
                fin += xq * 0.0 + pq * 0.0;
                xs[al * N + i] = xq;
                pr[q][al] = pq;
                a.q_cur[((size_t)(n + 1) * 3 + al) * N + i] = xq;
                a.p_cur[((size_t)(n + 1) * 3 + al) * N + i] = pq;
            }
        }
        const double sfin = block_sum(fin, red);
        if (!isfinite(sfin)) {
            bad = n;
            break;
        }
        if (a.mode == 1) {
            const double sd = block_sum(d2, red), sp = block_sum(p2, red);
            num += sqrt(sd);
            den += sqrt(sp);
            delta = den > 0.0 ? num / den : 0.0;
            if (delta > a.delta_expl) {
                nfi_new = max(n, a.n_in + 1);
                break;
            }
        }
    }
    if (overflow) a.out[3] = 1.0;
    if (tid == 0) {
        a.out[0] = delta;
        a.out[1] = (double)nfi_new;
        a.out[2] = (double)bad;
    }
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
// reduction order).
__global__ void __launch_bounds__(1024) k_slab_end(int N, int mode, size_t SN, size_t s, double *__restrict__ xs,
                                                   double *__restrict__ ps, const double *__restrict__ jq,
                                                   const double *__restrict__ jp,
                                                   const double *__restrict__ qprev_next,
                                                   double *__restrict__ qcur_next, double *__restrict__ pcur_next,
                                                   double *__restrict__ part) {
    __shared__ double red[kSweepThreads];
    double d2 = 0.0, p2 = 0.0, fin = 0.0;
    for (int i = threadIdx.x; i < N; i += kSweepThreads)
        for (int al = 0; al < 3; ++al) {
            double xq = xs[al * N + i], pq = ps[al * N + i];
            if (mode == 1) {
                xq += jq[al * SN + s * N + i];
                pq += jp[al * SN + s * N + i];
                const double pv = qprev_next[al * N + i];
                d2 += (xq - pv) * (xq - pv);
                p2 += pv * pv;
            }
            fin += xq * 0.0 + pq * 0.0;
            xs[al * N + i] = xq;
            ps[al * N + i] = pq;
            qcur_next[al * N + i] = xq;
            pcur_next[al * N + i] = pq;
        }
    const double a = block_sum(d2, red), b = block_sum(p2, red), c = block_sum(fin, red);
    if (threadIdx.x == 0) {
        part[0] = a;
        part[1] = b;
        part[2] = c;
    }
}

void launch_slab_end(int N, int mode, size_t SN, size_t s, double *xs, double *ps, const double *jq, const double *jp,
                     const double *qprev_next, double *qcur_next, double *pcur_next, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_slab_end, dim3(1), dim3(kSweepThreads), 0, st, N, mode, SN, s, xs, ps, jq, jp, qprev_next,
                       qcur_next, pcur_next, part);
}

bool sweep_fits_lds(int N) { return N <= kSweepLdsMaxAtoms && sweep_lds_bytes(N) <= 160 * 1024; }

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

void launch_coarse_sweep(const SweepLaunch &s, hipStream_t st) {
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
    a.mode = s.mode;
    a.delta_expl = s.delta_expl;
    a.q_cur = s.q_cur;
    a.p_cur = s.p_cur;
    a.q_prev = s.q_prev;
    a.p_prev = s.p_prev;
    a.jq = s.jq;
    a.jp = s.jp;
    a.wx = s.wx;
    a.wp = s.wp;
    a.wf = s.wf;
    a.wrho = s.wrho;
    a.xref = s.xref;
    a.nbr = s.nbr;
    a.cnt = s.cnt;
    a.out = s.out;
    if (sweep_fits_lds(s.N)) {
        hipLaunchKernelGGL(k_coarse_sweep_lds, dim3(1), dim3(kSweepThreads), sweep_lds_bytes(s.N), st, a);
    } else {
        hipLaunchKernelGGL(k_coarse_sweep, dim3(1), dim3(kSweepThreads), 0, st, a);
    }
}

void sweep_init_attributes() {
    (void)hipFuncSetAttribute((const void *)k_coarse_sweep_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

}  // namespace snapmd
