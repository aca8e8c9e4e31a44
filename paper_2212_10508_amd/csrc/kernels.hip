// HIP kernels of snapmd for gfx950 (CDNA4), FP64 throughout.
//
// Per force evaluation of a ragged batch (atoms of all systems back to back):
//   neighbours : k_neigh_build (brute force within the atom's own system, minimum
//                image) -> k_scan (prefix sums) -> k_compact (atom-major pair list,
//                CSR, and the index of the opposite pair)
//   FS EAM     : k_fs_rho -> k_fs_force (deterministic gather over the full list)
//   SNAP       : k_pair_ell (a, b, f_c once per pair, slot-major) -> k_density<J>
//                (u, lane = atom, one column chain of the Wigner-D polynomials per wave)
//                -> k_adjoint (Y by the coupling program, energy by Euler's identity)
//                -> k_dedr<J> (per pair dE_i/dr_ij = Re sum conj(Y~) d(f_c P), geometry
//                again from the positions) -> k_gather (F_k = sum over pairs
//                (g_kj - g_jk), no atomics, deterministic)
//   BAOAB      : k_baoab_pre (B A O A with Philox4x64-10 Gaussians; the SNAP gather opens
//                the following steps itself) / closing B in k_gather or k_fs_force
//   BBK        : k_bbk_pre / k_bbk_post (the paper's modified BBK scheme)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "kernels.h"
#include "snapmd_internal.h"

namespace snapmd {

#define KB_EV 8.617333262145179e-5
#define MVV2E 1.0364269652680506e-4

__device__ __forceinline__ double mimg(double d, double L, double iL) { return d - L * rint(d * iL); }

// ---------------------------------------------------------------------------
// Neighbour lists
// ---------------------------------------------------------------------------
// Candidate j of atom i: minimum image, squared distance below rc2.
__device__ __forceinline__ void nb_try(int i, int j, double xi, double yi, double zi, const double *__restrict__ x,
                                       int N, double Lx, double Ly, double Lz, double iLx, double iLy, double iLz,
                                       double rc2, int *__restrict__ nbr, int &c) {
    const double dx = mimg(x[j] - xi, Lx, iLx), dy = mimg(x[N + j] - yi, Ly, iLy), dz = mimg(x[2 * N + j] - zi, Lz, iLz);
    if (dx * dx + dy * dy + dz * dz < rc2) {
        if (c < kMaxNeigh) nbr[(size_t)i * kMaxNeigh + c] = j;
        ++c;
    }
}

// Full list of atom i: with cells (27-cell stencil of its system's grid, atoms of a cell
// in ascending index order) when the system has >= 3 cells per edge, else all atoms of
// its system.
__global__ void k_neigh_build(int N, int n_sys, const int *__restrict__ off, const double *__restrict__ box,
                              const double *__restrict__ x, double rc2, int *__restrict__ nbr,
                              int *__restrict__ cnt, int *__restrict__ status, const int *__restrict__ flag,
                              double *__restrict__ xref, const int4 *__restrict__ cells,
                              const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                              const int *__restrict__ cell_atoms) {
    if (*flag == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = sys_of(off, n_sys, i);
    const int j0 = off[s], j1 = off[s + 1];
    const double Lx = box[3 * s], Ly = box[3 * s + 1], Lz = box[3 * s + 2];
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    int c = 0;
    const int4 ci = cells ? cells[s] : make_int4(0, 0, 0, 0);
    if (ci.x >= 3) {
        const int me = cell_of[i] - ci.w;
        const int iz = me % ci.z, iy = (me / ci.z) % ci.y, ix = me / (ci.z * ci.y);
        for (int ax = -1; ax <= 1; ++ax) {
            const int cx = (ix + ax + ci.x) % ci.x;
            for (int ay = -1; ay <= 1; ++ay) {
                const int cy = (iy + ay + ci.y) % ci.y;
                for (int az = -1; az <= 1; ++az) {
                    const int cz = (iz + az + ci.z) % ci.z;
                    const int cc = ci.w + (cx * ci.y + cy) * ci.z + cz;
                    for (int q = cell_start[cc]; q < cell_start[cc + 1]; ++q) {
                        const int j = cell_atoms[q];
                        if (j != i) nb_try(i, j, xi, yi, zi, x, N, Lx, Ly, Lz, iLx, iLy, iLz, rc2, nbr, c);
                    }
                }
            }
        }
    } else {
        for (int j = j0; j < j1; ++j)
            if (j != i) nb_try(i, j, xi, yi, zi, x, N, Lx, Ly, Lz, iLx, iLy, iLz, rc2, nbr, c);
    }
    if (c > kMaxNeigh) {
        atomicOr(status, 1);
        c = kMaxNeigh;
    }
    cnt[i] = c;
    xref[i] = xi;
    xref[N + i] = yi;
    xref[2 * N + i] = zi;
}

// Full lists of every atom of a batch of small systems (at most kSysLdsAtoms atoms each):
// the workgroups (s, g) of system s (blockIdx.x = s, blockIdx.y = g) each copy the
// system's positions to LDS and bin them into its cell grid in LDS (cells[s] = (nx, ny,
// nz, .), nx = 0 or too many cells: all pairs) with atoms ascending in each cell; then
// workgroup g builds the lists of the system's atoms g T .. g T + T - 1 (T threads, one
// atom each) from the 27-cell stencil.  Several workgroups per system keep the rebuild
// short when a batch holds only a few systems.
constexpr int kSysLdsAtoms = 4096;
constexpr int kSysCells = 1024;
constexpr int kNeighSysThreads = 256;

size_t neigh_sys_lds_bytes(int max_sys) {
    return (size_t)max_sys * (3 * sizeof(double) + 2 * sizeof(uint16_t)) + (2 * kSysCells + 1) * sizeof(int) + 16;
}

__global__ void __launch_bounds__(kNeighSysThreads) k_neigh_sys(int N, const int *__restrict__ off, const double *__restrict__ box,
                                                    const double *__restrict__ x, double rc2,
                                                    const int4 *__restrict__ cells, int *__restrict__ nbr,
                                                    int *__restrict__ cnt, int *__restrict__ status,
                                                    const int *__restrict__ flag, double *__restrict__ xref) {
    if (*flag == 0) return;
    extern __shared__ double sm[];
    const int s = blockIdx.x, j0 = off[s], ns = off[s + 1] - j0;
    const int tid = threadIdx.x, T = blockDim.x;
    const int q_me = blockIdx.y * T + tid;  // the atom this thread builds the list of
    if (blockIdx.y * T >= ns) return;
    double *xs = sm;                                                 // [3][ns]
    int *ccnt = reinterpret_cast<int *>(xs + 3 * ns);                // [kSysCells] counts / fill pointers
    int *cstart = ccnt + kSysCells;                                  // [kSysCells + 1]
    uint16_t *catom = reinterpret_cast<uint16_t *>(cstart + kSysCells + 1);  // [ns]
    uint16_t *cid = catom + ns;                                      // [ns]
    const double Lx = box[3 * s], Ly = box[3 * s + 1], Lz = box[3 * s + 2];
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    for (int q = tid; q < ns; q += T) {
        xs[q] = x[j0 + q];
        xs[ns + q] = x[N + j0 + q];
        xs[2 * ns + q] = x[2 * N + j0 + q];
    }
    const int4 ci = cells ? cells[s] : make_int4(0, 0, 0, 0);
    const int NC = ci.x * ci.y * ci.z;
    const bool use_cells = ci.x >= 3 && ci.y >= 3 && ci.z >= 3 && NC <= kSysCells;
    __syncthreads();
    if (use_cells) {
        for (int c = tid; c < NC; c += T) ccnt[c] = 0;
        __syncthreads();
        for (int q = tid; q < ns; q += T) {
            int k3[3];
            const double v[3] = {xs[q] * iLx, xs[ns + q] * iLy, xs[2 * ns + q] * iLz};
            const int n3[3] = {ci.x, ci.y, ci.z};
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const double fr = v[al] - floor(v[al]);
                const int k = (int)(fr * n3[al]);
                k3[al] = k < 0 ? 0 : (k >= n3[al] ? n3[al] - 1 : k);
            }
            const int c = (k3[0] * ci.y + k3[1]) * ci.z + k3[2];
            cid[q] = (uint16_t)c;
            atomicAdd(&ccnt[c], 1);
        }
        __syncthreads();
        if (tid < 64) {
            constexpr int per = kSysCells / 64;
            int loc[per], sum = 0;
#pragma unroll
            for (int k = 0; k < per; ++k) {
                const int c = tid * per + k;
                loc[k] = c < NC ? ccnt[c] : 0;
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
                    cstart[c] = run;
                    ccnt[c] = run;
                }
                run += loc[k];
            }
            if (tid == 63) cstart[NC] = incl;
        }
        __syncthreads();
        for (int q = tid; q < ns; q += T) catom[atomicAdd(&ccnt[cid[q]], 1)] = (uint16_t)q;
        __syncthreads();
        for (int c = tid; c < NC; c += T) {
            const int b = cstart[c], e = cstart[c + 1];
            for (int q = b + 1; q < e; ++q) {
                const uint16_t v = catom[q];
                int r = q - 1;
                while (r >= b && catom[r] > v) {
                    catom[r + 1] = catom[r];
                    --r;
                }
                catom[r + 1] = v;
            }
        }
        __syncthreads();
    }
    if (q_me < ns) {
        const int q = q_me;
        const int i = j0 + q;
        const double xi = xs[q], yi = xs[ns + q], zi = xs[2 * ns + q];
        int c = 0;
        auto try_j = [&](int jl) {
            const double dx = mimg(xs[jl] - xi, Lx, iLx), dy = mimg(xs[ns + jl] - yi, Ly, iLy),
                         dz = mimg(xs[2 * ns + jl] - zi, Lz, iLz);
            if (dx * dx + dy * dy + dz * dz < rc2) {
                if (c < kMaxNeigh) nbr[(size_t)i * kMaxNeigh + c] = j0 + jl;
                ++c;
            }
        };
        if (use_cells) {
            const int me = cid[q];
            const int iz = me % ci.z, iy = (me / ci.z) % ci.y, ix = me / (ci.z * ci.y);
            for (int ax = -1; ax <= 1; ++ax) {
                const int cx = (ix + ax + ci.x) % ci.x;
                for (int ay = -1; ay <= 1; ++ay) {
                    const int cy = (iy + ay + ci.y) % ci.y;
                    for (int az = -1; az <= 1; ++az) {
                        const int cc = (cx * ci.y + cy) * ci.z + (iz + az + ci.z) % ci.z;
                        // four candidates per step: their loads and distances are
                        // independent, the list keeps the cell's ascending order
                        for (int qq = cstart[cc], qe = cstart[cc + 1]; qq < qe; qq += 4) {
                            int jl[4];
                            double r2[4];
#pragma unroll
                            for (int k = 0; k < 4; ++k) jl[k] = qq + k < qe ? (int)catom[qq + k] : q;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const double dx = mimg(xs[jl[k]] - xi, Lx, iLx), dy = mimg(xs[ns + jl[k]] - yi, Ly, iLy),
                                             dz = mimg(xs[2 * ns + jl[k]] - zi, Lz, iLz);
                                r2[k] = dx * dx + dy * dy + dz * dz;
                            }
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (jl[k] != q && r2[k] < rc2) {
                                    if (c < kMaxNeigh) nbr[(size_t)i * kMaxNeigh + c] = j0 + jl[k];
                                    ++c;
                                }
                        }
                    }
                }
            }
        } else {
            for (int jl = 0; jl < ns; ++jl)
                if (jl != q) try_j(jl);
        }
        if (c > kMaxNeigh) {
            atomicOr(status, 1);
            c = kMaxNeigh;
        }
        cnt[i] = c;
        xref[i] = xi;
        xref[N + i] = yi;
        xref[2 * N + i] = zi;
    }
}

void neigh_init_attributes() {
    (void)hipFuncSetAttribute((const void *)k_neigh_sys, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)neigh_sys_lds_bytes(kSysLdsAtoms));
}

// Cell binning (only when a rebuild is requested): cells[s] = (nx, ny, nz, first cell)
// with nx = 0 for systems searched by brute force.
__global__ void k_cell_zero(int C, int *__restrict__ cnt, int *__restrict__ fill, const int *__restrict__ flag) {
    if (*flag == 0) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < C) {
        cnt[c] = 0;
        fill[c] = 0;
    }
}

__global__ void k_cell_assign(int N, int n_sys, const int *__restrict__ off, const double *__restrict__ box,
                              const double *__restrict__ x, const int4 *__restrict__ cells, int *__restrict__ cell_of,
                              int *__restrict__ cnt, const int *__restrict__ flag) {
    if (*flag == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = sys_of(off, n_sys, i);
    const int4 ci = cells[s];
    if (ci.x < 3) {
        cell_of[i] = -1;
        return;
    }
    int idx[3];
    const int n3[3] = {ci.x, ci.y, ci.z};
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const double f = x[al * N + i] / box[3 * s + al];
        const double fr = f - floor(f);
        int k = (int)(fr * n3[al]);
        idx[al] = k < 0 ? 0 : (k >= n3[al] ? n3[al] - 1 : k);
    }
    const int c = ci.w + (idx[0] * ci.y + idx[1]) * ci.z + idx[2];
    cell_of[i] = c;
    atomicAdd(&cnt[c], 1);
}

__global__ void k_cell_fill(int N, const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                            int *__restrict__ fill, int *__restrict__ cell_atoms, const int *__restrict__ flag) {
    if (*flag == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int c = cell_of[i];
    if (c < 0) return;
    cell_atoms[cell_start[c] + atomicAdd(&fill[c], 1)] = i;
}

// ascending atom order inside every cell, so that neighbour lists are deterministic
__global__ void k_cell_sort(int C, const int *__restrict__ cell_start, int *__restrict__ cell_atoms,
                            const int *__restrict__ flag) {
    if (*flag == 0) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int b = cell_start[c], e = cell_start[c + 1];
    for (int q = b + 1; q < e; ++q) {
        const int v = cell_atoms[q];
        int r = q - 1;
        while (r >= b && cell_atoms[r] > v) {
            cell_atoms[r + 1] = cell_atoms[r];
            --r;
        }
        cell_atoms[r + 1] = v;
    }
}

// Request a rebuild (flag = 1) when some atom moved more than half the skin since the
// last build.
__global__ void k_check_disp(int N, const double *__restrict__ x, const double *__restrict__ xref, double lim2,
                             int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double dx = x[i] - xref[i], dy = x[N + i] - xref[N + i], dz = x[2 * N + i] - xref[2 * N + i];
    if (!(dx * dx + dy * dy + dz * dz <= lim2)) atomicOr(flag, 1);   // NaN also rebuilds
}

__global__ void k_set_flag(int *__restrict__ flag, int v) { *flag = v; }

// Exclusive prefix sum of cnt[0..N) into poff[0..N] (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) k_scan(int N, const int *__restrict__ cnt, int *__restrict__ poff,
                                              const int *__restrict__ flag) {
    if (*flag == 0) return;
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int chunk = (N + 1023) / 1024;
    const int b = t * chunk, e = min(N, b + chunk);
    int s = 0;
    // unrolled so that several of the thread's loads are in flight at once
#pragma unroll 8
    for (int i = b; i < e; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = (t >= d) ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;  // exclusive
#pragma unroll 8
    for (int i = b; i < e; ++i) {
        poff[i] = run;
        run += cnt[i];
    }
    if (t == 1023) poff[N] = part[1023];
}

// CSR pair list from the per-atom lists, one thread per (atom i, slot t): pair p =
// poff[i] + t, its slot-major copy for the SNAP density (lane = atom), and the index of
// the opposite pair (j, i), which is poff[j] plus the rank of i in j's list (status bit 4
// when i is missing there).
__global__ void k_compact(int N, const int *__restrict__ nbr, const int *__restrict__ cnt,
                          const int *__restrict__ poff, int *__restrict__ pair_i, int *__restrict__ pair_j,
                          int *__restrict__ nbr_t, int *__restrict__ rev, int *__restrict__ status,
                          const int *__restrict__ flag) {
    if (*flag == 0) return;
    // grid-stride over the N * kMaxNeigh list slots (a bounded grid keeps the launch cheap
    // on the steps where no rebuild is due)
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < (size_t)N * kMaxNeigh;
         q += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / kMaxNeigh), t = (int)(q - (size_t)i * kMaxNeigh);
        if (t >= cnt[i]) continue;
        const int p = poff[i] + t, j = nbr[q];
        pair_i[p] = i;
        pair_j[p] = j;
        if (nbr_t) nbr_t[(size_t)t * N + i] = j;
        // rank of i in j's list: eight entries (two 16-byte loads) per step, the entries
        // past j's count ignored (they hold an earlier build's neighbours)
        const int4 *lj4 = reinterpret_cast<const int4 *>(nbr + (size_t)j * kMaxNeigh);
        const int cj = cnt[j];
        int r = -1;
        for (int u = 0; u < cj && r < 0; u += 8) {
            const int4 a = lj4[u / 4], b = lj4[u / 4 + 1];
            const int v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
            for (int k = 7; k >= 0; --k)
                if (v[k] == i && u + k < cj) r = u + k;
        }
        if (r >= 0) r += poff[j];
        if (r < 0) { atomicOr(status, 4); r = p; }
        rev[p] = r;
    }
}

// ---------------------------------------------------------------------------
// Finnis-Sinclair EAM
// ---------------------------------------------------------------------------
// Finnis-Sinclair passes, kFsLanes consecutive lanes per atom: lane q takes the atom's
// list entries q, q + kFsLanes, ...; the partial sums are combined by a fixed butterfly,
// so the result does not depend on the launch (deterministic).  Several lanes per atom
// keep enough waves in flight to hide the latency of the neighbours' position loads.
constexpr int kFsLanes = 4;

__device__ __forceinline__ double fs_lane_sum(double v) {
#pragma unroll
    for (int o = 1; o < kFsLanes; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_fs_rho(int N, int n_sys, const int *__restrict__ off,
                                                const double *__restrict__ box, const double *__restrict__ x,
                                                const int *__restrict__ poff, const int *__restrict__ pair_j,
                                                double d, double *__restrict__ rho, int *__restrict__ clear_flag) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    // the neighbour pipeline that read the rebuild flag has finished: clear it for the next step
    if (clear_flag && g == 0) *clear_flag = 0;
    const int i0 = g / kFsLanes, q = g % kFsLanes;
    const bool own = i0 < N;
    const int i = own ? i0 : N - 1;
    const int s = sys_of(off, n_sys, i);
    const double Lx = box[3 * s], Ly = box[3 * s + 1], Lz = box[3 * s + 2];
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    double acc = 0.0;
    const int pe = own ? poff[i + 1] : 0;
    for (int p = poff[i] + q; p < pe; p += kFsLanes) {
        const int j = pair_j[p];
        const double dx = mimg(x[j] - xi, Lx, iLx), dy = mimg(x[N + j] - yi, Ly, iLy), dz = mimg(x[2 * N + j] - zi, Lz, iLz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double r = r2 * rsqrt_nr(r2);
        if (r2 < d * d) acc += (r - d) * (r - d);
    }
    acc = fs_lane_sum(acc);
    if (own && q == 0) rho[i] = acc;
}

// pk (nullable): momenta that receive the closing half kick p += (dt/2) f of a BAOAB step
// (the gather's expression).  The next step's opening stays a kernel of its own: it moves
// x, which the other atoms of this pass still read.
__global__ void __launch_bounds__(256) k_fs_force(int N, int n_sys, const int *__restrict__ off,
                                                  const double *__restrict__ box, const double *__restrict__ x,
                                                  const int *__restrict__ poff, const int *__restrict__ pair_j,
                                                  FsParams fp, const double *__restrict__ rho, double *__restrict__ f,
                                                  double *__restrict__ e_atom, int accumulate, double *__restrict__ pk,
                                                  double dt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int i0 = g / kFsLanes, q = g % kFsLanes;
    const bool own = i0 < N;
    const int i = own ? i0 : N - 1;
    const int s = sys_of(off, n_sys, i);
    const double Lx = box[3 * s], Ly = box[3 * s + 1], Lz = box[3 * s + 2];
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    const double ri = rho[i];
    const double dFi = ri > 0.0 ? -fp.A / (2.0 * sqrt(ri)) : 0.0;
    double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
    const int pe = own ? poff[i + 1] : 0;
    for (int p = poff[i] + q; p < pe; p += kFsLanes) {
        const int j = pair_j[p];
        const double dx = mimg(x[j] - xi, Lx, iLx), dy = mimg(x[N + j] - yi, Ly, iLy), dz = mimg(x[2 * N + j] - zi, Lz, iLz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ir = rsqrt_nr(r2), r = r2 * ir;
        double dEdr = 0.0;
        if (r < fp.c) {
            const double t = r - fp.c, poly = fp.c0 + r * (fp.c1 + r * fp.c2);
            ep += 0.5 * t * t * poly;
            dEdr += 2.0 * t * poly + t * t * (fp.c1 + 2.0 * fp.c2 * r);
        }
        if (r < fp.d) {
            const double rj = rho[j];
            const double dFj = rj > 0.0 ? -fp.A / (2.0 * sqrt(rj)) : 0.0;
            dEdr += (dFi + dFj) * 2.0 * (r - fp.d);
        }
        if (r < fp.c || r < fp.d) {
            const double w = dEdr * ir;
            fx += w * dx;
            fy += w * dy;
            fz += w * dz;
        }
    }
    fx = fs_lane_sum(fx);
    fy = fs_lane_sum(fy);
    fz = fs_lane_sum(fz);
    ep = fs_lane_sum(ep);
    if (!own || q != 0) return;
    if (accumulate) {
        fx += f[i];
        fy += f[N + i];
        fz += f[2 * N + i];
    }
    f[i] = fx;
    f[N + i] = fy;
    f[2 * N + i] = fz;
    if (pk) {
        pk[i] = fma(0.5 * dt / MVV2E, fx, pk[i]);
        pk[N + i] = fma(0.5 * dt / MVV2E, fy, pk[N + i]);
        pk[2 * N + i] = fma(0.5 * dt / MVV2E, fz, pk[2 * N + i]);
    }
    if (e_atom) {
        const double e = -fp.A * sqrt(ri) + ep;
        e_atom[i] = accumulate ? e_atom[i] + e : e;
    }
}

// ---------------------------------------------------------------------------
// SNAP: per-pair geometry
//   theta0 = rfac0 pi (r - rmin0)/(rcut - rmin0); a = cos theta0 - i z sin(theta0)/r,
//   b = (y - i x) sin(theta0)/r;  f_c = (cos(pi (r - rmin0)/(rcut - rmin0)) + 1)/2.
// geo layout (SoA, stride Pcap): 0 ar, 1 ai, 2 br, 3 bi, 4 fc,
//   5..7 d(ar)/dx_al, 8..10 d(ai), 11..13 d(br), 14..16 d(bi), 17..19 d(fc)
// ---------------------------------------------------------------------------
// Geometry of a pair at separation d (x_j - x_i): g[0..3] = a, b (re, im), g[4] = f_c,
// g[5..19] their gradients with respect to d (layout above); pairs at or beyond the
// cutoff get a = 1, b = 0, f_c = 0 and zero gradients.
__device__ __forceinline__ void snap_geo(const double (&d)[3], const SnapGeoParams &sp, double (&g)[20]) {
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int q = 0; q < 20; ++q) g[q] = 0.0;
    g[0] = 1.0;
    if (r < sp.rcut) {
        const double w = M_PI / (sp.rcut - sp.rmin0);
        const double c = sp.rfac0 * w;
        double sth, cth, sph, cph;
        sincos(c * (r - sp.rmin0), &sth, &cth);
        sincos(w * (r - sp.rmin0), &sph, &cph);
        const double rinv = 1.0 / r;
        const double sr = sth * rinv;                                // sin(theta0)/r
        const double dsr = (c * cth * r - sth) * rinv * rinv;        // d(sr)/dr
        g[0] = cth;
        g[1] = -d[2] * sr;
        g[2] = d[1] * sr;
        g[3] = -d[0] * sr;
        g[4] = 0.5 * (cph + 1.0);
        const double dfdr = -0.5 * w * sph;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const double u = d[al] * rinv;                           // dr/dx_al
            g[5 + al] = -sth * c * u;
            g[8 + al] = -d[2] * dsr * u - (al == 2 ? sr : 0.0);
            g[11 + al] = d[1] * dsr * u + (al == 1 ? sr : 0.0);
            g[14 + al] = -d[0] * dsr * u - (al == 0 ? sr : 0.0);
            g[17 + al] = dfdr * u;
        }
    }
}
// a, b and f_c only (same expressions as snap_geo)
__device__ __forceinline__ void snap_geo_abf(const double (&d)[3], const SnapGeoParams &sp, double2 &a, double2 &b,
                                             double &fc) {
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    a = make_double2(1.0, 0.0);
    b = make_double2(0.0, 0.0);
    fc = 0.0;
    if (r < sp.rcut) {
        const double w = M_PI / (sp.rcut - sp.rmin0);
        const double c = sp.rfac0 * w;
        double sth, cth, sph, cph;
        sincos(c * (r - sp.rmin0), &sth, &cth);
        sincos(w * (r - sp.rmin0), &sph, &cph);
        const double sr = sth * (1.0 / r);
        a = make_double2(cth, -d[2] * sr);
        b = make_double2(d[1] * sr, -d[0] * sr);
        fc = 0.5 * (cph + 1.0);
    }
}
// minimum-image separation x_j - x_i in system s
__device__ __forceinline__ void pair_sep(const double *__restrict__ x, int N, const double *__restrict__ box, int s,
                                         int i, int j, double (&d)[3]) {
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const double L = box[3 * s + al];
        d[al] = mimg(x[al * N + j] - x[al * N + i], L, 1.0 / L);
    }
}

// pair geometry in CSR order (for the coefficient-gradient passes)
__global__ void k_pair_geo(int N, int n_sys, const int *__restrict__ off, const double *__restrict__ box,
                           const double *__restrict__ x, const int *__restrict__ poff,
                           const int *__restrict__ pair_i, const int *__restrict__ pair_j, SnapGeoParams sp,
                           double *__restrict__ geo, size_t Pcap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= poff[N]) return;
    const int i = pair_i[p], j = pair_j[p];
    double d[3], g[20];
    pair_sep(x, N, box, sys_of(off, n_sys, i), i, j, d);
    snap_geo(d, sp, g);
#pragma unroll
    for (int q = 0; q < 20; ++q) geo[q * Pcap + p] = g[q];
}

// ---------------------------------------------------------------------------
// Column chains of the Wigner-D polynomials P^n[k][l] for a fixed column l.
// advance: level n -> n+1 in place (descending k):  P[k] = b P[k-1] + conj(a) P[k].
// mirror : at odd level n = 2l-1, column l-1 -> column l:
//          P_l[k] = (-1)^(l-k) conj(P_{l-1}[n-k]).
// ---------------------------------------------------------------------------
template <int J, int N>
__device__ __forceinline__ void chain_advance(double2 (&P)[J + 1], double2 b, double2 ab) {
    P[N + 1] = cmul(b, P[N]);
#pragma unroll
    for (int k = N; k >= 1; --k) P[k] = cmul2(b, P[k - 1], ab, P[k]);
    P[0] = cmul(ab, P[0]);
}

template <int J, int N>
__device__ __forceinline__ void chain_advance_d(double2 (&P)[J + 1], double2 (&dP)[3][J + 1], double2 b,
                                                double2 ab, const double2 (&db)[3], const double2 (&dab)[3]) {
#pragma unroll
    for (int al = 0; al < 3; ++al) dP[al][N + 1] = cmul2(db[al], P[N], b, dP[al][N]);
    P[N + 1] = cmul(b, P[N]);
#pragma unroll
    for (int k = N; k >= 1; --k) {
#pragma unroll
        for (int al = 0; al < 3; ++al)
            dP[al][k] = cmul4(db[al], P[k - 1], b, dP[al][k - 1], dab[al], P[k], ab, dP[al][k]);
        P[k] = cmul2(b, P[k - 1], ab, P[k]);
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) dP[al][0] = cmul2(dab[al], P[0], ab, dP[al][0]);
    P[0] = cmul(ab, P[0]);
}

template <int J, int L>  // n = 2L-1 (odd), column L-1 -> L, in place
__device__ __forceinline__ void chain_mirror(double2 (&P)[J + 1]) {
    constexpr int n = 2 * L - 1;
#pragma unroll
    for (int k = 0; 2 * k < n; ++k) {
        const double2 lo = P[k], hi = P[n - k];
        const double sk = ((L - k) & 1) ? -1.0 : 1.0;            // (-1)^(L-k)
        const double sh = ((L - (n - k)) & 1) ? -1.0 : 1.0;      // (-1)^(L-(n-k))
        P[k] = make_double2(sk * hi.x, -sk * hi.y);
        P[n - k] = make_double2(sh * lo.x, -sh * lo.y);
    }
}

// acc index of (n, k) in chain C: elements of levels 2C .. n-1 come first
// (sum_{m=2C}^{n-1} (m+1) in closed form)
__host__ __device__ constexpr int chain_acc_idx(int C, int n, int k) {
    return n * (n + 1) / 2 - C * (2 * C + 1) + k;
}

// Levels N .. N1 of column chain C; the elements of levels N0 .. N1 are accumulated
// (acc index relative to level N0), the lower levels only advance the chain.  TAIL: the
// segment also carries the last column C + 1 = J / 2, whose one level J branches off
// column C at level J - 1 = 2C + 1 (mirror, then one advance), into tacc: the same
// operations the column's own staircase performs, without repeating the chain below.
template <int J, int C, int N0, int N1, int N, bool TAIL>
__device__ __forceinline__ void density_step(
    double2 (&P)[J + 1], double2 (&acc)[chain_acc_idx(C, N1 + 1, 0) - chain_acc_idx(C, N0, 0)],
    double2 (&tacc)[J + 1], double2 b, double2 ab, double fc) {
    if constexpr (N > 2 * C) chain_advance<J, N - 1>(P, b, ab);
    if constexpr (N >= N0) {
        constexpr int a0 = chain_acc_idx(C, N0, 0);
#pragma unroll
        for (int k = 0; k <= N; ++k) {
            acc[chain_acc_idx(C, N, k) - a0].x = fma(fc, P[k].x, acc[chain_acc_idx(C, N, k) - a0].x);
            acc[chain_acc_idx(C, N, k) - a0].y = fma(fc, P[k].y, acc[chain_acc_idx(C, N, k) - a0].y);
        }
    }
    if constexpr (TAIL && N == J - 1) {
        static_assert(2 * C + 1 == J - 1, "the tail column branches off at level 2C + 1");
        double2 Q[J + 1];
#pragma unroll
        for (int k = 0; k <= N; ++k) Q[k] = P[k];
        chain_mirror<J, C + 1>(Q);
        chain_advance<J, J - 1>(Q, b, ab);
#pragma unroll
        for (int k = 0; k <= J; ++k) {
            tacc[k].x = fma(fc, Q[k].x, tacc[k].x);
            tacc[k].y = fma(fc, Q[k].y, tacc[k].y);
        }
    }
    if constexpr (N < N1) density_step<J, C, N0, N1, N + 1, TAIL>(P, acc, tacc, b, ab, fc);
}

template <int J, int C, int c>  // staircase: column c at level 2c -> column c+1 at level 2c+2
__device__ __forceinline__ void staircase(double2 (&P)[J + 1], double2 b, double2 ab) {
    if constexpr (c < C) {
        chain_advance<J, 2 * c>(P, b, ab);
        chain_mirror<J, c + 1>(P);
        chain_advance<J, 2 * c + 1>(P, b, ab);
        staircase<J, C, c + 1>(P, b, ab);
    }
}

// a, b and f_c of every listed pair in slot-major layout ell[f][t][i] (t = rank of the
// pair in i's list), one thread per (slot, atom) with the atom fastest, so that the
// density pass (lane = atom) reads slot t of 64 atoms with one coalesced load per field.
// With fs_d > 0 field 5 holds the Finnis-Sinclair density term phi(r) = (r - d)^2 (r < d).
// clear_flag (non-null): the neighbour pipeline that read the rebuild flag has finished
// on this stream, so the flag is cleared for the next step.
__global__ void k_pair_ell(int N, int n_sys, const int *__restrict__ off, const double *__restrict__ box,
                           const double *__restrict__ x, const int *__restrict__ poff,
                           const int *__restrict__ nbr_t, SnapGeoParams sp, double *__restrict__ ell, double fs_d,
                           int *__restrict__ clear_flag) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (clear_flag && q == 0) *clear_flag = 0;
    const int t = (int)(q / (size_t)N), i = (int)(q - (size_t)t * N);
    if (t >= kMaxNeigh || t >= poff[i + 1] - poff[i]) return;
    double d[3];
    pair_sep(x, N, box, sys_of(off, n_sys, i), i, nbr_t[q], d);
    double2 a, b;
    double fc;
    snap_geo_abf(d, sp, a, b, fc);
    const size_t sN = (size_t)kMaxNeigh * N;
    ell[q] = a.x;
    ell[sN + q] = a.y;
    ell[2 * sN + q] = b.x;
    ell[3 * sN + q] = b.y;
    ell[4 * sN + q] = fc;
    if (fs_d > 0.0) {
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double r = r2 * rsqrt_nr(r2);
        ell[5 * sN + q] = r2 < fs_d * fs_d ? (r - fs_d) * (r - fs_d) : 0.0;
    }
}

// u (half storage, [e][N] double2) for column C, levels N0 .. N1: one wave per tile of 64
// atoms, lane = atom.  Step t reads slot t of the 64 atoms' lists from the slot-major copy
// of a, b and f_c (one coalesced load per field); slots past an atom's count add nothing.
// With gridDim.z = parts > 1 each atom's slots are split into parts (blockIdx.z = part;
// part p takes slots [p cnt / parts, (p + 1) cnt / parts) of an atom with cnt, rounded
// up), each writing its partial sum to u + part nh N (nh = half elements): step k then
// reads slot tb + k of each lane, a few neighbouring rows per load.  The identity term
// of every level goes with part 0, and the Finnis-Sinclair density (dF non-null, column
// 0) is summed over all slots by part 0.
template <int J, int C, int N0, int N1, bool AHEAD, bool TAIL>
__device__ __forceinline__ void density_lane(int tile, int N, const int *__restrict__ poff,
                                             const double *__restrict__ ell, const double *__restrict__ nrm,
                                             double2 *__restrict__ u, double fs_A, double *__restrict__ dF) {
    const int i = tile * 64 + threadIdx.x;
    constexpr int NA = chain_acc_idx(C, N1 + 1, 0) - chain_acc_idx(C, N0, 0);
    double2 acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = make_double2(0.0, 0.0);
    double2 tacc[J + 1];  // the merged last column (TAIL)
#pragma unroll
    for (int q = 0; q <= J; ++q) tacc[q] = make_double2(0.0, 0.0);
    const int cnt = i < N ? poff[i + 1] - poff[i] : 0;
    // this lane's slots [tb, te): its own list cut into parts, so that a partial density
    // depends on the atom alone and not on which atoms share its tile
    const int part = blockIdx.z, parts = gridDim.z;
    const int tb = (part * cnt + parts - 1) / parts, te = ((part + 1) * cnt + parts - 1) / parts;
    int kmax = te - tb;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const size_t sN = (size_t)kMaxNeigh * N;
    constexpr bool kRho = C == 0 && N0 == 0;
    constexpr int NF = kRho ? 6 : 5;
    const bool rho_here = kRho && dF && part == 0;
    const bool rho_apart = rho_here && parts > 1;  // all slots, in a loop of its own
    double rho = 0.0;  // Finnis-Sinclair density (column 0 with dF)
    if (rho_apart)
        for (int t = 0; t < cnt; ++t) rho += ell[5 * sN + (size_t)t * N + i];
    // Fields of the lane's k-th slot tb + k: a, b, f_c (and phi); past te the identity
    // rotation with zero weight (slot contents unused).
    auto fetch = [&](int k, double (&f)[NF]) {
        const int t = tb + k;
        const bool v = t < te;
        const size_t q = v ? (size_t)t * N + i : 0;
        f[0] = v ? ell[q] : 1.0;
        f[1] = v ? ell[sN + q] : 0.0;
        f[2] = v ? ell[2 * sN + q] : 0.0;
        f[3] = v ? ell[3 * sN + q] : 0.0;
        f[4] = v ? ell[4 * sN + q] : 0.0;
        if constexpr (kRho) f[NF - 1] = (rho_here && !rho_apart && v) ? ell[5 * sN + q] : 0.0;
    };
    // AHEAD: slot t + 1 is in flight while slot t is computed (at two waves per SIMD too
    // few other waves hide the load latency).
    double nx[NF];
    if (AHEAD && kmax > 0) fetch(0, nx);
    for (int k = 0; k < kmax; ++k) {
        double f[NF];
        if constexpr (AHEAD) {
#pragma unroll
            for (int m = 0; m < NF; ++m) f[m] = nx[m];
            if (k + 1 < kmax) fetch(k + 1, nx);
        } else {
            fetch(k, f);
        }
        if constexpr (kRho) rho += f[NF - 1];
        const double2 a = make_double2(f[0], f[1]);
        const double2 b = make_double2(f[2], f[3]);
        const double fc = f[4];
        const double2 ab = cconj(a);
        double2 P[J + 1];
        P[0] = make_double2(1.0, 0.0);
        staircase<J, C, 0>(P, b, ab);
        density_step<J, C, N0, N1, 2 * C, TAIL>(P, acc, tacc, b, ab, fc);
    }
    if (i >= N) return;
    if (rho_here) dF[i] = rho > 0.0 ? -fs_A / (2.0 * sqrt(rho)) : 0.0;
    double2 *up = u + (size_t)part * n_half(J) * N;
    const double one = part == 0 ? 1.0 : 0.0;
#pragma unroll
    for (int n = N0; n <= N1; ++n)
#pragma unroll
        for (int k = 0; k <= n; ++k) {
            const int e = half_idx(n, k, C);
            const double sc = nrm[e];
            const double2 v = acc[chain_acc_idx(C, n, k) - chain_acc_idx(C, N0, 0)];
            up[(size_t)e * N + i] = make_double2(fma(sc, v.x, k == C ? one : 0.0), sc * v.y);
        }
    if constexpr (TAIL)
#pragma unroll
        for (int k = 0; k <= J; ++k) {
            const int e = half_idx(J, k, C + 1);
            const double sc = nrm[e];
            up[(size_t)e * N + i] = make_double2(fma(sc, tacc[k].x, k == C + 1 ? one : 0.0), sc * tacc[k].y);
        }
}

// Work split of the density pass: segment s = (column C, levels N0 .. N1) with at most
// kDensAcc accumulated elements each (the register budget of one lane; at twojmax <= 8
// every column chain is one segment).  A segment above a column's first level recomputes
// the chain's lower levels without accumulating them.
// ACC is the kernel-shape choice of the density pass (smaller: more, shorter segments,
// fewer registers per lane, more waves in flight, more recomputed chain levels).
// The last column (one level, J + 1 elements) has no segment of its own when it fits the
// budget of the previous column's last segment (T): its chain is that column's up to
// level J - 1, so a segment of its own would repeat the whole staircase (at twojmax 8,
// 576 of its 612 operations per pair).
struct DensSeg {
    int C, N0, N1;
    bool T;
};
// elements of the last segment of column C
__host__ __device__ constexpr int dens_last_acc(int J, int ACC, int C) {
    int lev = 2 * C, acc = 0;
    while (lev <= J) {
        int top = lev;
        acc = 0;
        while (top <= J && (top == lev || acc + top + 1 <= ACC)) acc += ++top;  // adds level top - 1
        lev = top;
    }
    return acc;
}
// (budget: the merged elements plus the branch's own chain copy, J + 1 more registers pairs)
__host__ __device__ constexpr bool dens_tail_merged(int J, int ACC) {
    return J >= 2 && dens_last_acc(J, ACC, J / 2 - 1) + 2 * (J + 1) <= ACC;
}
__host__ __device__ constexpr int dens_segments(int J, int ACC) {
    int n = 0;
    for (int C = 0; 2 * C <= J; ++C) {
        if (2 * C == J && dens_tail_merged(J, ACC)) break;
        int lev = 2 * C;
        while (lev <= J) {
            int acc = 0, top = lev;
            while (top <= J && (top == lev || acc + top + 1 <= ACC)) acc += ++top;  // adds level top - 1
            ++n;
            lev = top;
        }
    }
    return n;
}
__host__ __device__ constexpr DensSeg dens_segment(int J, int ACC, int s) {
    int n = 0;
    for (int C = 0; 2 * C <= J; ++C) {
        if (2 * C == J && dens_tail_merged(J, ACC)) break;
        int lev = 2 * C;
        while (lev <= J) {
            int acc = 0, top = lev;
            while (top <= J && (top == lev || acc + top + 1 <= ACC)) acc += ++top;
            if (n == s) return DensSeg{C, lev, top - 1, top > J && 2 * C + 2 == J && dens_tail_merged(J, ACC)};
            ++n;
            lev = top;
        }
    }
    return DensSeg{0, 0, 0, false};
}

// Least waves per SIMD that the compiler is held to for a register budget: the budget of
// 28 elements fits three waves (at most 168 registers) only when held to it; the budget
// of 45 takes up to 256 registers (two waves), that of 21 about 130 (three; held to four
// waves it spills).
// Only the budget of 45 loads one slot ahead.
__host__ __device__ constexpr int dens_waves(int ACC) { return ACC == 28 ? 3 : 1; }
__host__ __device__ constexpr bool dens_ahead(int ACC) { return ACC > 28; }

template <int J, int ACC, int S>
__device__ __forceinline__ void density_dispatch(int y, int tile, int N, const int *__restrict__ poff,
                                                 const double *__restrict__ ell, const double *__restrict__ nrm,
                                                 double2 *__restrict__ u, double fs_A, double *__restrict__ dF) {
    if (y == S) {
        constexpr DensSeg g = dens_segment(J, ACC, S);
        density_lane<J, g.C, g.N0, g.N1, dens_ahead(ACC), g.T>(tile, N, poff, ell, nrm, u, fs_A,
                                                              (g.C == 0 && g.N0 == 0) ? dF : nullptr);
    } else if constexpr (S + 1 < dens_segments(J, ACC)) {
        density_dispatch<J, ACC, S + 1>(y, tile, N, poff, ell, nrm, u, fs_A, dF);
    }
}

// dF non-null: column 0 also sums the Finnis-Sinclair density of field 5 and writes
// dF[i] = F'(rho_i) = -A / (2 sqrt(rho_i)) (0 for rho_i = 0).
// Workgroup order: workgroups go to the eight chiplets (each with its own L2) in turn,
// so the segments of tile x are numbered 8 (S q + y) + r with x = 8 q + r: all S of them
// run on one chiplet one after the other, and the tile's slot table comes from HBM once
// instead of once per segment.  Workgroups past the last tile exit at once.
template <int J, int ACC>
__global__ void __launch_bounds__(64, dens_waves(ACC)) k_density(int N, const int *__restrict__ poff, const double *__restrict__ ell,
                                                const double *__restrict__ nrm, double2 *__restrict__ u,
                                                double fs_A, double *__restrict__ dF) {
    constexpr int S = dens_segments(J, ACC);
    const int L = blockIdx.x, r = L & 7, w = L >> 3;
    const int y = w % S, tile = (w / S) * 8 + r;
    if (tile * 64 >= N) return;
    density_dispatch<J, ACC, 0>(y, tile, N, poff, ell, nrm, u, fs_A, dF);
}

// ---------------------------------------------------------------------------
// Adjoint by the coupling program (lane = atom):
//   Y_e = sum_t coef_t op1(u[h1]) op2(u[h2]),  Y~_e = Y_e * Nrm_e * mult_e,
//   E_i = beta0 + (1/3) sum_e mult_e Re(conj(Y_e) u_e)   (Euler, E cubic in u).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adjoint(int N, int nh, const double2 *__restrict__ u,
                                                 const int *__restrict__ ystart, const uint32_t *__restrict__ yidx,
                                                 const double *__restrict__ ycoef, const double *__restrict__ nrm,
                                                 const double *__restrict__ ymult, double beta0,
                                                 double2 *__restrict__ ytil, double *__restrict__ e_atom,
                                                 int accumulate_e) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double esum = 0.0;
    for (int e = 0; e < nh; ++e) {
        const int t0 = ystart[e], t1 = ystart[e + 1];
        double2 acc = make_double2(0.0, 0.0);
        for (int t = t0; t < t1; ++t) {
            const uint32_t w = yidx[t];
            double2 a = u[(size_t)(w & 0xfffu) * N + i];
            double2 b = u[(size_t)((w >> 12) & 0xfffu) * N + i];
            if (w & (1u << 24)) a.y = -a.y;
            if (w & (1u << 25)) b.y = -b.y;
            const double c = ycoef[t];
            acc.x = fma(c, a.x * b.x - a.y * b.y, acc.x);
            acc.y = fma(c, a.x * b.y + a.y * b.x, acc.y);
        }
        const double m = ymult[e];
        const double2 ue = u[(size_t)e * N + i];
        esum += m * (acc.x * ue.x + acc.y * ue.y);
        const double s = m * nrm[e];
        ytil[(size_t)e * N + i] = make_double2(s * acc.x, s * acc.y);
    }
    if (e_atom) {
        const double en = beta0 + esum / 3.0;
        e_atom[i] = accumulate_e ? e_atom[i] + en : en;
    }
}

// The coupling program split over (64-atom tile, chunk of output elements) workgroups, so
// that a batch of a few thousand atoms still gives every CU several waves to hide the
// latency of the u loads (twojmax above 8, where u stays in device memory).  Chunk c
// covers the output elements ychunk[c] .. ychunk[c+1]-1 (balanced by term count on the
// host).  Workgroup w runs on chiplet w mod 8 (the dispatcher's round robin); the
// mapping keeps every chunk of a tile on one chiplet, so the tile's u rows are read
// through one L2.  epart[c][i]: the chunk's part of the Euler sum (null: no energies).
__global__ void __launch_bounds__(64) k_adjoint_chunks(int N, int n_tiles, int n_chunks,
                                                       const int *__restrict__ ychunk, const double2 *__restrict__ u,
                                                       const int *__restrict__ ystart,
                                                       const uint32_t *__restrict__ yidx,
                                                       const double *__restrict__ ycoef, const double *__restrict__ nrm,
                                                       const double *__restrict__ ymult, double2 *__restrict__ ytil,
                                                       double *__restrict__ epart) {
    const int w = blockIdx.x, xcd = w & 7, loc = w >> 3;
    const int tile = (loc / n_chunks) * 8 + xcd, c = loc % n_chunks;
    if (tile >= n_tiles) return;
    const int i = tile * 64 + threadIdx.x;
    const bool own = i < N;
    const int ii = own ? i : N - 1;
    double esum = 0.0;
    for (int e = ychunk[c]; e < ychunk[c + 1]; ++e) {
        const int t0 = ystart[e], t1 = ystart[e + 1];
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
        for (int t = t0; t < t1; ++t) {
            const uint32_t wd = yidx[t];
            double2 a = u[(size_t)(wd & 0xfffu) * N + ii];
            double2 b = u[(size_t)((wd >> 12) & 0xfffu) * N + ii];
            if (wd & (1u << 24)) a.y = -a.y;
            if (wd & (1u << 25)) b.y = -b.y;
            const double cf = ycoef[t];
            acc.x = fma(cf, a.x * b.x - a.y * b.y, acc.x);
            acc.y = fma(cf, a.x * b.y + a.y * b.x, acc.y);
        }
        const double m = ymult[e];
        const double2 ue = u[(size_t)e * N + ii];
        esum += m * (acc.x * ue.x + acc.y * ue.y);
        const double sc = m * nrm[e];
        if (own) ytil[(size_t)e * N + i] = make_double2(sc * acc.x, sc * acc.y);
    }
    if (epart && own) epart[(size_t)c * N + i] = esum;
}

// E_i = beta0 + (1/3) sum_c epart[c][i], summed in chunk order (deterministic)
__global__ void k_energy_chunks(int N, int n_chunks, const double *__restrict__ epart, double beta0,
                                double *__restrict__ e_atom, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += epart[(size_t)c * N + i];
    const double en = beta0 + s / 3.0;
    e_atom[i] = accumulate ? e_atom[i] + en : en;
}

// Bispectrum by the coupling program (lane = atom): B[t][i].
__global__ void __launch_bounds__(256) k_bispectrum(int N, int K, const double2 *__restrict__ u,
                                                    const int *__restrict__ bstart, const uint32_t *__restrict__ bidx,
                                                    const int *__restrict__ bel, const double *__restrict__ bcg,
                                                    double *__restrict__ B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int t = 0; t < K; ++t) {
        double acc = 0.0;
        for (int q = bstart[t]; q < bstart[t + 1]; ++q) {
            const uint32_t w = bidx[q];
            double2 a = u[(size_t)(w & 0xfffu) * N + i];
            double2 b = u[(size_t)((w >> 12) & 0xfffu) * N + i];
            if (w & (1u << 24)) a.y = -a.y;
            if (w & (1u << 25)) b.y = -b.y;
            const double2 ue = u[(size_t)bel[q] * N + i];
            const double2 z = cmul(a, b);
            acc = fma(bcg[q], ue.x * z.x + ue.y * z.y, acc);
        }
        B[(size_t)t * N + i] = acc;
    }
}

// ---------------------------------------------------------------------------
// dE_i/dr_ij per pair: lane = pair.  Column chains l = 0..J/2 of P only; the column at
// level 2l+1 is saved as the (mirrored) seed of chain l+1.
//
// The derivatives of P come from the Lie algebra of SU(2) instead of a recursion of their
// own.  D is a representation, so dD/dr_al = dD(X_al) D with X_al = (dg/dr_al) g^-1 in
// su(2), and dD(X) acts on the rows of a column as a three-term operator: in the
// unnormalised coefficients P (D = Nrm P, Nrm(n, k, l) = sqrt(k! (n-k)! / (l! (n-l)!)))
//   dP[k] = X11 (2k - n) P[k] + X21 (k + 1) P[k+1] + X12 (n - k + 1) P[k-1],
// X11 = a' conj(a) + b' conj(b), X12 = b' a - a' b, X21 = -conj(X12).  X_al does not depend
// on the element, so the contraction needs three sums per pair, whatever the direction:
//   Q0 = sum (2k - n) conj(Y~) P[k],  Qp = sum (k + 1) conj(Y~) P[k+1],
//   Qm = sum (n - k + 1) conj(Y~) P[k-1],
// and S_al = Re(X11_al Q0 + X21_al Qp + X12_al Qm), S0 = sum Re(conj(Y~) P[k]),
// g_al = dfc_al S0 + fc S_al.
// ---------------------------------------------------------------------------
struct DedrAcc {
    double S0 = 0.0;
    double2 Q0 = {0.0, 0.0}, Qp = {0.0, 0.0}, Qm = {0.0, 0.0};
};

// acc += w conj(y) v
__device__ __forceinline__ void cjmac(double2 &acc, double w, double2 y, double2 v) {
    const double yx = w * y.x, yy = w * y.y;
    acc.x = fma(yx, v.x, fma(yy, v.y, acc.x));
    acc.y = fma(yx, v.y, fma(-yy, v.x, acc.y));
}

template <int J, int C, int N>
__device__ __forceinline__ void dedr_level(double2 (&P)[J + 1], double2 (&sP)[J + 1], double2 b, double2 ab,
                                           const double2 *__restrict__ yt, int Natoms, DedrAcc &A) {
    if constexpr (N > 2 * C) chain_advance<J, N - 1>(P, b, ab);
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        if (2 * C == N && 2 * k > N) continue;  // mirrored half of the middle column
        const double2 y = yt[(size_t)half_idx(N, k, C) * Natoms];
        const double tx = fma(y.x, P[k].x, y.y * P[k].y);
        A.S0 += tx;
        if (2 * k != N) {
            const double ty = fma(y.x, P[k].y, -y.y * P[k].x);
            A.Q0.x = fma((double)(2 * k - N), tx, A.Q0.x);
            A.Q0.y = fma((double)(2 * k - N), ty, A.Q0.y);
        }
        if (k + 1 <= N) cjmac(A.Qp, (double)(k + 1), y, P[k + 1]);
        if (k >= 1) cjmac(A.Qm, (double)(N - k + 1), y, P[k - 1]);
    }
    if constexpr (N == 2 * C + 1 && 2 * C + 2 <= J) {
#pragma unroll
        for (int k = 0; k <= N; ++k) sP[k] = P[k];
    }
    if constexpr (N < J) dedr_level<J, C, N + 1>(P, sP, b, ab, yt, Natoms, A);
}

template <int J, int C>
__device__ __forceinline__ void dedr_chain(double2 (&P)[J + 1], double2 (&sP)[J + 1], double2 b, double2 ab,
                                           const double2 *__restrict__ yt, int Natoms, DedrAcc &A) {
    if constexpr (C == 0) {
        P[0] = make_double2(1.0, 0.0);
    } else {
        constexpr int n = 2 * C - 1;
#pragma unroll
        for (int k = 0; k <= n; ++k) P[k] = sP[k];
        chain_mirror<J, C>(P);
        chain_advance<J, n>(P, b, ab);
    }
    dedr_level<J, C, 2 * C>(P, sP, b, ab, yt, Natoms, A);
    if constexpr (2 * C + 2 <= J) dedr_chain<J, C + 1>(P, sP, b, ab, yt, Natoms, A);
}

// One wave of 64 consecutive pairs (CSR order, so a few atoms i).  When the wave's
// pairs belong to at most SA atoms (the kernel-shape choice of this pass; 0: never),
// their Y~ rows are first copied into LDS (coalesced: consecutive lanes take consecutive
// atoms of one element) and the chains read Y~ from there; otherwise from global memory.

// fs (stride 64, or null): a Finnis-Sinclair addend per component
template <int J>
__device__ __forceinline__ void dedr_pair(int p, size_t Pcap, const double (&g)[20],
                                          const double2 *__restrict__ yt, int ystride, double *__restrict__ dedr,
                                          const double *fs) {
    const double fc = g[4];
    const double2 a = make_double2(g[0], g[1]);
    const double2 b = make_double2(g[2], g[3]);
    const double2 ab = cconj(a);
    double2 P[J + 1], sP[J + 1];
    DedrAcc A;
    dedr_chain<J, 0>(P, sP, b, ab, yt, ystride, A);
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const double2 da = make_double2(g[5 + al], g[8 + al]);
        const double2 db = make_double2(g[11 + al], g[14 + al]);
        // X11 = da conj(a) + db conj(b) (imaginary), X12 = db a - da b, X21 = -conj(X12)
        const double x11 = fma(da.y, a.x, fma(-da.x, a.y, fma(db.y, b.x, -db.x * b.y)));
        const double2 x12 = csub(cmul(db, a), cmul(da, b));
        // Re(i x11 Q0 + X21 Qp + X12 Qm), X21 = (-x12.x, x12.y)
        const double s = fma(-x11, A.Q0.y, fma(-x12.x, A.Qp.x, fma(-x12.y, A.Qp.y,
                                                                    fma(x12.x, A.Qm.x, -x12.y * A.Qm.y))));
        const double v = fma(g[17 + al], A.S0, fc * s);
        dedr[al * Pcap + p] = fs ? v + fs[64 * al] : v;
    }
}

// With fz.on the Finnis-Sinclair part of the same derivative is added: for
// E_i = F(rho_i) + (1/2) sum_j V(r_ij), dE_i/d(x_j - x_i) = (F'(rho_i) phi'(r) + V'(r)/2) d/r,
// with F'(rho_i) from the density pass.  (The gather's g_p - g_rev(p) then assembles the
// pair force (F'(rho_i) + F'(rho_j)) phi' + V'.)  It is staged in LDS so that no register
// stays live across the SNAP contraction.
template <int J, int SA>
__global__ void __launch_bounds__(64) k_dedr(int N, int n_sys, const int *__restrict__ off,
                                             const double *__restrict__ box, const double *__restrict__ x,
                                             const int *__restrict__ poff, const int *__restrict__ pair_i,
                                             const int *__restrict__ pair_j, SnapGeoParams sp, size_t Pcap,
                                             const double2 *__restrict__ ytil, double *__restrict__ dedr,
                                             FsFuse fz) {
    constexpr int NH = n_half(J);
    constexpr bool kStage = SA > 0;
    __shared__ double2 ys[kStage ? SA * NH : 1];
    __shared__ double fsb[3 * 64];
    const int P = poff[N];
    const int p0 = blockIdx.x * 64;
    if (p0 >= P) return;
    const int lane = threadIdx.x, p = p0 + lane;
    const int i0 = pair_i[p0], na = pair_i[min(p0 + 63, P - 1)] - i0 + 1;
    const bool live = p < P;
    const int i = live ? pair_i[p] : i0;
    // geometry of the pair from the positions
    double g[20];
    {
        double d[3] = {1.0, 0.0, 0.0};
        if (live) pair_sep(x, N, box, sys_of(off, n_sys, i), i, pair_j[p], d);
        if (fz.on) {
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double ir = rsqrt_nr(r2), r = r2 * ir;
            const FsParams &fp = fz.fp;
            double dEdr = 0.0;
            if (r < fp.c) {
                const double t = r - fp.c, poly = fp.c0 + r * (fp.c1 + r * fp.c2);
                dEdr += 0.5 * (2.0 * t * poly + t * t * (fp.c1 + 2.0 * fp.c2 * r));
            }
            if (r < fp.d) dEdr += fz.dF[i] * 2.0 * (r - fp.d);
            const double wf = live ? dEdr * ir : 0.0;
#pragma unroll
            for (int al = 0; al < 3; ++al) fsb[64 * al + lane] = wf * d[al];
        }
        snap_geo(d, sp, g);
    }
    const double fc = live ? g[4] : 0.0;
    const double *fs = fz.on ? fsb + lane : nullptr;
    if (kStage && na <= SA) {
        for (int q = lane; q < na * NH; q += 64) {
            const int e = q / na, at = q - e * na;
            ys[q] = ytil[(size_t)e * N + i0 + at];
        }
        __syncthreads();
        if (fc != 0.0) dedr_pair<J>(p, Pcap, g, ys + (i - i0), na, dedr, fs);
    } else {
        if (fc != 0.0) dedr_pair<J>(p, Pcap, g, ytil + i, N, dedr, fs);
    }
    if (live && fc == 0.0) {
        dedr[p] = fs ? fs[0] : 0.0;
        dedr[Pcap + p] = fs ? fs[64] : 0.0;
        dedr[2 * Pcap + p] = fs ? fs[128] : 0.0;
    }
}

// F_k (+)= sum_{p in pairs(k)} (g_p - g_rev(p)), optionally followed by the closing half
// kick p_k += (dt/2) F_k of a BAOAB step (pk non-null).  A workgroup takes 64 atoms;
// their pairs are one contiguous range of the list, read in windows of kGatherWin pairs
// by all 256 threads (coalesced, one reverse index each), differences staged in LDS.
// Wave c then sums component c of each atom's differences in list order, so the sum
// is the same sequence of additions as a loop over the atom's pairs.
constexpr int kGatherWin = 2048;
__device__ __forceinline__ void baoab_open(int N, int i, int s, int local, const double (&pv)[3],
                                           const double (&fv)[3], double *__restrict__ x, double *__restrict__ p,
                                           const LangevinDev &ld, int s_step, const double *__restrict__ xref,
                                           double lim2, int *__restrict__ flag);

// With open.open_step >= 0 (and pk) the workgroup then also opens step open_step for its
// 64 atoms, one lane per atom (the three components meet in LDS): the B A O A and the
// displacement test of k_baoab_pre, through the same function, on the kicked momenta.
__global__ void __launch_bounds__(256) k_gather(int N, const int *__restrict__ poff, const int *__restrict__ rev,
                                                const double *__restrict__ dedr, size_t Pcap,
                                                double *__restrict__ f, int accumulate, double *__restrict__ pk,
                                                double dt, StepOpen open) {
    __shared__ double dg[3][kGatherWin];
    const int k0 = blockIdx.x * 64, k1 = min(k0 + 64, N);
    const int tid = threadIdx.x, c = tid >> 6, k = k0 + (tid & 63);
    const bool own = c < 3 && k < k1;
    const int P0 = poff[k0], P1 = poff[k1];
    const int pb = own ? poff[k] : 0, pe = own ? poff[k + 1] : 0;
    double g = 0.0;
    for (int w0 = P0; w0 < P1; w0 += kGatherWin) {
        const int n = min(kGatherWin, P1 - w0);
        for (int q = tid; q < n; q += 256) {
            const int p = w0 + q, r = rev[p];
            dg[0][q] = dedr[p] - dedr[r];
            dg[1][q] = dedr[Pcap + p] - dedr[Pcap + r];
            dg[2][q] = dedr[2 * Pcap + p] - dedr[2 * Pcap + r];
        }
        __syncthreads();
        if (own) {
            const int a = max(pb, w0), b = min(pe, w0 + n);
            for (int p = a; p < b; ++p) g += dg[c][p - w0];
        }
        __syncthreads();
    }
    const bool opening = pk && open.open_step >= 0;
    double fk = 0.0, pn = 0.0;
    if (own) {
        const size_t o = (size_t)c * N + k;
        fk = accumulate ? f[o] + g : g;
        f[o] = fk;
        if (pk) {
            pn = fma(0.5 * dt / MVV2E, fk, pk[o]);
            if (!opening) pk[o] = pn;
        }
    }
    if (!opening) return;
    // dg is free: the last window ended with a barrier
    double *sf = &dg[0][0], *sp = &dg[1][0];
    if (own) {
        sf[c * 64 + (tid & 63)] = fk;
        sp[c * 64 + (tid & 63)] = pn;
    }
    __syncthreads();
    if (tid < 64 && k0 + tid < N) {
        const int i = k0 + tid, s = sys_of(open.off, open.n_sys, i);
        const double pv[3] = {sp[tid], sp[64 + tid], sp[128 + tid]};
        const double fv[3] = {sf[tid], sf[64 + tid], sf[128 + tid]};
        baoab_open(N, i, s, i - open.off[s], pv, fv, open.x, pk, open.ld, open.open_step, open.xref, open.lim2,
                   open.flag);
    }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
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
}

// tag: fourth counter word (0: BAOAB; 1 and 2: the BBK scheme's G_l, l < L, and G_L)
__device__ __forceinline__ void gauss3(uint64_t seed, uint64_t noise_id, uint64_t step, uint64_t atom,
                                       double &g0, double &g1, double &g2, uint64_t tag = 0) {
    uint64_t c[4] = {noise_id, step, atom, tag};
    philox4x64_10(c, seed, 0);
    const double two53 = 1.0 / 9007199254740992.0;
    const double u1 = 1.0 - (double)(c[0] >> 11) * two53;
    const double u2 = (double)(c[1] >> 11) * two53;
    const double u3 = 1.0 - (double)(c[2] >> 11) * two53;
    const double u4 = (double)(c[3] >> 11) * two53;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    double s2, c2, s4, c4;
    sincos(2.0 * M_PI * u2, &s2, &c2);
    sincos(2.0 * M_PI * u4, &s4, &c4);
    g0 = r1 * c2;
    g1 = r1 * s2;
    g2 = r2 * c4;
}

// B (half kick), A (half drift), O (exact OU), A (half drift)
// B A O A of one step; also requests a Verlet-list rebuild (flag) when the new position
// is more than sqrt(lim2) from the one of the last build.
// B A O A of step s_step for atom i (system s, index `local` in it) from its momentum pv
// and force fv: writes p and x, and flags a list rebuild past the displacement limit.
// Explicit FMAs, so that the standalone pass and the one fused into the gather round alike.
__device__ __forceinline__ void baoab_open(int N, int i, int s, int local, const double (&pv)[3],
                                           const double (&fv)[3], double *__restrict__ x, double *__restrict__ p,
                                           const LangevinDev &ld, int s_step, const double *__restrict__ xref,
                                           double lim2, int *__restrict__ flag) {
    const uint64_t gstep = (uint64_t)(ld.step0[s] + s_step);
    double g[3];
    gauss3(ld.seed, (uint64_t)ld.noise_id[s], gstep, (uint64_t)local, g[0], g[1], g[2]);
    const double hk = 0.5 * ld.dt / MVV2E, hd = 0.5 * ld.dt / ld.mass, sig = ld.sig[s];
    double d2 = 0.0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        double pp = fma(hk, fv[al], pv[al]);
        double xx = fma(hd, pp, x[al * N + i]);
        pp = fma(ld.c1, pp, sig * g[al]);
        xx = fma(hd, pp, xx);
        p[al * N + i] = pp;
        x[al * N + i] = xx;
        const double dd = xx - xref[al * N + i];
        d2 = fma(dd, dd, d2);
    }
    if (!(d2 <= lim2)) atomicOr(flag, 1);  // NaN also rebuilds
}

__global__ void k_baoab_pre(int N, int n_sys, const int *__restrict__ off, double *__restrict__ x,
                            double *__restrict__ p, const double *__restrict__ f, LangevinDev ld, int s_step,
                            const double *__restrict__ xref, double lim2, int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = sys_of(off, n_sys, i);
    const double pv[3] = {p[i], p[N + i], p[2 * N + i]};
    const double fv[3] = {f[i], f[N + i], f[2 * N + i]};
    baoab_open(N, i, s, i - off[s], pv, fv, x, p, ld, s_step, xref, lim2, flag);
}

// The paper's modified BBK scheme, one call = one application of L iterates.  First half
// of iterate l (s_step): p_{l+1/2} = p_l + (dt/2) F_l - (dt/2) gamma p_{l-1/2} + s_l G_l
// (p_{-1/2} := p_0 at l = 0), q_{l+1} = q_l + dt p_{l+1/2} / m.  p then holds p_{l+1/2},
// and ph keeps a copy for the friction term of iterate l + 1.  G_l: counter
// (noise_id, step0 + l, atom, 1).  Also the Verlet-list displacement test of k_baoab_pre.
__global__ void k_bbk_pre(int N, int n_sys, const int *__restrict__ off, double *__restrict__ x,
                          double *__restrict__ p, double *__restrict__ ph, const double *__restrict__ f,
                          LangevinDev ld, int s_step, const double *__restrict__ xref, double lim2,
                          int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = sys_of(off, n_sys, i);
    double g[3];
    gauss3(ld.seed, (uint64_t)ld.noise_id[s], (uint64_t)(ld.step0[s] + s_step), (uint64_t)(i - off[s]), g[0], g[1],
           g[2], 1);
    const double hk = 0.5 * ld.dt / MVV2E, hg = 0.5 * ld.dt * ld.gamma, dm = ld.dt / ld.mass;
    const double sig = s_step == 0 ? ld.sb0[s] : ld.sb1[s];
    double d2 = 0.0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const size_t q = (size_t)al * N + i;
        const double pl = p[q];
        const double prev = s_step == 0 ? pl : ph[q];
        const double half = pl + hk * f[q] - hg * prev + sig * g[al];
        const double xx = x[q] + dm * half;
        p[q] = half;
        ph[q] = half;
        x[q] = xx;
        const double dd = xx - xref[q];
        d2 += dd * dd;
    }
    if (!(d2 <= lim2)) atomicOr(flag, 1);  // NaN also rebuilds
}

// Second half of iterate l: p_{l+1} = p_{l+1/2} + (dt/2) F_{l+1} - (dt/2) gamma p_{l+1/2}
// + s_{l+1} G_{l+1} (s1 = l + 1 >= 1); G_L of the call (s1 == L) uses tag 2.
__global__ void k_bbk_post(int N, int n_sys, const int *__restrict__ off, double *__restrict__ p,
                           const double *__restrict__ f, LangevinDev ld, int s1, int last) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = sys_of(off, n_sys, i);
    double g[3];
    gauss3(ld.seed, (uint64_t)ld.noise_id[s], (uint64_t)(ld.step0[s] + s1), (uint64_t)(i - off[s]), g[0], g[1], g[2],
           last ? 2 : 1);
    const double hk = 0.5 * ld.dt / MVV2E, hg = 0.5 * ld.dt * ld.gamma, sig = ld.sb1[s];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const size_t q = (size_t)al * N + i;
        const double half = p[q];
        p[q] = half + hk * f[q] - hg * half + sig * g[al];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// Verlet list: built with rc + skin when forced or when an atom has moved more than
// skin/2 since the last build (decided on the device); the pair kernels apply the exact
// cutoffs, so the list only decides which pairs are examined.
void launch_neighbors(const BatchDev &bd, const double *x, double rc, Work &w, hipStream_t st, bool force,
                      double skin, bool checked, bool clear_in_fs) {
    const int N = bd.N;
    if (force) {
        hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, st, w.flag, 1);
    } else if (!checked) {
        hipLaunchKernelGGL(k_check_disp, dim3(nblk(N, 256)), dim3(256), 0, st, N, x, w.xref, 0.25 * skin * skin,
                           w.flag);
    }
    const double rl = rc + skin;
    if (bd.max_sys > 0 && bd.max_sys <= kSysLdsAtoms) {
        // small systems: the whole build in one kernel, one workgroup per system
        hipLaunchKernelGGL(k_neigh_sys, dim3(bd.n_sys, nblk(bd.max_sys, kNeighSysThreads)), dim3(kNeighSysThreads),
                           neigh_sys_lds_bytes(bd.max_sys), st, N, bd.off,
                           bd.box, x, rl * rl, (bd.cells && bd.n_cells > 0) ? bd.cells : nullptr, w.nbr, w.cnt,
                           w.status, w.flag, w.xref);
    } else if (bd.cells && bd.n_cells > 0) {
        const int C = bd.n_cells;
        hipLaunchKernelGGL(k_cell_zero, dim3(nblk(C, 256)), dim3(256), 0, st, C, w.cell_cnt, w.cell_fill, w.flag);
        hipLaunchKernelGGL(k_cell_assign, dim3(nblk(N, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box, x,
                           bd.cells, w.cell_of, w.cell_cnt, w.flag);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, C, w.cell_cnt, w.cell_start, w.flag);
        hipLaunchKernelGGL(k_cell_fill, dim3(nblk(N, 256)), dim3(256), 0, st, N, w.cell_of, w.cell_start, w.cell_fill,
                           w.cell_atoms, w.flag);
        hipLaunchKernelGGL(k_cell_sort, dim3(nblk(C, 256)), dim3(256), 0, st, C, w.cell_start, w.cell_atoms, w.flag);
    }
    if (!(bd.max_sys > 0 && bd.max_sys <= kSysLdsAtoms))
        hipLaunchKernelGGL(k_neigh_build, dim3(nblk(N, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box, x,
                           rl * rl, w.nbr, w.cnt, w.status, w.flag, w.xref,
                           (bd.cells && bd.n_cells > 0) ? bd.cells : nullptr, w.cell_of, w.cell_start, w.cell_atoms);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, N, w.cnt, w.poff, w.flag);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)std::min<size_t>(nblk((size_t)N * kMaxNeigh, 256), 1024)), dim3(256), 0,
                       st, N, w.nbr, w.cnt, w.poff,
                       w.pair_i, w.pair_j, w.nbr_t, w.rev, w.status, w.flag);
    if (!clear_in_fs) hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, st, w.flag, 0);
}

void launch_fs(const BatchDev &bd, const double *x, const FsParams &fp, Work &w, double *f, double *e_atom,
               int accumulate, hipStream_t st, bool clear_flag, double *p_kick, double dt) {
    const int N = bd.N;
    hipLaunchKernelGGL(k_fs_rho, dim3(nblk((size_t)N * kFsLanes, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box, x, w.poff,
                       w.pair_j, fp.d, w.rho, clear_flag ? w.flag : nullptr);
    hipLaunchKernelGGL(k_fs_force, dim3(nblk((size_t)N * kFsLanes, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box, x, w.poff,
                       w.pair_j, fp, w.rho, f, e_atom, accumulate, p_kick, dt);
}

template <int J, int ACC>
static void density_launch_acc(int N, Work &w, const SnapDev &sd, double fs_A, double *dF, hipStream_t st,
                               int parts) {
    hipLaunchKernelGGL((k_density<J, ACC>), dim3(8 * nblk(N, 512) * dens_segments(J, ACC), 1, parts), dim3(64), 0, st, N,
                       w.poff, w.ell,
                       sd.nrm, w.u, fs_A, dF);
}

// parts: the slot split of the pass (1: u whole; 2: partial sums at u and u + nh N)
template <int J>
static void density_launch(int N, Work &w, const SnapDev &sd, double fs_A, double *dF, hipStream_t st,
                           int parts = 1) {
    if constexpr (J <= 8) {
        switch (sd.shape.dens_acc) {
            case 28: density_launch_acc<J, 28>(N, w, sd, fs_A, dF, st, parts); return;
            case 21: density_launch_acc<J, 21>(N, w, sd, fs_A, dF, st, parts); return;
            default: break;
        }
    }
    density_launch_acc<J, 45>(N, w, sd, fs_A, dF, st, parts);
}

template <int J, int SA>
static void dedr_launch(const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, const FsFuse &fz,
                        hipStream_t st) {
    const int N = bd.N;
    hipLaunchKernelGGL((k_dedr<J, SA>), dim3(nblk((size_t)N * kMaxNeigh, 64)), dim3(64), 0, st, N, bd.n_sys, bd.off,
                       bd.box, x, w.poff, w.pair_i, w.pair_j, sd.gp, w.Pcap, w.ytil, w.dedr, fz);
}

template <int J>
static void launch_snap_J(const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, double *f,
                          double *e_atom, int accumulate, hipStream_t st, KernelProf *prof, hipEvent_t join,
                          double *p_kick, double dt, const FsParams *fuse, const StepOpen *open) {
    const int N = bd.N;
    KernelProf dummy;
    KernelProf &pf = prof ? *prof : dummy;
    FsFuse fz{};
    if (fuse) {
        fz.fp = *fuse;
        fz.dF = w.rho;
        fz.on = 1;
    }
    hipLaunchKernelGGL(k_pair_ell, dim3(nblk((size_t)N * kMaxNeigh, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box,
                       x, w.poff, w.nbr_t, sd.gp, w.ell, fuse ? fuse->d : 0.0, fuse ? w.flag : nullptr);
    // the LDS-tiled adjoint adds the two parts of a split density as it loads its tile
    int parts = 1;
    if constexpr (J <= 8) {
        const int acc = sd.shape.dens_acc;
        const int segs = acc == 28 ? dens_segments(J, 28) : acc == 21 ? dens_segments(J, 21) : dens_segments(J, 45);
        if (sd.shape.dens_parts == 2 || (sd.shape.dens_parts == 0 && (long)nblk(N, 64) * segs < sd.simds)) parts = 2;
    }
    pf.begin(PROF_DENSITY, st);
    density_launch<J>(N, w, sd, fuse ? fuse->A : 0.0, fuse ? w.rho : nullptr, st, parts);
    pf.end(st);
    pf.begin(PROF_ADJOINT, st);
    if constexpr (J <= 8) {
        launch_adjoint(J, sd.adj, N, w.u, parts == 2 ? w.u + (size_t)n_half(J) * N : nullptr, sd.nrm, sd.ymult,
                       sd.beta0, w.ytil, e_atom, accumulate, st, sd.shape.adj_waves);
    } else {
        // above twojmax 8 a 64-atom tile of u no longer fits the LDS: the coupling program
        // reads u from memory (lane = atom, coefficients wave-uniform), split over
        // chunks of output elements
        const int tiles = (int)nblk(N, 64), t8 = (tiles + 7) / 8;
        hipLaunchKernelGGL(k_adjoint_chunks, dim3(t8 * 8 * sd.n_ychunk), dim3(64), 0, st, N, tiles, sd.n_ychunk,
                           sd.ychunk, w.u, sd.ystart, sd.yidx, sd.ycoef, sd.nrm, sd.ymult, w.ytil,
                           e_atom ? w.epart : nullptr);
        if (e_atom)
            hipLaunchKernelGGL(k_energy_chunks, dim3(nblk(N, 256)), dim3(256), 0, st, N, sd.n_ychunk, w.epart,
                               sd.beta0, e_atom, accumulate);
    }
    pf.end(st);
    pf.begin(PROF_DEDR, st);
    if constexpr (J <= 8) {
        switch (sd.shape.dedr_atoms) {
            case 0: dedr_launch<J, 0>(bd, x, sd, w, fz, st); break;
            case 3: dedr_launch<J, 3>(bd, x, sd, w, fz, st); break;
            default: dedr_launch<J, 5>(bd, x, sd, w, fz, st); break;
        }
    } else {
        dedr_launch<J, 0>(bd, x, sd, w, fz, st);
    }
    pf.end(st);
    if (join) (void)hipStreamWaitEvent(st, join, 0);  // f written by work on another stream
    hipLaunchKernelGGL(k_gather, dim3(nblk(N, 64)), dim3(256), 0, st, N, w.poff, w.rev, w.dedr, w.Pcap, f,
                       accumulate, p_kick, dt, open ? *open : StepOpen{});
}

void launch_snap(int J, const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, double *f,
                 double *e_atom, int accumulate, hipStream_t st, KernelProf *prof, hipEvent_t join, double *p_kick,
                 double dt, const FsParams *fuse, const StepOpen *open) {
    switch (J) {
        case 2: launch_snap_J<2>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 4: launch_snap_J<4>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 6: launch_snap_J<6>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 8: launch_snap_J<8>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 10: launch_snap_J<10>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 12: launch_snap_J<12>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        case 14: launch_snap_J<14>(bd, x, sd, w, f, e_atom, accumulate, st, prof, join, p_kick, dt, fuse, open); break;
        default: break;
    }
}


void launch_snap_density(int J, const BatchDev &bd, const double *x, const SnapDev &sd, Work &w, hipStream_t st) {
    const int N = bd.N;
    hipLaunchKernelGGL(k_pair_geo, dim3(nblk((size_t)N * kMaxNeigh, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box, x,
                       w.poff, w.pair_i, w.pair_j, sd.gp, w.geo, w.Pcap);
    hipLaunchKernelGGL(k_pair_ell, dim3(nblk((size_t)N * kMaxNeigh, 256)), dim3(256), 0, st, N, bd.n_sys, bd.off, bd.box,
                       x, w.poff, w.nbr_t, sd.gp, w.ell, 0.0, nullptr);
    switch (J) {
        case 2: density_launch<2>(N, w, sd, 0.0, nullptr, st); break;
        case 4: density_launch<4>(N, w, sd, 0.0, nullptr, st); break;
        case 6: density_launch<6>(N, w, sd, 0.0, nullptr, st); break;
        case 8: density_launch<8>(N, w, sd, 0.0, nullptr, st); break;
        case 10: density_launch<10>(N, w, sd, 0.0, nullptr, st); break;
        case 12: density_launch<12>(N, w, sd, 0.0, nullptr, st); break;
        case 14: density_launch<14>(N, w, sd, 0.0, nullptr, st); break;
        default: break;
    }
}

void launch_bispectrum(const BatchDev &bd, const SnapDev &sd, Work &w, double *B, hipStream_t st) {
    const int N = bd.N;
    hipLaunchKernelGGL(k_bispectrum, dim3(nblk(N, 256)), dim3(256), 0, st, N, sd.K, w.u, sd.bstart, sd.bidx, sd.bel,
                       sd.bcg, B);
}

void launch_baoab_pre(const BatchDev &bd, double *x, double *p, const double *f, const LangevinDev &ld, int s_step,
                      const Work &w, double skin, hipStream_t st) {
    hipLaunchKernelGGL(k_baoab_pre, dim3(nblk(bd.N, 256)), dim3(256), 0, st, bd.N, bd.n_sys, bd.off, x, p, f, ld,
                       s_step, w.xref, 0.25 * skin * skin, w.flag);
}

void launch_bbk_pre(const BatchDev &bd, double *x, double *p, const double *f, const LangevinDev &ld, int s_step,
                    const Work &w, double skin, hipStream_t st) {
    hipLaunchKernelGGL(k_bbk_pre, dim3(nblk(bd.N, 256)), dim3(256), 0, st, bd.N, bd.n_sys, bd.off, x, p, w.ph, f, ld,
                       s_step, w.xref, 0.25 * skin * skin, w.flag);
}

// adds delta to n int64 values (the step offsets of a segmented propagation)
__global__ void k_add_i64(int n, int64_t *__restrict__ v, int64_t delta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] += delta;
}

void launch_add_i64(int n, int64_t *v, int64_t delta, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_add_i64, dim3(nblk(n, 256)), dim3(256), 0, st, n, v, delta);
}

void launch_bbk_post(const BatchDev &bd, double *p, const double *f, const LangevinDev &ld, int s1, int n_steps,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_bbk_post, dim3(nblk(bd.N, 256)), dim3(256), 0, st, bd.N, bd.n_sys, bd.off, p, f, ld, s1,
                       s1 == n_steps ? 1 : 0);
}

}  // namespace snapmd
