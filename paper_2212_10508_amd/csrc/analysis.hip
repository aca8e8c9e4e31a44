// Analysis and preparation kernels around the propagation (gfx950, FP64):
//
// * Wigner-Seitz sites.  The interstitial is located by the Wigner-Seitz cells of the
//   perfect bcc lattice (cubic cells of edge a, sites at the corners and the centres):
//   each atom is assigned to its nearest site, and the site holding two atoms is the
//   interstitial dumbbell.  This stands in for the Voronoi analysis the paper runs in
//   OVITO (section "Numerical results") to follow the defect between metastable states.
// * Steepest descent of the potential energy, the minimisation that starts the paper's
//   equilibration procedure: x <- x + F * min(alpha, dmax / |F|) per atom.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace snapmd {

__global__ void k_fill_int(size_t n, int *__restrict__ p, int v) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

// ws[s] = (nx, ny, nz, first site of system s); sites of system s: first + 2 (ix ny nz +
// iy nz + iz) + b, b = 0 for the cube corner (ix a, iy a, iz a), 1 for the centre.
// Positions may be unwrapped: cell indices are taken modulo the cell counts.  Of two
// sites at exactly equal distance the corner site wins.
__global__ void k_ws_sites(int N, int n_sys, const int *__restrict__ off, const int4 *__restrict__ ws, double a,
                           const double *__restrict__ x, int *__restrict__ site, int *__restrict__ occ) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int4 w = ws[lo];
    const int nc[3] = {w.x, w.y, w.z};
    const double ia = 1.0 / a;
    int c0[3], c1[3];
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const double f = x[(size_t)al * N + i] * ia;
        const double r0 = rint(f), r1 = rint(f - 0.5);
        d0 += (f - r0) * (f - r0);
        d1 += (f - r1 - 0.5) * (f - r1 - 0.5);
        const long long n = nc[al];
        c0[al] = (int)((((long long)r0 % n) + n) % n);
        c1[al] = (int)((((long long)r1 % n) + n) % n);
    }
    const bool centre = d1 < d0;
    const int *c = centre ? c1 : c0;
    const int s = w.w + 2 * ((c[0] * nc[1] + c[1]) * nc[2] + c[2]) + (centre ? 1 : 0);
    site[i] = s;
    atomicAdd(&occ[s], 1);
}

// x += F * min(alpha, dmax / |F|) for every atom (a step of at most dmax)
__global__ void k_descent_step(int N, double *__restrict__ x, const double *__restrict__ f, double alpha,
                               double dmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double fx = f[i], fy = f[N + i], fz = f[2 * (size_t)N + i];
    const double fn = sqrt(fx * fx + fy * fy + fz * fz);
    const double s = (fn * alpha > dmax) ? dmax / fn : alpha;
    x[i] += s * fx;
    x[N + i] += s * fy;
    x[2 * (size_t)N + i] += s * fz;
}

// out = max_i |F_i|^2 (as the bits of a non-negative double, which order like the values)
__global__ void k_fmax2(int N, const double *__restrict__ f, unsigned long long *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < N) {
        const double fx = f[i], fy = f[N + i], fz = f[2 * (size_t)N + i];
        v = fx * fx + fy * fy + fz * fz;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

void launch_ws_sites(const BatchDev &bd, const int4 *ws, int n_sites, double a, const double *x, int *site,
                     int *occ, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3((n_sites + 255) / 256), dim3(256), 0, st, (size_t)n_sites, occ, 0);
    if (bd.N > 0)
        hipLaunchKernelGGL(k_ws_sites, dim3((bd.N + 255) / 256), dim3(256), 0, st, bd.N, bd.n_sys, bd.off, ws, a, x,
                           site, occ);
}

void launch_descent_step(int N, double *x, const double *f, double alpha, double dmax, hipStream_t st) {
    hipLaunchKernelGGL(k_descent_step, dim3((N + 255) / 256), dim3(256), 0, st, N, x, f, alpha, dmax);
}

void launch_fmax2(int N, const double *f, unsigned long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, (size_t)2, reinterpret_cast<int *>(out), 0);
    hipLaunchKernelGGL(k_fmax2, dim3((N + 255) / 256), dim3(256), 0, st, N, f, out);
}

}  // namespace snapmd
