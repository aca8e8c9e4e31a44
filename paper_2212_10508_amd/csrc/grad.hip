// SNAP coefficient gradients (gfx950, FP64).
//
// E = sum_i (beta_0 + sum_k beta_k B_k(i)) is linear in beta, so
//   dE/dbeta_k = sum_i B_k(i),
// and the forces F_i = -dE/dx_i give, for a weight field w (e.g. dLoss/dF),
//   sum_i w_i . dF_i/dbeta_k = -(d/de) sum_j B_k(j)(x + e w) at e = 0.
// The directional derivative is a forward (tangent) pass:
//   k_jvp_density<J,C> : du_j = sum over neighbours i of d(f_c U)(r_ji) along (w_i - w_j),
//                        one column chain of the Wigner-D polynomials and of their
//                        directional derivative per lane (same staircase as the density);
//   k_bispectrum_jvp   : dB_t = Re sum conj(du^j) Z + conj(u^j) (Z(du, u) + Z(u, du))
//                        by the bispectrum coupling program;
//   k_reduce_rows      : deterministic per-component sums over atoms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_util.h"
#include "kernels.h"
#include "snapmd_internal.h"

namespace snapmd {

// level N -> N+1 of column chain P and of its directional derivative D
template <int J, int N>
__device__ __forceinline__ void chain_advance_v(double2 (&P)[J + 1], double2 (&D)[J + 1], double2 b, double2 ab,
                                                double2 dbv, double2 dabv) {
    D[N + 1] = cmul2(dbv, P[N], b, D[N]);
    P[N + 1] = cmul(b, P[N]);
#pragma unroll
    for (int k = N; k >= 1; --k) {
        D[k] = cadd(cmul2(dbv, P[k - 1], b, D[k - 1]), cmul2(dabv, P[k], ab, D[k]));
        P[k] = cmul2(b, P[k - 1], ab, P[k]);
    }
    D[0] = cmul2(dabv, P[0], ab, D[0]);
    P[0] = cmul(ab, P[0]);
}

template <int J, int L>  // n = 2L-1, column L-1 -> L in place: P_L[k] = (-1)^(L-k) conj(P_{L-1}[n-k])
__device__ __forceinline__ void chain_mirror_v(double2 (&P)[J + 1]) {
    constexpr int n = 2 * L - 1;
#pragma unroll
    for (int k = 0; 2 * k < n; ++k) {
        const double2 lo = P[k], hi = P[n - k];
        const double sk = ((L - k) & 1) ? -1.0 : 1.0;
        const double sh = ((L - (n - k)) & 1) ? -1.0 : 1.0;
        P[k] = make_double2(sk * hi.x, -sk * hi.y);
        P[n - k] = make_double2(sh * lo.x, -sh * lo.y);
    }
}

__host__ __device__ constexpr int jvp_acc_idx(int C, int n, int k) { return n * (n + 1) / 2 - C * (2 * C + 1) + k; }

template <int J, int C, int c>
__device__ __forceinline__ void staircase_v(double2 (&P)[J + 1], double2 (&D)[J + 1], double2 b, double2 ab,
                                            double2 dbv, double2 dabv) {
    if constexpr (c < C) {
        chain_advance_v<J, 2 * c>(P, D, b, ab, dbv, dabv);
        chain_mirror_v<J, c + 1>(P);
        chain_mirror_v<J, c + 1>(D);
        chain_advance_v<J, 2 * c + 1>(P, D, b, ab, dbv, dabv);
        staircase_v<J, C, c + 1>(P, D, b, ab, dbv, dabv);
    }
}

template <int J, int C, int N>
__device__ __forceinline__ void jvp_step(double2 (&P)[J + 1], double2 (&D)[J + 1],
                                         double2 (&acc)[jvp_acc_idx(C, J + 1, 0)], double2 b, double2 ab, double2 dbv,
                                         double2 dabv, double fc, double dfcv) {
    if constexpr (N > 2 * C) chain_advance_v<J, N - 1>(P, D, b, ab, dbv, dabv);
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        double2 &a = acc[jvp_acc_idx(C, N, k)];
        a.x = fma(dfcv, P[k].x, fma(fc, D[k].x, a.x));
        a.y = fma(dfcv, P[k].y, fma(fc, D[k].y, a.y));
    }
    if constexpr (N < J) jvp_step<J, C, N + 1>(P, D, acc, b, ab, dbv, dabv, fc, dfcv);
}

template <int J, int C>
__device__ void jvp_column(int N, const int *__restrict__ poff, const int *__restrict__ pair_j,
                           const double *__restrict__ geo, size_t Pcap, const double *__restrict__ w,
                           const double *__restrict__ nrm, double2 *__restrict__ du) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    constexpr int NA = jvp_acc_idx(C, J + 1, 0);
    double2 acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = make_double2(0.0, 0.0);
    const double wi0 = w[i], wi1 = w[N + i], wi2 = w[2 * N + i];
    const int p0 = poff[i], p1 = poff[i + 1];
    double nfc = p0 < p1 ? geo[4 * Pcap + p0] : 0.0;
    for (int p = p0; p < p1; ++p) {
        const double fc = nfc;
        if (p + 1 < p1) nfc = geo[4 * Pcap + p + 1];  // next pair's switch value in flight
        if (fc == 0.0) continue;
        const int j = pair_j[p];
        // the pair vector is x_j - x_i: its variation along the field is w_j - w_i
        const double v[3] = {w[j] - wi0, w[N + j] - wi1, w[2 * N + j] - wi2};
        double2 dav = make_double2(0.0, 0.0), dbv = make_double2(0.0, 0.0);
        double dfcv = 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            dav.x = fma(v[al], geo[(5 + al) * Pcap + p], dav.x);
            dav.y = fma(v[al], geo[(8 + al) * Pcap + p], dav.y);
            dbv.x = fma(v[al], geo[(11 + al) * Pcap + p], dbv.x);
            dbv.y = fma(v[al], geo[(14 + al) * Pcap + p], dbv.y);
            dfcv = fma(v[al], geo[(17 + al) * Pcap + p], dfcv);
        }
        const double2 a = make_double2(geo[p], geo[Pcap + p]);
        const double2 b = make_double2(geo[2 * Pcap + p], geo[3 * Pcap + p]);
        const double2 ab = cconj(a), dabv = cconj(dav);
        double2 P[J + 1], D[J + 1];
        P[0] = make_double2(1.0, 0.0);
        D[0] = make_double2(0.0, 0.0);
        staircase_v<J, C, 0>(P, D, b, ab, dbv, dabv);
        jvp_step<J, C, 2 * C>(P, D, acc, b, ab, dbv, dabv, fc, dfcv);
    }
#pragma unroll
    for (int n = 2 * C; n <= J; ++n)
#pragma unroll
        for (int k = 0; k <= n; ++k) {
            const int e = half_idx(n, k, C);
            const double s = nrm[e];
            const double2 v = acc[jvp_acc_idx(C, n, k)];
            du[(size_t)e * N + i] = make_double2(s * v.x, s * v.y);
        }
}

template <int J>
__global__ void __launch_bounds__(128) k_jvp_density(int N, const int *__restrict__ poff,
                                                     const int *__restrict__ pair_j, const double *__restrict__ geo,
                                                     size_t Pcap, const double *__restrict__ w,
                                                     const double *__restrict__ nrm, double2 *__restrict__ du) {
    switch (blockIdx.y) {
        case 0: jvp_column<J, 0>(N, poff, pair_j, geo, Pcap, w, nrm, du); break;
        case 1: if constexpr (J >= 2) jvp_column<J, 1>(N, poff, pair_j, geo, Pcap, w, nrm, du); break;
        case 2: if constexpr (J >= 4) jvp_column<J, 2>(N, poff, pair_j, geo, Pcap, w, nrm, du); break;
        case 3: if constexpr (J >= 6) jvp_column<J, 3>(N, poff, pair_j, geo, Pcap, w, nrm, du); break;
        case 4: if constexpr (J >= 8) jvp_column<J, 4>(N, poff, pair_j, geo, Pcap, w, nrm, du); break;
        default: break;
    }
}

// dB[t][i] = sum_q c_q Re( conj(du_e) a b + conj(u_e) (da b + a db) ), with the conj flags
// of the bispectrum coupling program applied to a, b and to their variations.
__global__ void __launch_bounds__(256) k_bispectrum_jvp(int N, int K, const double2 *__restrict__ u,
                                                        const double2 *__restrict__ du,
                                                        const int *__restrict__ bstart,
                                                        const uint32_t *__restrict__ bidx,
                                                        const int *__restrict__ bel, const double *__restrict__ bcg,
                                                        double *__restrict__ dB) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int t = 0; t < K; ++t) {
        double acc = 0.0;
        for (int q = bstart[t]; q < bstart[t + 1]; ++q) {
            const uint32_t wq = bidx[q];
            const size_t h1 = (size_t)(wq & 0xfffu) * N + i, h2 = (size_t)((wq >> 12) & 0xfffu) * N + i;
            double2 a = u[h1], b = u[h2], da = du[h1], db = du[h2];
            if (wq & (1u << 24)) { a.y = -a.y; da.y = -da.y; }
            if (wq & (1u << 25)) { b.y = -b.y; db.y = -db.y; }
            const size_t he = (size_t)bel[q] * N + i;
            const double2 ue = u[he], due = du[he];
            const double2 ab = cmul(a, b);
            const double2 dab = cadd(cmul(da, b), cmul(a, db));
            acc = fma(bcg[q], (due.x * ab.x + due.y * ab.y) + (ue.x * dab.x + ue.y * dab.y), acc);
        }
        dB[(size_t)t * N + i] = acc;
    }
}

// out[r * ostride] = scale * sum_i in[r][i]  (one workgroup per row, fixed summation order)
__global__ void __launch_bounds__(256) k_reduce_rows(int N, const double *__restrict__ in, double scale,
                                                     double *__restrict__ out) {
    __shared__ double red[256];
    const int r = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int i = t; i < N; i += 256) s += in[(size_t)r * N + i];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) out[r] = scale * red[0];
}

__global__ void k_set_value(double *__restrict__ p, double v) { *p = v; }

// ---------------------------------------------------------------------------
void launch_jvp_density(int J, int N, const Work &w, const double *wf, const double *nrm, double2 *du,
                        hipStream_t st) {
    const dim3 g((N + 127) / 128, J / 2 + 1);
    switch (J) {
        case 2: hipLaunchKernelGGL(k_jvp_density<2>, g, dim3(128), 0, st, N, w.poff, w.pair_j, w.geo, w.Pcap, wf, nrm, du); break;
        case 4: hipLaunchKernelGGL(k_jvp_density<4>, g, dim3(128), 0, st, N, w.poff, w.pair_j, w.geo, w.Pcap, wf, nrm, du); break;
        case 6: hipLaunchKernelGGL(k_jvp_density<6>, g, dim3(128), 0, st, N, w.poff, w.pair_j, w.geo, w.Pcap, wf, nrm, du); break;
        case 8: hipLaunchKernelGGL(k_jvp_density<8>, g, dim3(128), 0, st, N, w.poff, w.pair_j, w.geo, w.Pcap, wf, nrm, du); break;
        default: break;
    }
}

void launch_bispectrum_jvp(int N, const SnapDev &sd, const double2 *u, const double2 *du, double *dB,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_bispectrum_jvp, dim3((N + 255) / 256), dim3(256), 0, st, N, sd.K, u, du, sd.bstart, sd.bidx,
                       sd.bel, sd.bcg, dB);
}

void launch_reduce_rows(int rows, int N, const double *in, double scale, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, st, N, in, scale, out);
}

void launch_set_value(double *p, double v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_value, dim3(1), dim3(1), 0, st, p, v);
}

}  // namespace snapmd
