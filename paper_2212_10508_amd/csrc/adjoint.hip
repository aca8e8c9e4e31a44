// SNAP adjoint Y = 2 dE/d conj(u) and atomic energy, LDS-staged (gfx950, FP64).
//
// One workgroup owns a tile of 64 atoms (lane = atom) and stages their densities u
// (half storage, [element][64] double2) in LDS.  Its waves own disjoint sets of
// output rows m (2m in -J..J, balanced by cost on the host); control flow and all
// coupling coefficients are wave-uniform.  For output row m, coupling block
// (j1 >= j2) and left index m1 (m2 = m - m1), the row u^{j2}[m2][.] is read from LDS
// into registers, the entries of u^{j1}[m1][.] are taken from LDS one at a time (so the
// kernel fits 168 registers: three waves per SIMD), and a compile-time-unrolled
// "row-pair motif" forms
//   c_j[m'] = sum_{m1'+m2'=m'} C^{j m'}_{j1 m1', j2 m2'} u^{j1}[m1][m1'] u^{j2}[m2][m2']
// for every coupled level j and m' <= 0 (each product u u shared by all j), then
//   Y^j[m][m'] += beta~(j1,j2,j) C^{j m}_{j1 m1, j2 m2} c_j[m'].
// beta~ is the adjoint weight beta_k * mult * (2 j_max + 1)/(2 j + 1) of the coupling
// block (see tables.cpp).  Rows above the half are recovered with
// u[n-k][n-l] = (-1)^(k-l) conj(u[k][l]).
// Outputs: Y~ = Y * Nrm * mult (the factor the force pass contracts with) and
// E_i = beta0 + (1/3) sum_e mult_e Re(conj(Y_e) u_e) (Euler's identity for the cubic E).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "device_util.h"
#include "kernels.h"
#include "snapmd_internal.h"

namespace snapmd {

// ---------------------------------------------------------------------------
// compile-time structure
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cpl_lo(int N1, int N2) { return N1 - N2; }
__host__ __device__ constexpr int cpl_hi(int J, int N1, int N2) { return cmin(J, N1 + N2); }
__host__ __device__ constexpr int cpl_n(int J, int N1, int N2) { return (cpl_hi(J, N1, N2) - cpl_lo(N1, N2)) / 2 + 1; }
__host__ __device__ constexpr int blk_index(int N1, int N2) { return N1 * (N1 + 1) / 2 + N2; }
__host__ __device__ constexpr int n_blocks(int J) { return (J + 1) * (J + 2) / 2; }

// c layout of block (N1,N2): levels n of its coupling set, columns l = 0..n/2
// (closed form of sum_{m = lo, lo+2, .., n-2} (floor(m/2) + 1) + l)
__host__ __device__ constexpr int c_index(int N1, int N2, int n, int l) {
    const int lo = cpl_lo(N1, N2), cnt = (n - lo) / 2;
    return cnt * ((lo - (lo & 1)) / 2 + 1) + cnt * (cnt - 1) / 2 + l;
}
__host__ __device__ constexpr int c_size(int J, int N1, int N2) {
    return c_index(N1, N2, cpl_hi(J, N1, N2) + 2, 0);
}
// Y layout for output rows of parity P (2m = P mod 2): levels n = P, P+2, .. <= J
__host__ __device__ constexpr int y_index(int P, int n, int l) {
    const int cnt = (n - P) / 2;
    return cnt * (cnt + 1) / 2 + l;
}
__host__ __device__ constexpr int y_size(int J, int P) {
    int o = 0;
    for (int m = P; m <= J; m += 2) o += m / 2 + 1;
    return o;
}
// number of motif constants of block (N1,N2)
__host__ __device__ constexpr int motif_terms(int J, int N1, int N2) {
    int t = 0;
    for (int l1 = 0; l1 <= N1; ++l1)
        for (int l2 = 0; l2 <= N2; ++l2) {
            const int tmp = (2 * l1 - N1) + (2 * l2 - N2);  // 2m'
            if (tmp > 0) continue;
            for (int n = cpl_lo(N1, N2); n <= cpl_hi(J, N1, N2); n += 2)
                if (-tmp <= n) ++t;
        }
    return t;
}
__host__ __device__ constexpr int motif_off(int J, int N1, int N2) {
    int o = 0;
    for (int a = 0; a <= J; ++a)
        for (int b = 0; b <= a; ++b) {
            if (a == N1 && b == N2) return o;
            o += motif_terms(J, a, b);
        }
    return o;
}

// ---------------------------------------------------------------------------
// device pieces
// ---------------------------------------------------------------------------
// Full row k of level N from half storage in LDS ([e][64] double2, lane-offset base).
template <int N>
__device__ __forceinline__ void load_row(const double2 *__restrict__ lds, int k, double2 (&r)[N + 1]) {
    constexpr int h0 = half_off(N);
    const double sk = (k & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int l = 0; l <= N; ++l) {
        if (2 * l <= N) {
            r[l] = lds[(h0 + l * (N + 1) + k) * 64];
        } else {
            const double2 v = lds[(h0 + (N - l) * (N + 1) + (N - k)) * 64];
            const double s = (l & 1) ? -sk : sk;  // (-1)^(k-l)
            r[l] = make_double2(s * v.x, -s * v.y);
        }
    }
}

template <int N>
__device__ __forceinline__ double2 load_entry(const double2 *__restrict__ lds, int k, int l) {
    constexpr int h0 = half_off(N);
    if (2 * l <= N) return lds[(h0 + l * (N + 1) + k) * 64];
    const double2 v = lds[(h0 + (N - l) * (N + 1) + (N - k)) * 64];
    const double s = ((k - l) & 1) ? -1.0 : 1.0;
    return make_double2(s * v.x, -s * v.y);
}

template <int J, int N1, int N2>
__device__ __forceinline__ void motif(const double2 *__restrict__ lds, int k1, const double2 (&r2)[N2 + 1],
                                      const double *__restrict__ cg, double2 (&c)[c_size(J, N1, N2)]) {
    int t = 0;
#pragma unroll
    for (int l1 = 0; l1 <= N1; ++l1) {
        const double2 r1l = load_entry<N1>(lds, k1, l1);
#pragma unroll
        for (int l2 = 0; l2 <= N2; ++l2) {
            const int tmp = (2 * l1 - N1) + (2 * l2 - N2);
            if (tmp > 0) continue;
            const double2 P = cmul(r1l, r2[l2]);
#pragma unroll
            for (int n = cpl_lo(N1, N2); n <= cpl_hi(J, N1, N2); n += 2) {
                if (-tmp > n) continue;
                const int l = (tmp + n) / 2;
                const double w = cg[t++];
                double2 &cc = c[c_index(N1, N2, n, l)];
                cc.x = fma(w, P.x, cc.x);
                cc.y = fma(w, P.y, cc.y);
            }
        }
    }
}

template <int J, int P, int N1, int N2>
__device__ __forceinline__ void do_block(int tm, const double2 *__restrict__ lds, const double *__restrict__ cgm,
                                         const double *__restrict__ coef, const int *__restrict__ coef_off,
                                         double2 (&Y)[y_size(J, P)]) {
    // A diagonal block (N1 == N2) pairs row m1 with m2 = m - m1 and row m2 with m1: the two
    // give the same contribution (the CG symmetry under exchange of the two couplings,
    // applied to both coefficients, with equal signs), so only 2 m1 <= m is visited and the
    // host table carries the doubled coefficient for 2 m1 < m.
    const int lo = max(-N1, tm - N2), hi = (N1 == N2) ? min(N1, tm / 2) : min(N1, tm + N2);
    if (lo > hi) return;
    constexpr int NCP = cpl_n(J, N1, N2);
    constexpr int NC = c_size(J, N1, N2);
    constexpr int MO = motif_off(J, N1, N2);
    constexpr int BI = blk_index(N1, N2);
    constexpr int NB = n_blocks(J);
    const double *cg = cgm + MO;
    int off = coef_off[(tm + J) * NB + BI];
    for (int tm1 = lo; tm1 <= hi; tm1 += 2, off += NCP) {
        // The motif's coupling constants are loop-invariant; left to itself the compiler
        // hoists them out of this loop, runs out of scalar registers and parks them in
        // vector-register lanes (two v_readlane per constant, one per FMA pair).  An
        // offset the compiler cannot see through keeps the scalar loads inside the loop,
        // so every FMA takes its constant straight from a scalar register.
        int opq = 0;
        asm volatile("" : "+s"(opq));
        const double *cgi = cg + opq;
        double2 r2[N2 + 1];
        load_row<N2>(lds, (tm - tm1 + N2) / 2, r2);
        double2 c[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) c[q] = make_double2(0.0, 0.0);
        motif<J, N1, N2>(lds, (tm1 + N1) / 2, r2, cgi, c);
#pragma unroll
        for (int n = cpl_lo(N1, N2); n <= cpl_hi(J, N1, N2); n += 2) {
            const double w = coef[off + (n - cpl_lo(N1, N2)) / 2];
#pragma unroll
            for (int l = 0; 2 * l <= n; ++l) {
                double2 &y = Y[y_index(P, n, l)];
                const double2 v = c[c_index(N1, N2, n, l)];
                y.x = fma(w, v.x, y.x);
                y.y = fma(w, v.y, y.y);
            }
        }
    }
}

template <int J, int P, int N1, int N2>
__device__ __forceinline__ void all_blocks(int tm, const double2 *__restrict__ lds, const double *__restrict__ cgm,
                                           const double *__restrict__ coef, const int *__restrict__ coef_off,
                                           double2 (&Y)[y_size(J, P)]) {
    if constexpr (((N1 + N2) & 1) == P) do_block<J, P, N1, N2>(tm, lds, cgm, coef, coef_off, Y);
    if constexpr (N2 < N1) all_blocks<J, P, N1, N2 + 1>(tm, lds, cgm, coef, coef_off, Y);
    else if constexpr (N1 < J) all_blocks<J, P, N1 + 1, 0>(tm, lds, cgm, coef, coef_off, Y);
}

template <int J, int P>
__device__ __forceinline__ double process_row(int tm, int atom, int N, const double2 *__restrict__ lds,
                                              const double *__restrict__ cgm, const double *__restrict__ coef,
                                              const int *__restrict__ coef_off, const double *__restrict__ nrm,
                                              const double *__restrict__ ymult, double2 *__restrict__ ytil) {
    constexpr int NY = y_size(J, P);
    double2 Y[NY];
#pragma unroll
    for (int q = 0; q < NY; ++q) Y[q] = make_double2(0.0, 0.0);
    all_blocks<J, P, 0, 0>(tm, lds, cgm, coef, coef_off, Y);
    double esum = 0.0;
    const int atm = tm < 0 ? -tm : tm;
#pragma unroll
    for (int n = P; n <= J; n += 2) {
        if (n < atm) continue;
        const int k = (tm + n) / 2;
#pragma unroll
        for (int l = 0; 2 * l <= n; ++l) {
            if (2 * l == n && tm > 0) continue;  // mirrored half of the middle column
            const int e = half_off(n) + l * (n + 1) + k;
            const double2 y = Y[y_index(P, n, l)];
            const double m = ymult[e];
            const double s = m * nrm[e];
            if (atom < N) ytil[(size_t)e * N + atom] = make_double2(s * y.x, s * y.y);
            const double2 ue = lds[e * 64];
            esum = fma(m, fma(y.x, ue.x, y.y * ue.y), esum);
        }
    }
    return esum;
}

// R waves per workgroup (the kernel-shape choice of this pass: 12, three per SIMD, or 8)
// u2 non-null: the density comes in two parts (u + u2), added as the tile is loaded.
template <int J, int R>
__global__ void __launch_bounds__(64 * R) k_adjoint_lds(int N, const double2 *__restrict__ u,
                                                     const double2 *__restrict__ u2,
                                                     const double *__restrict__ cgm, const double *__restrict__ coef,
                                                     const int *__restrict__ coef_off, const int *__restrict__ roles,
                                                     int role_len, const double *__restrict__ nrm,
                                                     const double *__restrict__ ymult, double beta0,
                                                     double2 *__restrict__ ytil, double *__restrict__ e_atom,
                                                     int accumulate_e) {
    extern __shared__ double2 lds[];
    __shared__ int simd_waves[4];
    constexpr int NH = n_half(J);
    constexpr int PER = R / 4;  // waves per SIMD (one workgroup fills the compute unit)
    const int a0 = blockIdx.x * 64;
    if (threadIdx.x < 4) simd_waves[threadIdx.x] = 0;
    for (int idx = threadIdx.x; idx < NH * 64; idx += 64 * R) {
        const int e = idx >> 6, a = idx & 63;
        double2 v = make_double2(0.0, 0.0);
        if (a0 + a < N) {
            v = u[(size_t)e * N + a0 + a];
            if (u2) v = cadd(v, u2[(size_t)e * N + a0 + a]);
        }
        lds[idx] = v;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // The roles are balanced per SIMD (the waves of one SIMD share its FP64 unit): a wave
    // takes role PER * simd + (its arrival rank on that SIMD), whatever order the hardware
    // placed the waves in.  If the waves are not spread PER to a SIMD, role = wave index.
    const int simd = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_s_getreg((1 << 11) | (4 << 6) | 4));
    int slot = 0;
    if (lane == 0) slot = atomicAdd(&simd_waves[simd], 1);
    slot = __builtin_amdgcn_readfirstlane(slot);
    __syncthreads();
    const bool spread = simd_waves[0] == PER && simd_waves[1] == PER && simd_waves[2] == PER && simd_waves[3] == PER;
    const int role = spread ? simd * PER + slot : wave;
    const double2 *my = lds + lane;
    double esum = 0.0;
    for (int q = 0; q < role_len; ++q) {
        const int tm = roles[role * role_len + q];
        if (tm > J) break;
        if ((tm & 1) == 0)
            esum += process_row<J, 0>(tm, a0 + lane, N, my, cgm, coef, coef_off, nrm, ymult, ytil);
        else
            esum += process_row<J, 1>(tm, a0 + lane, N, my, cgm, coef, coef_off, nrm, ymult, ytil);
    }
    __syncthreads();  // every wave is done with the u tile: reuse it for the energy partials
    double *epart = reinterpret_cast<double *>(lds);  // [R][64], by role (a fixed summation order)
    epart[role * 64 + lane] = esum;
    __syncthreads();
    if (wave == 0 && e_atom && a0 + lane < N) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < R; ++w) s += epart[w * 64 + lane];
        const double en = beta0 + s / 3.0;
        e_atom[a0 + lane] = accumulate_e ? e_atom[a0 + lane] + en : en;
    }
}

// ---------------------------------------------------------------------------
// host side: tables and launch
// ---------------------------------------------------------------------------
constexpr int kAdjWaves = 12;

// Items (indices into cost, in decreasing cost order) to nb bins with the largest bin load
// as small as possible: branch and bound seeded with the longest-processing-time-first
// assignment, bins of equal load tried once, at most 4e6 nodes.  Returns the bin of each
// item (in the order given).
static std::vector<int> partition_rows(const std::vector<double> &cost, const std::vector<int> &items, int nb) {
    const size_t n = items.size();
    std::vector<int> best(n), cur(n);
    std::vector<double> load(nb, 0.0);
    for (size_t k = 0; k < n; ++k) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        best[k] = b;
        load[b] += cost[items[k]];
    }
    double bound = *std::max_element(load.begin(), load.end());
    std::fill(load.begin(), load.end(), 0.0);
    long nodes = 0;
    std::vector<int> stack_bin(n, -1);  // iterative depth-first search
    size_t k = 0;
    while (true) {
        if (k == n) {
            const double m = *std::max_element(load.begin(), load.end());
            if (m < bound) {
                bound = m;
                best = cur;
            }
            if (k == 0) break;
            --k;
            load[cur[k]] -= cost[items[k]];
            continue;
        }
        int b = stack_bin[k] + 1;
        const double c = cost[items[k]];
        for (; b < nb; ++b) {
            bool dup = false;  // a bin with the load of an earlier one gives the same subtrees
            for (int e = 0; e < b && !dup; ++e) dup = load[e] == load[b];
            if (!dup && load[b] + c < bound) break;
        }
        if (b >= nb || ++nodes > 4000000) {
            stack_bin[k] = -1;
            if (k == 0 || nodes > 4000000) break;
            --k;
            load[cur[k]] -= cost[items[k]];
            continue;
        }
        stack_bin[k] = b;
        cur[k] = b;
        load[b] += c;
        ++k;
    }
    return best;
}

void adjoint_tables(int J, const double *beta, AdjointHost &A) {
    const SnapTables &T = snap_tables(J);
    const int NB = n_blocks(J);
    // map (n1, n2, n) -> Z block of SnapTables (canonical triple, adjoint weight)
    auto zb = [&](int n1, int n2, int n) {
        for (size_t b = 0; b < T.zb_n.size(); ++b)
            if (T.zb_n1[b] == n1 && T.zb_n2[b] == n2 && T.zb_n[b] == n) return (int)b;
        return -1;
    };
    if (A.J != J) {
        A.J = J;
        A.cgm.clear();
        for (int n1 = 0; n1 <= J; ++n1)
            for (int n2 = 0; n2 <= n1; ++n2)
                for (int l1 = 0; l1 <= n1; ++l1)
                    for (int l2 = 0; l2 <= n2; ++l2) {
                        const int tmp = (2 * l1 - n1) + (2 * l2 - n2);
                        if (tmp > 0) continue;
                        for (int n = n1 - n2; n <= std::min(J, n1 + n2); n += 2)
                            if (-tmp <= n) A.cgm.push_back(cg_coeff(n1, l1, n2, l2, n, (tmp + n) / 2));
                    }
        // cost of each output row 2m (products + terms + row updates), for role balancing
        std::vector<double> cost(2 * J + 1, 0.0);
        for (int tm = -J; tm <= J; ++tm)
            for (int n1 = 0; n1 <= J; ++n1)
                for (int n2 = 0; n2 <= n1; ++n2) {
                    if (((n1 + n2 - tm) & 1) != 0) continue;
                    const int lo = std::max(-n1, tm - n2), hi = std::min(n1, tm + n2);
                    if (lo > hi) continue;
                    const double mt = motif_terms(J, n1, n2);
                    const int hk = n1 == n2 ? std::min(hi, tm / 2) : hi;  // diagonal blocks: half the rows
                    cost[tm + J] += ((hk - lo) / 2 + 1) * (3.0 * mt + 2.0 * (n1 + n2 + 2) + 2.0 * c_size(J, n1, n2));
                }
        std::vector<int> order(2 * J + 1);
        for (int i = 0; i <= 2 * J; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        // rows to SIMDs, then each SIMD's rows to its waves (12 waves: three per SIMD, 8: two)
        auto assign = [&](int nw, std::vector<int> &flat, int &len) {
            const int per = nw / 4;
            std::vector<std::vector<int>> roles(nw);
            const std::vector<int> simd_of = partition_rows(cost, order, 4);
            for (int sd = 0; sd < 4; ++sd) {
                std::vector<int> mine;
                for (size_t q = 0; q < order.size(); ++q)
                    if (simd_of[q] == sd) mine.push_back(order[q]);
                const std::vector<int> wave_of = partition_rows(cost, mine, per);
                for (size_t q = 0; q < mine.size(); ++q) roles[sd * per + wave_of[q]].push_back(mine[q] - J);
            }
            len = 0;
            for (auto &r : roles) len = std::max(len, (int)r.size() + 1);
            flat.assign(nw * len, 1 << 20);
            for (int w = 0; w < nw; ++w)
                for (size_t q = 0; q < roles[w].size(); ++q) flat[w * len + q] = roles[w][q];
        };
        assign(kAdjWaves, A.roles, A.role_len);
        assign(8, A.roles8, A.role_len8);
        A.beta.clear();
    }
    if (A.beta.size() == (size_t)T.K + 1 && std::equal(A.beta.begin(), A.beta.end(), beta)) return;
    A.beta.assign(beta, beta + T.K + 1);
    A.coef.clear();
    A.coef_off.assign((2 * J + 1) * NB, -1);
    for (int tm = -J; tm <= J; ++tm)
        for (int n1 = 0; n1 <= J; ++n1)
            for (int n2 = 0; n2 <= n1; ++n2) {
                if (((n1 + n2 - tm) & 1) != 0) continue;
                const int lo = std::max(-n1, tm - n2), hi = std::min(n1, tm + n2);
                if (lo > hi) continue;
                A.coef_off[(tm + J) * NB + blk_index(n1, n2)] = (int)A.coef.size();
                // diagonal blocks: m1 <= m - m1 only, the pair (m1, m - m1) counted twice
                const int hk = n1 == n2 ? std::min(hi, tm / 2) : hi;
                for (int tm1 = lo; tm1 <= hk; tm1 += 2)
                    for (int n = n1 - n2; n <= std::min(J, n1 + n2); n += 2) {
                        double v = 0.0;
                        if (std::abs(tm) <= n) {
                            const int b = zb(n1, n2, n);
                            const double bt = T.zb_wt[b] * A.beta[1 + T.zb_canon[b]];
                            v = bt * cg_coeff(n1, (tm1 + n1) / 2, n2, (tm - tm1 + n2) / 2, n, (tm + n) / 2);
                            if (n1 == n2 && 2 * tm1 < tm) v *= 2.0;
                        }
                        A.coef.push_back(v);
                    }
            }
    A.coef_changed = true;
}

size_t adjoint_lds_bytes(int J) {
    return std::max((size_t)n_half(J) * 64 * sizeof(double2), (size_t)kAdjWaves * 64 * sizeof(double));
}

template <int J>
static void launch_adj(const AdjointDev &ad, int waves, int N, const double2 *u, const double2 *u2, const double *nrm,
                       const double *ymult, double beta0, double2 *ytil, double *e_atom, int accumulate,
                       hipStream_t st) {
    const size_t lds = adjoint_lds_bytes(J);
    if (waves == 8 && ad.roles8)
        hipLaunchKernelGGL((k_adjoint_lds<J, 8>), dim3((N + 63) / 64), dim3(64 * 8), lds, st, N, u, u2, ad.cgm, ad.coef,
                           ad.coef_off, ad.roles8, ad.role_len8, nrm, ymult, beta0, ytil, e_atom, accumulate);
    else
        hipLaunchKernelGGL((k_adjoint_lds<J, kAdjWaves>), dim3((N + 63) / 64), dim3(64 * kAdjWaves), lds, st, N, u,
                           u2, ad.cgm, ad.coef, ad.coef_off, ad.roles, ad.role_len, nrm, ymult, beta0, ytil, e_atom,
                           accumulate);
}

void launch_adjoint(int J, const AdjointDev &ad, int N, const double2 *u, const double2 *u2, const double *nrm,
                    const double *ymult, double beta0, double2 *ytil, double *e_atom, int accumulate, hipStream_t st,
                    int waves) {
    switch (J) {
        case 2: launch_adj<2>(ad, waves, N, u, u2, nrm, ymult, beta0, ytil, e_atom, accumulate, st); break;
        case 4: launch_adj<4>(ad, waves, N, u, u2, nrm, ymult, beta0, ytil, e_atom, accumulate, st); break;
        case 6: launch_adj<6>(ad, waves, N, u, u2, nrm, ymult, beta0, ytil, e_atom, accumulate, st); break;
        case 8: launch_adj<8>(ad, waves, N, u, u2, nrm, ymult, beta0, ytil, e_atom, accumulate, st); break;
        default: break;
    }
}

void adjoint_init_attributes() {
    (void)hipFuncSetAttribute((const void *)k_adjoint_lds<8, kAdjWaves>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)adjoint_lds_bytes(8));
    (void)hipFuncSetAttribute((const void *)k_adjoint_lds<6, kAdjWaves>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)adjoint_lds_bytes(6));
    (void)hipFuncSetAttribute((const void *)k_adjoint_lds<8, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)adjoint_lds_bytes(8));
    (void)hipFuncSetAttribute((const void *)k_adjoint_lds<6, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)adjoint_lds_bytes(6));
}

}  // namespace snapmd
