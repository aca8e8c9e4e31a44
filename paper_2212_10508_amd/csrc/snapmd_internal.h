// Internal declarations shared by the snapmd HIP sources (not part of the C ABI).
//
// Index conventions (2j-integers): level n = 2j in 0..J (J = twojmax); rows k and
// columns l of the (n+1)x(n+1) Wigner-D block in 0..n (m = k - n/2, m' = l - n/2).
// "Half" storage keeps the columns l <= n/2 of every level; the rest follows from
//   D[n-k][n-l] = (-1)^(k-l) conj(D[k][l]),
// which every density u, adjoint Y and derivative block inherits.
// Half index of (n, k, l):  half_off(n) + l*(n+1) + k.
//
// The Wigner-D blocks are built from unnormalised polynomial coefficients
//   P^n[k][l] = coefficient of u^k v^(n-k) in (a u - conj(b) v)^l (b u + conj(a) v)^(n-l),
//   D^n[k][l] = Nrm(n,k,l) P^n[k][l],  Nrm(n,k,l) = sqrt(k!(n-k)! / (l!(n-l)!)),
// so that a column advances one level by P^{n+1}[k][l] = b P^n[k-1][l] + conj(a) P^n[k][l]
// (no square roots), and Nrm(n,n-k,n-l) = Nrm(n,k,l) keeps the mirror relation for P.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace snapmd {

constexpr int kMaxJ = 14;     // largest twojmax (SNAP-205)
constexpr int kMaxJLds = 8;   // largest twojmax of the LDS-tiled adjoint
constexpr int kMaxNeigh = 64;

// half_off(n) = sum_{m<n} (m+1)(floor(m/2)+1), in closed form so that it folds to a
// constant wherever n is one (levels m = 2i and 2i+1 contribute (i+1)(4i+3)).
__host__ __device__ constexpr int half_off(int n) {
    const int q = n / 2;
    const int pairs = 4 * ((q - 1) * q * (2 * q - 1) / 6) + 7 * (q * (q - 1) / 2) + 3 * q;
    return pairs + ((n & 1) ? (2 * q + 1) * (q + 1) : 0);
}
__host__ __device__ constexpr int half_idx(int n, int k, int l) { return half_off(n) + l * (n + 1) + k; }
__host__ __device__ constexpr int n_half(int J) { return half_off(J + 1); }

// Host tables for one twojmax.
struct SnapTables {
    int J = -1;
    int K = 0;                         // bispectrum components
    int nh = 0;                        // half elements
    std::vector<double> nrm;           // [nh] Nrm(n,k,l)
    std::vector<double> ymult;         // [nh] multiplicity of the element in full sums (0,1,2)
    std::vector<int> elem_n, elem_k, elem_l;
    // Y program: for output element e, terms [ystart[e], ystart[e+1])
    std::vector<int> ystart;
    std::vector<uint32_t> yidx;        // h1 | h2 << 12 | conj1 << 24 | conj2 << 25
    std::vector<double> ycg;           // CG product * mirror signs (beta-free)
    std::vector<int> yblock;           // Z block of the term (to apply beta tilde)
    // Z blocks (n1 >= n2, n) and their beta-tilde recipe
    std::vector<int> zb_n1, zb_n2, zb_n, zb_canon;  // canonical triple index of the block
    std::vector<double> zb_wt;                     // mult * (r+1)/(n+1)
    // canonical triples
    std::vector<int> tr_n1, tr_n2, tr_n;
    // B program: for triple t, terms [bstart[t], bstart[t+1]): element e, u1, u2, weight
    std::vector<int> bstart;
    std::vector<uint32_t> bidx;        // as yidx plus element e in bits 0..11 of bel
    std::vector<int> bel;
    std::vector<double> bcg;           // CG product * mirror signs * ymult(e)
};

const SnapTables &snap_tables(int J);
double cg_coeff(int n1, int k1, int n2, int k2, int n, int k);
int snap_ncoeff(int J);

}  // namespace snapmd
