// Candidate stencils and their coefficients for ENO-MR (arXiv 2311.15504, Sec. 3).
//
// The candidate pool is the 29-stencil list of Eq. (Candidates); the pool of a
// (2r-1)-point scheme keeps, in the same order, the stencils S_{j-m}^{j+n} with
// m, n <= r-1.  Coefficients are generated on the host in exact rational
// arithmetic:
//   a_l  (Eq. ReconstructedFlux): the reconstruction polynomial is the
//        derivative of the polynomial V that interpolates the primitive of H at
//        the stencil's interfaces; a_l = sum over interfaces to the right of
//        cell l of the Lagrange basis derivatives at x_{j+1/2}.
//   b_l  (Eq. CurrentIS/ISCoe): h^{m+n} d^{m+n}P/dx^{m+n} is the (m+n)-th
//        undivided difference, b_l = (-1)^{m+n-(l+m)} C(m+n, l+m).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace enomr {

constexpr int kPool = 29;   // stencils in the 17-point pool
constexpr int kMaxW = 17;   // widest stencil

// Eq. (Candidates): S_{j-m}^{j+n} as (m, n), in selection order.
__host__ __device__ constexpr int pool_mn(int c, int which)
{
    constexpr int t[kPool][2] = {
        {8, 8}, {7, 8}, {8, 7}, {7, 7}, {8, 6}, {6, 7}, {7, 6}, {6, 6}, {7, 5},
        {5, 6}, {6, 5}, {5, 5}, {6, 4}, {4, 5}, {5, 4}, {4, 4}, {5, 3}, {3, 4}, {4, 3},
        {3, 3}, {2, 3}, {3, 2}, {2, 2}, {1, 2}, {2, 1}, {1, 1}, {0, 1}, {1, 0}, {0, 0}};
    return t[c][which];
}

// Number of candidates of the (2R-1)-point scheme.
__host__ __device__ constexpr int n_cands(int R)
{
    int k = 0;
    for (int c = 0; c < kPool; ++c)
        if (pool_mn(c, 0) <= R - 1 && pool_mn(c, 1) <= R - 1) ++k;
    return k;
}

// Pool index of the C-th candidate of the (2R-1)-point scheme.
__host__ __device__ constexpr int cand_pool(int R, int C)
{
    int k = 0;
    for (int c = 0; c < kPool; ++c)
        if (pool_mn(c, 0) <= R - 1 && pool_mn(c, 1) <= R - 1) {
            if (k == C) return c;
            ++k;
        }
    return -1;
}

// Host-side generation of a_l and b_l for every pool stencil, as doubles
// nearest to the exact rationals.  a[c][l+m], b[c][l+m].
bool generate_tables(double a[kPool][kMaxW], double b[kPool][kMaxW]);

}  // namespace enomr
