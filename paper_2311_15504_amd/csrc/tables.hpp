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

// a_l and b_l of every pool stencil, a[c][l+m], b[c][l+m], generated at
// compile time in exact rational arithmetic and rounded to the nearest
// doubles.  Kernels index the table with compile-time positions, so the
// coefficients become instruction immediates.
namespace coefgen {

typedef __int128 i128;

constexpr i128 iabs(i128 x) { return x < 0 ? -x : x; }

constexpr i128 gcd(i128 a, i128 b)
{
    a = iabs(a);
    b = iabs(b);
    while (b != 0) {
        const i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

struct Rat {
    i128 p, q;   // q > 0, reduced
};

constexpr Rat make(i128 p, i128 q)
{
    if (q < 0) { p = -p; q = -q; }
    i128 g = gcd(p, q);
    if (g == 0) g = 1;
    return Rat{p / g, q / g};
}

constexpr Rat add(Rat x, Rat y) { return make(x.p * y.q + y.p * x.q, x.q * y.q); }

// Derivative at interface node s of the Lagrange basis polynomial of node q,
// nodes at the integers 0..K (unit spacing).
constexpr Rat basis_derivative(int q, int s, int K)
{
    if (q != s) {
        i128 num = 1, den = 1;
        for (int t = 0; t <= K; ++t) {
            if (t != q && t != s) num *= (s - t);
            if (t != q) den *= (q - t);
        }
        return make(num, den);
    }
    Rat acc = make(0, 1);
    for (int t = 0; t <= K; ++t)
        if (t != s) acc = add(acc, make(1, s - t));
    return acc;
}

constexpr i128 binom(int n, int k)
{
    i128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Reduced numerators and denominators stay below 2^53 (checked when the
// table is built), so both convert exactly and one IEEE division rounds the
// quotient correctly.
constexpr double to_double(Rat x) { return (double)(long long)x.p / (double)(long long)x.q; }
constexpr bool fits(Rat x) { return iabs(x.p) < (((i128)1) << 53) && x.q < (((i128)1) << 53); }

struct CoefTable {
    double a[kPool][kMaxW];
    double b[kPool][kMaxW];
    bool exact;   // every rational converted exactly before rounding
};

constexpr CoefTable make_table()
{
    CoefTable t{};
    t.exact = true;
    for (int c = 0; c < kPool; ++c) {
        const int m = pool_mn(c, 0), n = pool_mn(c, 1);
        const int K = m + n + 1;   // interfaces x_{j-m-1/2} .. x_{j+n+1/2} -> nodes 0..K
        const int s = m + 1;       // x_{j+1/2}
        Rat d[kMaxW + 2] = {};
        for (int q = 0; q <= K; ++q) d[q] = basis_derivative(q, s, K);
        for (int i = 0; i < K; ++i) {
            // a_i: sum over interfaces right of cell i of the basis derivatives
            Rat acc = make(0, 1);
            for (int q = i + 1; q <= K; ++q) acc = add(acc, d[q]);
            t.exact = t.exact && fits(acc);
            t.a[c][i] = to_double(acc);
            const int deg = m + n;
            i128 bv = binom(deg, i);
            if ((deg - i) % 2) bv = -bv;
            t.b[c][i] = (double)(long long)bv;
        }
    }
    return t;
}

}  // namespace coefgen

inline constexpr coefgen::CoefTable kCoef = coefgen::make_table();
static_assert(kCoef.exact, "a coefficient's numerator or denominator exceeds 2^53");

// Host copies of the table (a[c][l+m], b[c][l+m]).
bool generate_tables(double a[kPool][kMaxW], double b[kPool][kMaxW]);

}  // namespace enomr
