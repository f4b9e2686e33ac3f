// Exact-rational generation of the ENO-MR stencil coefficients (host only).
#include "tables.hpp"

#include <cstdlib>

namespace enomr {
namespace {

typedef __int128 i128;

i128 iabs(i128 x) { return x < 0 ? -x : x; }

i128 gcd(i128 a, i128 b)
{
    a = iabs(a);
    b = iabs(b);
    while (b != 0) {
        i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

struct Rat {
    i128 p, q;   // q > 0, reduced
};

Rat make(i128 p, i128 q)
{
    if (q < 0) { p = -p; q = -q; }
    i128 g = gcd(p, q);
    if (g == 0) g = 1;
    return Rat{p / g, q / g};
}

Rat add(Rat x, Rat y) { return make(x.p * y.q + y.p * x.q, x.q * y.q); }

// Derivative at interface node s of the Lagrange basis polynomial of node q,
// nodes at the integers 0..K (unit spacing).
Rat basis_derivative(int q, int s, int K)
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

i128 binom(int n, int k)
{
    i128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

double to_double(Rat x)
{
    // reduced numerators and denominators here stay far below 2^53, so both
    // convert exactly and one IEEE division rounds the quotient correctly
    const i128 lim = ((i128)1) << 53;
    if (iabs(x.p) >= lim || x.q >= lim) std::abort();
    return (double)(long long)x.p / (double)(long long)x.q;
}

}  // namespace

bool generate_tables(double a[kPool][kMaxW], double b[kPool][kMaxW])
{
    for (int c = 0; c < kPool; ++c) {
        for (int l = 0; l < kMaxW; ++l) a[c][l] = b[c][l] = 0.0;
        const int m = pool_mn(c, 0), n = pool_mn(c, 1);
        const int K = m + n + 1;   // interfaces x_{j-m-1/2} .. x_{j+n+1/2} -> nodes 0..K
        const int s = m + 1;       // x_{j+1/2}
        Rat d[kMaxW + 2];
        for (int q = 0; q <= K; ++q) d[q] = basis_derivative(q, s, K);
        for (int i = 0; i < K; ++i) {
            Rat acc = make(0, 1);
            for (int q = i + 1; q <= K; ++q) acc = add(acc, d[q]);
            a[c][i] = to_double(acc);
            const int deg = m + n;
            i128 bv = binom(deg, i);
            if ((deg - i) % 2) bv = -bv;
            b[c][i] = (double)(long long)bv;
        }
    }
    return true;
}

}  // namespace enomr
