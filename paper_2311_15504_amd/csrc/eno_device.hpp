// Device-side ENO-MR stencil selection (arXiv 2311.15504, Sec. 3.2).
//
// A reconstruction window w[0 .. 2R-2] holds 2R-1 values in ascending cell
// order with the centre cell at w[R-1].  For sign S = +1 the centre is the
// left cell j of face j+1/2 and stencil offset l is w[R-1+l]; for S = -1
// (f^-, the mirror image about x_{j+1/2}) the centre is j+1 and offset l is
// w[R-1-l].  Every dot product runs over ascending cells: a plain product for
// the first term, then fma.  The host compiles this with -ffp-contract=off, so
// no other operation is fused; the CPU oracle evaluates the same expressions
// in the same order, which makes the stencil choices bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include "tables.hpp"

namespace enomr {

// a_l of every pool stencil, entry l+m, for runtime-indexed use (filled at
// context creation; compile-time positions read kCoef instead).
extern __constant__ double c_a[kPool][kMaxW];

// The a_l aligned to a 17-entry window centred at entry 8 and zero outside
// the stencil: c_wa[s][P][i] multiplies window entry i for sign s (0: +,
// 1: -).  A (2R-1)-entry window starts at entry 9-R.  A zero coefficient adds
// an exact zero to an fma chain, so a padded chain rounds like the stencil's
// own chain (up to the sign of a zero result).
extern __constant__ double c_wa[2][kPool][kMaxW];
// Pool index of candidate c of the (2R-1)-point scheme: c_candpool[R][c].
extern __constant__ int c_candpool[10][kPool];

// Coefficient index of window entry i for stencil (m, n) and sign S.
template <int R, int S, int m>
__device__ constexpr int coef_index(int i)
{
    return S > 0 ? i - (R - 1) + m : (R - 1 - i) + m;
}

// sum_l coef[l+m] w(l) over stencil pool entry P, ascending cells.
template <int R, int S, int P>
__device__ __forceinline__ double sdot(const double* coef, const double (&w)[2 * R - 1])
{
    constexpr int m = pool_mn(P, 0), n = pool_mn(P, 1);
    constexpr int lo = S > 0 ? R - 1 - m : R - 1 - n;
    constexpr int hi = S > 0 ? R - 1 + n : R - 1 + m;
    double acc = coef[coef_index<R, S, m>(lo)] * w[lo];
#pragma unroll
    for (int i = lo + 1; i <= hi; ++i) acc = fma(coef[coef_index<R, S, m>(i)], w[i], acc);
    return acc;
}

// Step 1: IS0 = min(IS_L, IS_R), Eq. (Baseline_IS).  The second differences
// are (f0 - 2 f1) + f2; 2 f1 is exact, so fma(-2, f1, f0) rounds f0 - 2 f1
// exactly as the subtraction does.
template <int R, int S>
__device__ __forceinline__ double baseline_is(const double (&w)[2 * R - 1])
{
    const double f0 = w[R - 1];
    const double fm1 = S > 0 ? w[R - 2] : w[R];
    const double fm2 = S > 0 ? w[R - 3] : w[R + 1];
    const double fp1 = S > 0 ? w[R] : w[R - 2];
    const double fp2 = S > 0 ? w[R + 1] : w[R - 3];
    const double isl = fmax(fabs(f0 - fm1), fabs(fma(-2.0, fm1, f0) + fm2));
    const double isr = fmax(fabs(f0 - fp1), fabs(fma(-2.0, fp1, f0) + fp2));
    return fmin(isl, isr);
}

// Step 3.2: f_c + minmod(f_{c+1} - f_c, f_c - f_{c-1}) / 2 in the sign's frame,
// from the centre value f0, its downwind neighbour fp1 and upwind fm1.
template <int R>
__device__ __forceinline__ double minmod3(double f0, double fp1, double fm1, int& idx)
{
    constexpr int NC = n_cands(R);
    const double da = fp1 - f0;
    const double db = f0 - fm1;
    double mm;
    if (da * db > 0.0) {
        if (fabs(da) <= fabs(db)) { mm = da; idx = NC - 3; }   // S_j^{j+1}
        else { mm = db; idx = NC - 2; }                          // S_{j-1}^{j}
    } else {
        mm = 0.0; idx = NC - 1;                                   // S_j^{j}
    }
    return f0 + 0.5 * mm;
}

template <int R, int S>
__device__ __forceinline__ double minmod_flux(const double (&w)[2 * R - 1], int& idx)
{
    return minmod3<R>(w[R - 1], S > 0 ? w[R] : w[R - 2], S > 0 ? w[R - 2] : w[R], idx);
}

// Step 3.1 beyond the full stencil.  The indicator of candidate (m, n) is the
// (m+n)-th undivided difference of its cells (Eq. CurrentIS: h^{m+n} times the
// (m+n)-th derivative of the stencil polynomial; Table ISCoe holds its binomial
// expansion), taken by repeated differencing of the window in ascending cell
// order.  One difference table of the window, built level by level in place,
// yields every candidate's indicator.  Levels are built upwards while list
// order runs downwards in level, so a passing candidate overwrites the choice
// made at lower levels, and within a level the candidates are visited in
// reverse list order: the last write is the first passing candidate in list
// order.  In the sign's frame stencil (m, n) starts at window entry R-1-m
// (f^+) or R-1-n (f^-, the mirror image).
template <int R, int S, int LEV, int C>
__device__ __forceinline__ void mark_level(const double (&d)[2 * R - 1], double is0, int& chosen)
{
    if constexpr (C >= 1) {
        constexpr int P = cand_pool(R, C);
        constexpr int m = pool_mn(P, 0), n = pool_mn(P, 1);
        if constexpr (m >= 1 && n >= 1 && m + n == LEV) {
            constexpr int s = S > 0 ? R - 1 - m : R - 1 - n;
            chosen = fabs(d[s]) < is0 ? C : chosen;
        }
        mark_level<R, S, LEV, C - 1>(d, is0, chosen);
    }
}

template <int R, int S, int LEV>
__device__ __forceinline__ void difference_levels(double (&d)[2 * R - 1], double is0, int& chosen)
{
    // the full stencil's level 2R-2 is not needed: candidate 0 is tested by its b_l chain
    if constexpr (LEV <= 2 * R - 3) {
#pragma unroll
        for (int i = 0; i + LEV < 2 * R - 1; ++i) d[i] = d[i + 1] - d[i];
        mark_level<R, S, LEV, n_cands(R) - 1>(d, is0, chosen);
        difference_levels<R, S, LEV + 1>(d, is0, chosen);
    }
}

// Step 3.1 from candidate 1 on: the first candidate whose indicator is below
// is0, or -1.  The window d is overwritten by its difference table.
template <int R, int S>
__device__ __forceinline__ int first_passing(double (&d)[2 * R - 1], double is0)
{
    int chosen = -1;
    difference_levels<R, S, 1>(d, is0, chosen);
    return chosen;
}

// The flux of candidate c over the window: padded window-aligned a_l row.
template <int R, int S>
__device__ __forceinline__ double candidate_flux(const double (&w)[2 * R - 1], int c)
{
    const double* wa = &c_wa[S > 0 ? 0 : 1][c_candpool[R][c]][9 - R];
    double f = wa[0] * w[0];
#pragma unroll
    for (int i = 1; i < 2 * R - 1; ++i) f = fma(wa[i], w[i], f);
    return f;
}

// Steps 3.1/3.2 from candidate 1 on, for a window whose full stencil failed.
template <int R, int S>
__device__ __forceinline__ double select_rest(const double (&w)[2 * R - 1], double is0, int& idx)
{
    double d[2 * R - 1];
#pragma unroll
    for (int i = 0; i < 2 * R - 1; ++i) d[i] = w[i];
    const int c = first_passing<R, S>(d, is0);
    if (c >= 0) {
        idx = c;
        return candidate_flux<R, S>(w, c);
    }
    return minmod_flux<R, S>(w, idx);
}

// The whole scalar reconstruction (Steps 1-3.2) of the window w[0 .. 2R-2]
// read where it lies (the LDS tile of a sweep), bitwise the same as recon():
// the full stencil's indicator and flux chains stream the window (the flux
// chain is kept only if the indicator passes), and only a window that fails
// is copied into registers for its difference table.  Holding no window in
// registers on the smooth path leaves room for more waves per SIMD.
template <int R, int S>
__device__ __forceinline__ double recon_streamed(const double* w, int& idx)
{
    constexpr int P0 = cand_pool(R, 0);
    constexpr int W = 2 * R - 1;
    const double f0 = w[R - 1];
    const double fm1 = S > 0 ? w[R - 2] : w[R];
    const double fm2 = S > 0 ? w[R - 3] : w[R + 1];
    const double fp1 = S > 0 ? w[R] : w[R - 2];
    const double fp2 = S > 0 ? w[R + 1] : w[R - 3];
    const double isl = fmax(fabs(f0 - fm1), fabs(fma(-2.0, fm1, f0) + fm2));
    const double isr = fmax(fabs(f0 - fp1), fabs(fma(-2.0, fp1, f0) + fp2));
    const double is0 = fmin(isl, isr);
    double is = kCoef.b[P0][coef_index<R, S, R - 1>(0)] * w[0];
    double fl = kCoef.a[P0][coef_index<R, S, R - 1>(0)] * w[0];
#pragma unroll
    for (int i = 1; i < W; ++i) {
        const double x = w[i];
        is = fma(kCoef.b[P0][coef_index<R, S, R - 1>(i)], x, is);
        fl = fma(kCoef.a[P0][coef_index<R, S, R - 1>(i)], x, fl);
    }
    if (fabs(is) < is0) {
        idx = 0;
        return fl;
    }
    double d[W];
#pragma unroll
    for (int i = 0; i < W; ++i) d[i] = w[i];
    const int c = first_passing<R, S>(d, is0);
    if (c >= 0) {
        idx = c;
        const double* wa = &c_wa[S > 0 ? 0 : 1][c_candpool[R][c]][9 - R];
        double f = wa[0] * w[0];
#pragma unroll
        for (int i = 1; i < W; ++i) f = fma(wa[i], w[i], f);
        return f;
    }
    return minmod3<R>(f0, fp1, fm1, idx);
}

// The whole scalar reconstruction (Steps 1-3.2) of one window.
template <int R, int S>
__device__ __forceinline__ double recon(const double (&w)[2 * R - 1], int& idx)
{
    constexpr int P0 = cand_pool(R, 0);
    const double is0 = baseline_is<R, S>(w);
    if (fabs(sdot<R, S, P0>(kCoef.b[P0], w)) < is0) {
        idx = 0;
        return sdot<R, S, P0>(kCoef.a[P0], w);
    }
    return select_rest<R, S>(w, is0, idx);
}

}  // namespace enomr
