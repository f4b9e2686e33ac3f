// Frozen-stencil discrete adjoint of the 1D Euler ENO-MR operator.
//
// With the stencil choices (per face, field and sign), the line's alpha and
// the step size fixed from a forward pass, the operator is the smooth map
//   G+-_i = (F(U_i) +- alpha U_i)/2                    (Sec. 2.1, Eq. LF_Flux_Split)
//   w-hat+-_k = sum_l a_l (L_k . G+-_l)               (the chosen stencil; minmod
//                                                      branches are the stencils
//                                                      S_j^{j+1}, S_{j-1}^j, S_j^j)
//   F-hat = R (w-hat+ + w-hat-)                       (Roe-averaged L, R at the face)
//   L_j = -(F-hat_{j+1/2} - F-hat_{j-1/2}) / h        (Eq. 1DWENOFD)
// and these kernels apply the transpose of its Jacobian to an adjoint vector.
//
// Phase 1 (one thread per face) runs the face backwards: phi = dJ/dF-hat,
// lambda_w-hat = R^T phi, the vectors v_k = lambda_w-hat_k L_k that every
// cell of field k's stencils receives (times its stencil coefficient), and
// the Roe-average path into the face's two cells.  Phase 2 (one thread per
// cell) gathers, over every face whose stencils touch the cell (ghost images
// included), the split-flux adjoints and turns them into lambda_U through
// dG+-/dU = (dF/dU +- alpha I)/2.  No atomics: the result is deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace enomr {

constexpr int kFaceAdj = 15;   // per face: v_k (3 x 3), left-cell and right-cell Roe adjoints (3 + 3)

struct AdjIn {
    const double* U;        // [3][n], the state the frozen operator was evaluated at
    const uint8_t* idx;     // [n+1][3][2] stencil choices
    const double* alpha;    // device scalar: the line's alpha
    const double* lamL;     // [3][n] adjoint of L(U)
    double* face;           // [n+1][kFaceAdj] workspace
    double* lamU;           // [3][n] result
    unsigned* status;
    long n;
    double ih, gamma;
    int bc;
};

// Pool index of a logged stencil choice; a byte outside the order's list is
// reported through the status word and read as the last candidate.
template <int R>
__device__ __forceinline__ int logged_pool(uint8_t b, unsigned* status)
{
    int C = b;
    if (C >= n_cands(R)) {
        flag_nonphysical(status);
        C = n_cands(R) - 1;
    }
    return c_candpool[R][C];
}

struct CellPrim {
    double rho, u, E, p, H, s;
};

__device__ __forceinline__ CellPrim cell_prim1d(const double* U, long n, long j, double gm1)
{
    CellPrim c;
    c.rho = U[j];
    const double m = U[n + j];
    c.E = U[2 * n + j];
    const double ir = 1.0 / c.rho;
    c.u = m * ir;
    c.p = gm1 * (c.E - 0.5 * (m * c.u));
    c.H = (c.E + c.p) * ir;
    c.s = sqrt(c.rho);
    return c;
}

// Split flux G+- of cell j (normal frame, 1D).
__device__ __forceinline__ void split_flux1d(const double* U, long n, long j, double gm1, double al, double (&Gp)[3],
                                             double (&Gm)[3])
{
    const double rho = U[j], m = U[n + j], E = U[2 * n + j];
    const double u = m / rho;
    const double p = gm1 * (E - 0.5 * (m * u));
    const double F[3] = {m, m * u + p, (E + p) * u};
    const double Uc[3] = {rho, m, E};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        Gp[q] = 0.5 * (F[q] + al * Uc[q]);
        Gm[q] = 0.5 * (F[q] - al * Uc[q]);
    }
}

template <int R>
__global__ __launch_bounds__(128) void k_adj_faces(AdjIn a)
{
    const long f = blockIdx.x * 128L + threadIdx.x;
    const long n = a.n;
    if (f > n) return;
    const double gamma = a.gamma, gm1 = gamma - 1.0;
    const double al = *a.alpha;
    const long jl = map_cell(f - 1, n, a.bc), jr = map_cell(f, n, a.bc);
    const CellPrim cL = cell_prim1d(a.U, n, jl, gm1), cR = cell_prim1d(a.U, n, jr, gm1);

    // Roe state and eigenvectors (fields u-c, u, u+c)
    const double id = 1.0 / (cL.s + cR.s);
    const double u = (cL.s * cL.u + cR.s * cR.u) * id;
    const double H = (cL.s * cL.H + cR.s * cR.H) * id;
    const double q2 = u * u;
    const double c2 = gm1 * (H - 0.5 * q2);
    const double c = sqrt(c2);
    const double k = gm1 / c2;
    const double ic = 1.0 / c;
    const double hq = 0.5 * k * q2, ku = k * u, uic = u * ic, uc = u * c;
    const double Lm[3][3] = {{0.5 * (hq + uic), -0.5 * (ku + ic), 0.5 * k},
                             {1.0 - hq, ku, -k},
                             {0.5 * (hq - uic), -0.5 * (ku - ic), 0.5 * k}};
    const double Rm[3][3] = {{1.0, 1.0, 1.0}, {u - c, u, u + c}, {H - uc, 0.5 * q2, H + uc}};

    // phi = dJ/dF-hat: face f is the left face of cell f and the right face of cell f-1
    double phi[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double right = f < n ? a.lamL[q * n + f] : 0.0;
        const double left = f > 0 ? a.lamL[q * n + f - 1] : 0.0;
        phi[q] = a.ih * (right - left);
    }

    // Gamma_k = sum over the chosen stencils of a_l G (conserved space), both signs
    double Gam[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int kp = a.idx[(f * 3 + q) * 2], km = a.idx[(f * 3 + q) * 2 + 1];
        const int Pp = logged_pool<R>((uint8_t)kp, a.status), Pm = logged_pool<R>((uint8_t)km, a.status);
        const int mp = pool_mn(Pp, 0), np_ = pool_mn(Pp, 1);
        const int mm = pool_mn(Pm, 0), nm = pool_mn(Pm, 1);
        double g[3] = {0.0, 0.0, 0.0};
        for (int l = -mp; l <= np_; ++l) {   // f^+: centre cell f-1, offset l -> cell f-1+l
            double Gp[3], Gm[3];
            split_flux1d(a.U, n, map_cell(f - 1 + l, n, a.bc), gm1, al, Gp, Gm);
            const double w = c_a[Pp][l + mp];
#pragma unroll
            for (int t = 0; t < 3; ++t) g[t] = fma(w, Gp[t], g[t]);
        }
        for (int l = -mm; l <= nm; ++l) {    // f^-: centre cell f, offset l -> cell f-l
            double Gp[3], Gm[3];
            split_flux1d(a.U, n, map_cell(f - l, n, a.bc), gm1, al, Gp, Gm);
            const double w = c_a[Pm][l + mm];
#pragma unroll
            for (int t = 0; t < 3; ++t) g[t] = fma(w, Gm[t], g[t]);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) Gam[q][t] = g[t];
    }
    double what[3], lw[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        what[q] = Lm[q][0] * Gam[q][0] + Lm[q][1] * Gam[q][1] + Lm[q][2] * Gam[q][2];
        lw[q] = Rm[0][q] * phi[0] + Rm[1][q] * phi[1] + Rm[2][q] * phi[2];
    }
    double* out = a.face + f * kFaceAdj;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int t = 0; t < 3; ++t) out[3 * q + t] = lw[q] * Lm[q][t];

    // adjoints of the eigenvector entries, then of the Roe state (u, H)
    // dL[i][j], dR[i][j] with respect to u and H
    const double c2u = -gm1 * u, c2H = gm1;
    const double cu = c2u / (2.0 * c), cH = c2H / (2.0 * c);
    const double ku_ = -k * c2u / c2, kH = -k * c2H / c2;
    const double icu = -ic * ic * cu, icH = -ic * ic * cH;
    const double hqu = 0.5 * ku_ * q2 + k * u, hqH = 0.5 * kH * q2;
    const double kuu = ku_ * u + k, kuH = kH * u;
    const double uicu = ic + u * icu, uicH = u * icH;
    const double ucu = c + u * cu, ucH = u * cH;
    const double dLu[3][3] = {{0.5 * (hqu + uicu), -0.5 * (kuu + icu), 0.5 * ku_},
                              {-hqu, kuu, -ku_},
                              {0.5 * (hqu - uicu), -0.5 * (kuu - icu), 0.5 * ku_}};
    const double dLH[3][3] = {{0.5 * (hqH + uicH), -0.5 * (kuH + icH), 0.5 * kH},
                              {-hqH, kuH, -kH},
                              {0.5 * (hqH - uicH), -0.5 * (kuH - icH), 0.5 * kH}};
    const double dRu[3][3] = {{0, 0, 0}, {1.0 - cu, 1.0, 1.0 + cu}, {-ucu, u, ucu}};
    const double dRH[3][3] = {{0, 0, 0}, {-cH, 0.0, cH}, {1.0 - ucH, 0.0, 1.0 + ucH}};
    double lu = 0.0, lH = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double lL = lw[q] * Gam[q][t];   // adjoint of Lm[q][t]
            const double lR = phi[q] * what[t];    // adjoint of Rm[q][t]
            lu += lL * dLu[q][t] + lR * dRu[q][t];
            lH += lL * dLH[q][t] + lR * dRH[q][t];
        }
    // Roe averages -> cell quantities (s, u, H) -> (rho, m, E)
    const CellPrim* cs[2] = {&cL, &cR};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const CellPrim& cc = *cs[side];
        const double lus = lu * cc.s * id;                           // d/du_cell
        const double lHs = lH * cc.s * id;                           // d/dH_cell
        const double lss = (lu * (cc.u - u) + lH * (cc.H - H)) * id; // d/ds_cell
        const double ir = 1.0 / cc.rho;
        double lrho = lss * 0.5 / cc.s - lus * cc.u * ir + lHs * (-gamma * cc.E * ir * ir + gm1 * cc.u * cc.u * ir);
        double lm = lus * ir - lHs * gm1 * cc.u * ir;
        double lE = lHs * gamma * ir;
        out[9 + 3 * side + 0] = lrho;
        out[9 + 3 * side + 1] = lm;
        out[9 + 3 * side + 2] = lE;
    }
}

template <int R>
__global__ __launch_bounds__(128) void k_adj_cells(AdjIn a)
{
    const long j = blockIdx.x * 128L + threadIdx.x;
    const long n = a.n;
    if (j >= n) return;
    const double gamma = a.gamma, gm1 = gamma - 1.0;
    const double al = *a.alpha;
    double lgp[3] = {0, 0, 0}, lgm[3] = {0, 0, 0}, lroe[3] = {0, 0, 0};
    // unmapped positions that read cell j
    long img[R + 3];
    int nimg = 0;
    img[nimg++] = j;
    if (a.bc == BC_PERIODIC) {
        if (j - n >= -(R + 1)) img[nimg++] = j - n;
        if (j + n <= n + R) img[nimg++] = j + n;
    } else {
        if (j == 0)
            for (int t = 1; t <= R + 1; ++t) img[nimg++] = -t;
        if (j == n - 1)
            for (int t = 1; t <= R + 1 && nimg < R + 3; ++t) img[nimg++] = n - 1 + t;
    }
    for (int s = 0; s < nimg; ++s) {
        const long p = img[s];
        // f^+ stencils: centre f-1, position p = f-1+l
        for (long f = p - R + 2; f <= p + R; ++f) {
            if (f < 0 || f > n) continue;
            const long l = p - (f - 1);
            for (int q = 0; q < 3; ++q) {
                const int P = logged_pool<R>(a.idx[(f * 3 + q) * 2], a.status);
                const int m = pool_mn(P, 0), nn = pool_mn(P, 1);
                if (l < -m || l > nn) continue;
                const double w = c_a[P][l + m];
                const double* v = a.face + f * kFaceAdj + 3 * q;
                for (int t = 0; t < 3; ++t) lgp[t] = fma(w, v[t], lgp[t]);
            }
        }
        // f^- stencils: centre f, position p = f-l
        for (long f = p - R + 1; f <= p + R - 1; ++f) {
            if (f < 0 || f > n) continue;
            const long l = f - p;
            for (int q = 0; q < 3; ++q) {
                const int P = logged_pool<R>(a.idx[(f * 3 + q) * 2 + 1], a.status);
                const int m = pool_mn(P, 0), nn = pool_mn(P, 1);
                if (l < -m || l > nn) continue;
                const double w = c_a[P][l + m];
                const double* v = a.face + f * kFaceAdj + 3 * q;
                for (int t = 0; t < 3; ++t) lgm[t] = fma(w, v[t], lgm[t]);
            }
        }
        // Roe averages: face p+1 has p as its left cell, face p as its right cell
        if (p + 1 >= 0 && p + 1 <= n)
            for (int t = 0; t < 3; ++t) lroe[t] += a.face[(p + 1) * kFaceAdj + 9 + t];
        if (p >= 0 && p <= n)
            for (int t = 0; t < 3; ++t) lroe[t] += a.face[p * kFaceAdj + 12 + t];
    }
    // dG+-/dU = (dF/dU +- alpha I) / 2
    const double rho = a.U[j], m = a.U[n + j], E = a.U[2 * n + j];
    const double u = m / rho;
    const double p = gm1 * (E - 0.5 * (m * u));
    const double H = (E + p) / rho;
    const double s0 = lgp[0] + lgm[0], s1 = lgp[1] + lgm[1], s2 = lgp[2] + lgm[2];
    const double jt0 = 0.5 * (gamma - 3.0) * u * u * s1 + u * (0.5 * gm1 * u * u - H) * s2;
    const double jt1 = s0 + (3.0 - gamma) * u * s1 + (H - gm1 * u * u) * s2;
    const double jt2 = gm1 * s1 + gamma * u * s2;
    a.lamU[j] = 0.5 * jt0 + 0.5 * al * (lgp[0] - lgm[0]) + lroe[0];
    a.lamU[n + j] = 0.5 * jt1 + 0.5 * al * (lgp[1] - lgm[1]) + lroe[1];
    a.lamU[2 * n + j] = 0.5 * jt2 + 0.5 * al * (lgp[2] - lgm[2]) + lroe[2];
}

// out = a x + b y (elementwise); y may be NULL (then out = a x)
__global__ void k_axpby(double* out, double a, const double* x, double b, const double* y, long n)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

// out = a x + dt_scale * (*dt) * y
__global__ void k_axpdty(double* out, double a, const double* x, double dscale, const double* dt, const double* y,
                         long n)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) out[i] = a * x[i] + (dscale * *dt) * y[i];
}

__global__ void k_copy1(double* dst, const double* src)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace enomr
