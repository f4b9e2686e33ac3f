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
// and k_adj_stage applies the transpose of its Jacobian to an adjoint vector.
//
// One workgroup owns a run of cells and works in LDS, without atomics (the
// result is deterministic):
//   1. stage, for every position its faces read, the split fluxes and the
//      cell quantities of the Roe average;
//   2. per (face, field): Gamma_k = sum over both chosen stencils of a_l G;
//   3. per face, backwards: phi = dJ/dF-hat, lambda_w-hat = R^T phi, the
//      vectors v_k = lambda_w-hat_k L_k that every cell of field k's stencils
//      receives (times its coefficient), and the Roe-average path into the
//      face's two cells (through the eigenvector entries' derivatives in u, H);
//   4. per (position, sign): gather the split-flux adjoints from every face
//      whose stencil holds the position;
//   5. per cell: sum the position images of the cell (ghost positions of an
//      outflow end), apply dG+-/dU = (dF/dU +- alpha I)/2 and the SSP-RK3
//      stage combination.
// The faces a workgroup needs reach R-1 positions past its cells (2R-1 at an
// outflow end, whose ghost positions it also owns); it computes them itself.
// With periodic ends faces are taken modulo n (face n is face 0: both see
// the same cells, hence the same stencils), so no position has an image.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace enomr {

// One stage of the reverse sweep.  The stage combined its input U_s and the
// step-start state U^n as  out = a U^n + b (U_s + dt L(U_s))  (stage 1: a = 0,
// b = 1, U_s = U^n).  Given lamIn = adjoint of `out`:
//   adjoint of L:   lamL = b dt lamIn
//   lamOut = cb lamIn + (dL/dU_s)^T lamL [+ addv]
//   lamAcc = a lamIn [+ lamAcc if accumulate]                       (adjoint of U^n so far)
// With b = 1, dt = NULL (read as 1), cb = 0 and no addv/lamAcc, lamOut is
// (dL/dU)^T lamIn: the operator adjoint alone.  lamOut and lamAcc must not
// alias lamIn or addv (other workgroups read lamIn at their neighbours).
struct AdjIn {
    const double* U;        // [3][n], the state the frozen operator was evaluated at
    const uint8_t* idx;     // [n+1][3][2] stencil choices
    const double* alpha;    // device scalar: the line's alpha
    const double* lamIn;    // [3][n]
    const double* dt;       // device scalar, or NULL for 1
    double a, b;            // stage coefficients
    double cb;              // weight of lamIn in lamOut
    const double* addv;     // nullable, added to lamOut
    double* lamAcc;         // nullable
    int accumulate;         // lamAcc += (1) or = (0)
    double* lamOut;         // [3][n]
    unsigned* status;
    long n;
    double ih, gamma;
    int bc;
};

// Pool index of a logged stencil choice; a byte outside the order's list is
// reported through the status word and read as the last candidate.
template <int R>
__device__ __forceinline__ int logged_cand(uint8_t b, unsigned* status)
{
    int C = b;
    if (C >= n_cands(R)) {
        flag_nonphysical(status);
        C = n_cands(R) - 1;
    }
    return C;
}

// LDS of one workgroup: T cells, order 2R-1.
template <int R, int T>
struct AdjLds {
    static constexpr int W = 2 * R - 1;            // window of stencil offsets l = -(R-1)..R-1
    static constexpr int NG = T + 2 * R;           // positions gathered (cells + outflow ghosts)
    static constexpr int NF = NG + 2 * R - 1;      // faces
    static constexpr int NP = NF + 2 * R - 1;      // staged positions
    double w[n_cands(R)][W];                       // a_l by candidate, zero outside [-m, n]
    double gp[3][NP], gm[3][NP];                   // split fluxes
    double s[NP], u[NP], H[NP], rho[NP], E[NP];    // Roe-average inputs
    uint8_t cand[2][3][NF];                        // chosen candidate per sign, field, face
    double gam[3][3][NF];                          // Gamma_k
    double v[3][3][NF];                            // v_k
    double roe[6][NF];                             // Roe-path adjoints: left cell (3), right cell (3)
    double lg[2][3][NG];                           // gathered split-flux adjoints per sign
    double lr[3][NG];                              // gathered Roe-path adjoints
};

template <int R, int T, int NT>
__global__ __launch_bounds__(NT) void k_adj_stage(AdjIn a)
{
    using Lds = AdjLds<R, T>;
    constexpr int W = Lds::W, NC = n_cands(R);
    __shared__ Lds sm;
    const long n = a.n;
    const bool periodic = a.bc == BC_PERIODIC;
    const long c0 = (long)blockIdx.x * T;
    const long c1 = c0 + T < n ? c0 + T : n;
    // gathered positions [pa, pb); faces [fa, fa + nf); staged positions from fa - R
    const long pa = (!periodic && c0 == 0) ? -R : c0;
    const long pb = (!periodic && c1 == n) ? n + R : c1;
    const long fa = pa - R + 1;
    const int ng = (int)(pb - pa), nf = ng + 2 * R - 1, np = nf + 2 * R - 1;
    const long p0 = fa - R;
    const double gamma = a.gamma, gm1 = gamma - 1.0;
    const double al = *a.alpha;
    const int tid = threadIdx.x;

    // 0. window-aligned coefficients of this order's candidates
    for (int e = tid; e < NC * W; e += NT) {
        const int C = e / W, k = e - C * W;
        const int P = c_candpool[R][C];
        const int m = pool_mn(P, 0), nn = pool_mn(P, 1);
        const int l = k - (R - 1);
        sm.w[C][k] = (l >= -m && l <= nn) ? c_a[P][l + m] : 0.0;
    }
    // 1. staged positions
    for (int e = tid; e < np; e += NT) {
        const long j = map_cell(p0 + e, n, a.bc);
        const double rho = a.U[j], m = a.U[n + j], E = a.U[2 * n + j];
        const double ir = 1.0 / rho;
        const double u = m * ir;
        const double p = gm1 * (E - 0.5 * (m * u));
        const double F[3] = {m, m * u + p, (E + p) * u};
        const double Uc[3] = {rho, m, E};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            sm.gp[q][e] = 0.5 * (F[q] + al * Uc[q]);
            sm.gm[q][e] = 0.5 * (F[q] - al * Uc[q]);
        }
        sm.s[e] = sqrt(rho);
        sm.u[e] = u;
        sm.H[e] = (E + p) * ir;
        sm.rho[e] = rho;
        sm.E[e] = E;
    }
    __syncthreads();

    // 2. Gamma_k per (face, field)
    for (int e = tid; e < 3 * nf; e += NT) {
        const int q = e / nf, fi = e - q * nf;
        const long f = fa + fi;
        double g[3] = {0.0, 0.0, 0.0};
        int Cp = 0, Cm = 0;
        if (periodic || (f >= 0 && f <= n)) {
            const long fl = periodic ? map_cell(f, n, a.bc) : f;   // logged face
            Cp = logged_cand<R>(a.idx[(fl * 3 + q) * 2], a.status);
            Cm = logged_cand<R>(a.idx[(fl * 3 + q) * 2 + 1], a.status);
            // f^+: centre f-1, offset l -> position f-1+l = f-R+k; f^-: centre f, position f-l = f+R-1-k
            const int bp = (int)(f - R - p0), bm = (int)(f + R - 1 - p0);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const double wp = sm.w[Cp][k], wm = sm.w[Cm][k];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    g[t] = fma(wp, sm.gp[t][bp + k], g[t]);
                    g[t] = fma(wm, sm.gm[t][bm - k], g[t]);
                }
            }
        }
        sm.cand[0][q][fi] = (uint8_t)Cp;
        sm.cand[1][q][fi] = (uint8_t)Cm;
#pragma unroll
        for (int t = 0; t < 3; ++t) sm.gam[q][t][fi] = g[t];
    }
    __syncthreads();

    // 3. faces backwards
    const double lscale = a.b * (a.dt ? *a.dt : 1.0) * a.ih;
    for (int fi = tid; fi < nf; fi += NT) {
        const long f = fa + fi;
        if (!periodic && (f < 0 || f > n)) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int t = 0; t < 3; ++t) sm.v[q][t][fi] = 0.0;
#pragma unroll
            for (int t = 0; t < 6; ++t) sm.roe[t][fi] = 0.0;
            continue;
        }
        const int iL = (int)(f - 1 - p0), iR = (int)(f - p0);
        const double sL = sm.s[iL], sR = sm.s[iR];
        const double id = 1.0 / (sL + sR);
        const double u = (sL * sm.u[iL] + sR * sm.u[iR]) * id;
        const double H = (sL * sm.H[iL] + sR * sm.H[iR]) * id;
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
        {
            const bool hasR = periodic || f < n, hasL = periodic || f > 0;
            const long jr = map_cell(f, n, a.bc), jl = map_cell(f - 1, n, a.bc);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double right = hasR ? a.lamIn[q * n + jr] : 0.0;
                const double left = hasL ? a.lamIn[q * n + jl] : 0.0;
                phi[q] = lscale * (right - left);
            }
        }
        double Gam[3][3], what[3], lw[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
#pragma unroll
            for (int t = 0; t < 3; ++t) Gam[q][t] = sm.gam[q][t][fi];
            what[q] = Lm[q][0] * Gam[q][0] + Lm[q][1] * Gam[q][1] + Lm[q][2] * Gam[q][2];
            lw[q] = Rm[0][q] * phi[0] + Rm[1][q] * phi[1] + Rm[2][q] * phi[2];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int t = 0; t < 3; ++t) sm.v[q][t][fi] = lw[q] * Lm[q][t];

        // adjoints of the eigenvector entries, then of the Roe state (u, H):
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
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int ic_ = side ? iR : iL;
            const double cs = sm.s[ic_], cuu = sm.u[ic_], cHH = sm.H[ic_], crho = sm.rho[ic_], cE = sm.E[ic_];
            const double lus = lu * cs * id;                          // d/du_cell
            const double lHs = lH * cs * id;                          // d/dH_cell
            const double lss = (lu * (cuu - u) + lH * (cHH - H)) * id; // d/ds_cell
            const double ir = 1.0 / crho;
            sm.roe[3 * side + 0][fi] =
                lss * 0.5 / cs - lus * cuu * ir + lHs * (-gamma * cE * ir * ir + gm1 * cuu * cuu * ir);
            sm.roe[3 * side + 1][fi] = lus * ir - lHs * gm1 * cuu * ir;
            sm.roe[3 * side + 2][fi] = lHs * gamma * ir;
        }
    }
    __syncthreads();

    // 4. gather per (position, sign)
    for (int e = tid; e < 2 * ng; e += NT) {
        const int sg = e / ng, gi = e - sg * ng;
        // face index of offset k: sign +: f = p + R - k; sign -: f = p + k - (R - 1)
        const int f0 = gi + (sg ? 0 : 2 * R - 1);   // (p + R) - fa, resp. (p - R + 1) - fa
        const int fs = sg ? 1 : -1;
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int fi = f0 + fs * k;
                const double w = sm.w[sm.cand[sg][q][fi]][k];
#pragma unroll
                for (int t = 0; t < 3; ++t) acc[t] = fma(w, sm.v[q][t][fi], acc[t]);
            }
#pragma unroll
        for (int t = 0; t < 3; ++t) sm.lg[sg][t][gi] = acc[t];
        if (sg == 0) {
            // face p+1 has p as its left cell, face p as its right cell
            const int fl = gi + R, fr = gi + R - 1;
#pragma unroll
            for (int t = 0; t < 3; ++t) sm.lr[t][gi] = sm.roe[t][fl] + sm.roe[3 + t][fr];
        }
    }
    __syncthreads();

    // 5. cells
    for (long j = c0 + tid; j < c1; j += NT) {
        // images of cell j among the gathered positions
        long qa = j, qb = j;
        if (!periodic && j == 0) qa = -R;
        if (!periodic && j == n - 1) qb = n - 1 + R;
        double lgp[3] = {0, 0, 0}, lgm[3] = {0, 0, 0}, lro[3] = {0, 0, 0};
        for (long pp = qa; pp <= qb; ++pp) {
            const int gi = (int)(pp - pa);
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                lgp[t] += sm.lg[0][t][gi];
                lgm[t] += sm.lg[1][t][gi];
                lro[t] += sm.lr[t][gi];
            }
        }
        const int ii = (int)(j - p0);
        const double u = sm.u[ii], H = sm.H[ii];
        const double s0 = lgp[0] + lgm[0], s1 = lgp[1] + lgm[1], s2 = lgp[2] + lgm[2];
        const double jt0 = 0.5 * (gamma - 3.0) * u * u * s1 + u * (0.5 * gm1 * u * u - H) * s2;
        const double jt1 = s0 + (3.0 - gamma) * u * s1 + (H - gm1 * u * u) * s2;
        const double jt2 = gm1 * s1 + gamma * u * s2;
        const double mu[3] = {0.5 * jt0 + 0.5 * al * (lgp[0] - lgm[0]) + lro[0],
                              0.5 * jt1 + 0.5 * al * (lgp[1] - lgm[1]) + lro[1],
                              0.5 * jt2 + 0.5 * al * (lgp[2] - lgm[2]) + lro[2]};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const long i = q * n + j;
            const double lin = a.lamIn[i];
            double o = a.cb * lin + mu[q];
            if (a.addv) o += a.addv[i];
            if (a.lamAcc) a.lamAcc[i] = a.accumulate ? a.lamAcc[i] + a.a * lin : a.a * lin;
            a.lamOut[i] = o;
        }
    }
}

__global__ void k_copy1(double* dst, const double* src)
{
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace enomr
