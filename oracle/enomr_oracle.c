/*
 * CPU oracle for the ENO-MR finite-difference scheme (H. Shen, arXiv 2311.15504).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * table with the GPU library: the stencil coefficients arrive as arguments,
 * derived in exact rational arithmetic by oracle/coeffs.py.
 *
 * Every step follows the method in the order the paper states it, with each
 * formula written the plain way:
 *   - primitive variables by division (u = m / rho, H = (E + p) / rho,
 *     c = sqrt(gamma p / rho));
 *   - the Roe state with sqrt(rho) weights divided by their sum, and the
 *     closed-form left and right eigenvectors of the face-normal Jacobian;
 *   - every cell of a face's window projected onto every characteristic field
 *     (l_k . G, a dot product over the conserved components in ascending
 *     order), then the scalar reconstruction of Sec. 3.2 applied to each field
 *     and sign on the projected values;
 *   - every indicator IS = |sum_l b_l f_{j+l}| with the b_l of Tables ISCoe1/2
 *     (Eq. ISCoe), every flux sum_l a_l f_{j+l} with the a_l of Tables
 *     Flux_reconstruction1/2 (Eq. ReconstructedFlux), candidates tested in
 *     list order until one passes (Step 3.1);
 *   - dot products as fma() chains over ascending cells (or components);
 *   - IS0 second differences as (f_c - 2 f_{c-1}) + f_{c-2}.
 * Built with -ffp-contract=off, so apart from the written fma() calls every
 * operation rounds on its own.  The paper fixes no floating-point order, so an
 * implementation that evaluates in another order can decide a comparison
 * differently where it lies within rounding of a tie.  The near-tie record
 * (orc_ties) measures the margin mu of each such comparison and, if asked,
 * takes the other implementation's choice where |mu| is below a tolerance.
 *
 * Method steps and where the paper states them:
 *   global Lax-Friedrichs splitting ............. Sec. 2.1, Eq. (LF_Flux_Split)
 *   conservative semi-discrete operator ......... Sec. 2.1, Eq. (1DWENOFD)
 *   ENO-MR stencil selection .................... Sec. 3.2, Steps 1-3.2,
 *                                                 Eqs. (Baseline_IS), (CurrentIS), (ISCoe)
 *   candidate pool and a_l, b_l ................. Sec. 3.1, Eq. (Candidates), Tables
 *   SSP-RK3 ..................................... Sec. 2.3, Eq. (TVD3rdRK)
 *   linear SSP-RK(m, m-1) ....................... Sec. 2.3, Eqs. (lSSPRK), (lSSPRK_Coe)
 *   Euler equations, characteristic projection .. Sec. 4 preamble (Roe average at the
 *                                                 face), Sec. 4.3, Sec. 4.4
 *
 * Variants of the Euler operator (each off by default):
 *   component-wise reconstruction: the split fluxes G+- of each conserved
 *     component are reconstructed as they are, with no projection (the
 *     scalar procedure applied to a system component by component);
 *   per-field alpha: each characteristic field k splits with its own
 *     alpha_k = max over the line of |lambda_k| (lambda = u-c, u, [u,] u+c),
 *     a field-wise reading of the maximum of Eq. (LF_Flux_Split):
 *     w+-_k = (l_k.F +- t) / 2 with t = alpha_k (l_k.U);
 *   gravity: the source g [0, 0, rho, rho v] of the Rayleigh-Taylor problem
 *     (Sec. 4.4) added to the 2D right-hand side after the two sweeps.
 *
 * Compiled twice: in FP64 (everything), and with -DORC_QUAD in IEEE binary128
 * (the scalar path only, names suffixed _q), the precision in which the paper
 * ran its convergence tests (Sec. 4 preamble).  The 2D operator and 1D faces
 * run in parallel over independent lines (faces) with OpenMP; every value is
 * computed by the same operations whatever the thread count.
 */
/*
 * ORC_PLANT (test builds only, 0 otherwise): a numbered, deliberate mistake
 * compiled into a scratch copy of the oracle, so that a test can show that
 * the pins catch it.  The shipped library is built with none.
 */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_QUAD
#include <quadmath.h>
typedef __float128 real;
#define R_ABS(x) fabsq(x)
#define R_MAX(a, b) fmaxq(a, b)
#define R_MIN(a, b) fminq(a, b)
/* at 113 significant bits the fusion of a product into a sum is immaterial */
#define R_FMA(a, b, c) ((a) * (b) + (c))
#define ORC_FN(name) name##_q
/* faces per line from which a scalar line's faces run in parallel */
#define ORC_PAR_FACES 64
#else
typedef double real;
#define R_ABS(x) fabs(x)
#define R_MAX(a, b) fmax(a, b)
#define R_MIN(a, b) fmin(a, b)
#define R_FMA(a, b, c) fma(a, b, c)
#define ORC_FN(name) name
#define ORC_PAR_FACES 4096
#endif

/* ------------------------------------------------------------------------ */
/* Operation counter (FP64 build)                                            */
/* ------------------------------------------------------------------------ */

/*
 * Algorithmic operation count of the Euler operator and the SSP-RK3 stage
 * combination, taken as the method's steps run: add, sub, mul, div, sqrt,
 * fma, min, max and compare count 1 each; |x| and negation are free.  Only
 * the candidates the paper's early exit reaches are counted (Step 3.1 stops
 * at the first passing candidate), even where the oracle evaluates more of
 * them to measure margins.  A value computed once and used twice counts once.
 * Primitive variables and split fluxes count once per cell of a line (its
 * ghost copies are not counted).  Per-line alphas and dt are not counted.
 * Categories: x lines (1D lines), y lines, the 2D sum L_x + L_y, and the
 * SSP-RK3 stage combination.
 */
enum { ORC_OPS_X = 0, ORC_OPS_Y = 1, ORC_OPS_SUM = 2, ORC_OPS_RK = 3, ORC_OPS_NCAT = 4 };

#ifndef ORC_QUAD
static int g_count_on;
static double g_ops[ORC_OPS_NCAT];
static _Thread_local double t_ops[ORC_OPS_NCAT];
static _Thread_local int t_cat, t_count;

#define OPS(n) do { if (t_count && g_count_on) t_ops[t_cat] += (double)(n); } while (0)

static void ops_enter(int cat)
{
    t_count = g_count_on;
    t_cat = cat;
}

static void ops_off(void) { t_count = 0; }

static void ops_flush(void)
{
    /* integer-valued partial sums: exact in any merge order */
    for (int i = 0; i < ORC_OPS_NCAT; ++i) {
        if (t_ops[i] != 0.0) {
#pragma omp critical(orc_ops)
            g_ops[i] += t_ops[i];
            t_ops[i] = 0.0;
        }
    }
}

void orc_ops_begin(void)
{
    for (int i = 0; i < ORC_OPS_NCAT; ++i) g_ops[i] = 0.0;
    g_count_on = 1;
}

/* Stops counting; the total, and per category into cats[4] (nullable). */
double orc_ops_end(double *cats)
{
    g_count_on = 0;
    double s = 0.0;
    for (int i = 0; i < ORC_OPS_NCAT; ++i) {
        if (cats) cats[i] = g_ops[i];
        s += g_ops[i];
    }
    return s;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
#else
#define OPS(n) do { } while (0)
static void ops_enter(int cat) { (void)cat; }
static void ops_off(void) { }
static void ops_flush(void) { }
#endif

#define ORC_MAXC 29
#define ORC_MAXW 17

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENONPHYS = 5 };
enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1 };
enum { ORC_ADVECTION = 0, ORC_BURGERS = 1 };
enum { ORC_SPLIT_NONE = 0, ORC_SPLIT_LF = 1 };

typedef struct {
    int order;              /* 2r-1 */
    int r;
    int ncand;
    int m[ORC_MAXC], n[ORC_MAXC];
    real a[ORC_MAXC][ORC_MAXW];   /* a[c][l+m], l = -m..n */
    real b[ORC_MAXC][ORC_MAXW];   /* b[c][l+m] */
} orc_table;

/*
 * A candidate table: mn holds (m, n) per candidate in list order; the a_l
 * arrive as exact fractions anum/aden (each rounded here to the nearest value
 * of the real type by one division of exactly representable integers), the
 * b_l as integers.  Arrays hold ORC_MAXW entries per candidate, entry l+m.
 */
orc_table *ORC_FN(orc_table_new)(int order, int ncand, const int *mn, const int64_t *anum, const int64_t *aden,
                                 const int64_t *bint)
{
    if (ncand < 1 || ncand > ORC_MAXC || order < 5 || order > 17 || !(order & 1)) return NULL;
    orc_table *t = (orc_table *)calloc(1, sizeof(orc_table));
    if (!t) return NULL;
    t->order = order;
    t->r = (order + 1) / 2;
    t->ncand = ncand;
    for (int c = 0; c < ncand; ++c) {
        t->m[c] = mn[2 * c];
        t->n[c] = mn[2 * c + 1];
        for (int l = 0; l < ORC_MAXW; ++l) {
            const int64_t d = aden[c * ORC_MAXW + l];
            t->a[c][l] = d ? (real)anum[c * ORC_MAXW + l] / (real)d : (real)0;
            t->b[c][l] = (real)bint[c * ORC_MAXW + l];
        }
    }
    return t;
}

void ORC_FN(orc_table_free)(orc_table *t) { free(t); }

/* ------------------------------------------------------------------------ */
/* Near-tie record (FP64 build)                                              */
/* ------------------------------------------------------------------------ */

/*
 * follow: another implementation's stencil log for the same call (the layout
 * of the call's own log), or NULL.  Where the two choices differ, the margin
 * mu of the comparison that decided them (see tie_margin) is recorded: the
 * first `max` differences go to pos[] (position in the log) and mu[]; count
 * counts them all.  Where |mu| < tol the oracle takes the other choice for the
 * flux (its own log keeps its own choice).
 */
typedef struct {
    const uint8_t *follow;
    double tol;
    int64_t *pos;
    double *mu;
    int64_t max;
    int64_t count;
} orc_ties;

/* ------------------------------------------------------------------------ */
/* Scalar ENO-MR reconstruction at one face (Sec. 3.2)                       */
/* ------------------------------------------------------------------------ */

/*
 * Value at stencil offset l in the reconstruction frame.  For sign +1 the
 * frame is centred on cell c = j and offsets run with the cell index; for
 * sign -1 (the mirror image about x_{j+1/2}, Sec. 3.1) the centre is c = j+1
 * and offset l is cell c - l.
 */
#define FR(l) (f[c + (long)s * (l)])

/*
 * Dot product of a stencil's coefficients with the values of its cells,
 * summed in ascending physical cell order.  coef[l+m] belongs to offset l.
 */
static real stencil_dot(const real *coef, int m, int n, const real *f, long c, int s)
{
    /* cells covered: offsets -m..n; ascending cell order means offsets
       ascending for s = +1 and descending for s = -1. */
    int l = (s > 0) ? -m : n;
    const int dl = (s > 0) ? 1 : -1;
    real acc = coef[l + m] * FR(l);
    for (int k = 1; k < m + n + 1; ++k) {
        l += dl;
        acc = R_FMA(coef[l + m], FR(l), acc);
    }
    return acc;
}

/* The value candidate k gives at the face (a stencil's a_l sum, or one of the
   three minmod branches of Step 3.2, which are the last three candidates). */
__attribute__((unused)) static real candidate_value(const orc_table *T, const real *f, long c, int s, int k)
{
    const int nfull = T->ncand - 3;
    if (k < nfull) return stencil_dot(T->a[k], T->m[k], T->n[k], f, c, s);
    const real f0 = FR(0);
    if (T->m[k] == 0 && T->n[k] == 1) return f0 + (real)0.5 * (FR(1) - f0);   /* S_j^{j+1} */
    if (T->m[k] == 1 && T->n[k] == 0) return f0 + (real)0.5 * (f0 - FR(-1));  /* S_{j-1}^j */
    return f0 + (real)0.5 * (real)0;                                         /* S_j^j */
}

#ifndef ORC_QUAD
/*
 * Where the magnitude A_l that rounding acts on comes from (see tie_margin):
 * |f_l| for a scalar law (ms NULL); for a system, every conserved component
 * of a cell carries rounding errors at the size of the cell's largest split
 * flux (each is updated from fluxes that include the pressure, so even a
 * component that is zero in exact arithmetic, a symmetric shear, holds
 * rounding noise of that size), so A_l = (sum_i |row_i|) max_i |G_i| (row
 * NULL: the component itself, sum = 1), or with per-field alphas
 * (sum_i |row_i|) (max_i |F_i| + ak max_i |U_i|) / 2.
 */
typedef struct {
    const double *row;
    const double *G;      /* split fluxes [cell][nv] (or U with per-field alphas) */
    const double *F;      /* per-field alphas: fluxes, stride fstride per cell */
    long fstride;
    double ak;
    int nv;
} mag_src;

static double mag_at(const mag_src *ms, const double *f, long i)
{
    if (!ms) return fabs(f[i]);
    double rs = ms->row ? 0.0 : 1.0, gm = 0.0;
    for (int k = 0; k < ms->nv; ++k) {
        if (ms->row) rs += fabs(ms->row[k]);
        gm = fmax(gm, fabs(ms->G[i * ms->nv + k]));
    }
    if (ms->F) {
        double fm = 0.0;
        for (int k = 0; k < ms->nv; ++k) fm = fmax(fm, fabs(ms->F[i * ms->fstride + k]));
        return 0.5 * rs * (fm + ms->ak * gm);
    }
    return rs * gm;
}

/*
 * Margin of the comparison that decides between choices `own` and `other` at
 * one face, on this side's values: d = the earlier of the two in list order.
 *   - d a stencil with m, n >= 1 (one side accepted it, the other did not):
 *     mu = (IS_d - IS0) / S, with S the larger of the rounding scales of the
 *     two sides of the comparison: sum_l |b_l| A_l for IS_d, and
 *     A_c + 2 A_{c-1} + A_{c-2} (either side of the centre) for IS0.
 *   - both chose minmod branches (Step 3.2): mu = min(|da|, |db|) / S if one
 *     took the zero branch (the sign test decided), else (|da| - |db|) / S,
 *     with da, db the two slopes and S = A_{c+1} + 2 A_c + A_{c-1}.
 * A_l is the magnitude that rounding acts on when f_l is formed (mag_at).
 * An invalid other choice gives +infinity.
 */
#define AR(l) mag_at(ms, f, c + (long)s * (l))
static double tie_margin(const orc_table *T, const double *f, const mag_src *ms, long c, int s, int own, int other,
                         const double *is, double is0)
{
    if (other < 0 || other >= T->ncand) return INFINITY;
    const int nfull = T->ncand - 3;
    const int d = own < other ? own : other;
    if (d < nfull) {
        const int m = T->m[d], n = T->n[d];
        double S = 0.0;
        for (int l = -m; l <= n; ++l) S += fabs(T->b[d][l + m]) * AR(l);
        const double s0l = AR(0) + 2.0 * AR(-1) + AR(-2);
        const double s0r = AR(0) + 2.0 * AR(1) + AR(2);
        S = fmax(S, fmax(s0l, s0r));
        return S > 0.0 ? (is[d] - is0) / S : 0.0;
    }
    const double da = FR(1) - FR(0), db = FR(0) - FR(-1);
    const double S = AR(1) + 2.0 * AR(0) + AR(-1);
    if (!(S > 0.0)) return 0.0;
    if (own == T->ncand - 1 || other == T->ncand - 1) return fmin(fabs(da), fabs(db)) / S;
    return (fabs(da) - fabs(db)) / S;
}
#undef AR

static void tie_record(orc_ties *t, int64_t pos, double mu)
{
    int64_t slot;
#pragma omp atomic capture
    slot = t->count++;
    if (slot < t->max) {
        if (t->pos) t->pos[slot] = pos;
        if (t->mu) t->mu[slot] = mu;
    }
}
#endif

/*
 * Reconstruct f-hat at face j+1/2 from cell values f (indexable from j-r+1 to
 * j+r).  sign = +1: f^+ (upwind on the left); sign = -1: f^-.  Writes the
 * chosen candidate's position in the candidate list to *idx.  ms (nullable):
 * where the near-tie margin takes the rounding magnitudes of f; ties
 * (nullable) with the log position pos of this (face, sign).
 */
static real recon_face(const orc_table *T, const real *f, const void *msv, long j, int sign, int *idx,
                       void *tiesv, int64_t pos)
{
    const int s = sign > 0 ? 1 : -1;
    const long c = (sign > 0 || ORC_PLANT == 1) ? j : j + 1;
    const int nfull = T->ncand - 3;   /* candidates 0 .. nfull-1 have m, n >= 1 */
#ifndef ORC_QUAD
    orc_ties *ties = (orc_ties *)tiesv;
    const mag_src *ms = (const mag_src *)msv;
#else
    (void)msv; (void)tiesv; (void)pos;
#endif

    /* Step 1: baseline indicator IS0 = min(IS_L, IS_R), Eq. (Baseline_IS). */
    const real f0 = FR(0), fm1 = FR(-1), fm2 = FR(-2), fp1 = FR(1), fp2 = FR(2);
    const real isl = R_MAX(R_ABS(f0 - fm1), R_ABS((f0 - (real)2 * fm1) + fm2));
    const real isr = R_MAX(R_ABS(f0 - fp1), R_ABS((f0 - (real)2 * fp1) + fp2));
    const real is0 = ORC_PLANT == 2 ? R_MAX(isl, isr) : R_MIN(isl, isr);
    OPS(11);   /* two sides of (sub, mul, sub, add, max), then min */

    /* Steps 2 and 3.1: the indicators of the candidates with m, n >= 1 in list
       order, Eqs. (CurrentIS), (ISCoe); the first with IS < IS0 is taken.
       (A near-tie margin needs the indicator of a candidate at or before the
       accepted one, so the early exit leaves every one it can need.) */
    real is[ORC_MAXC];
    int own = -1;
    for (int k = 0; k < nfull; ++k) {
        is[k] = R_ABS(stencil_dot(T->b[k], T->m[k], T->n[k], f, c, s));
        OPS(T->m[k] + T->n[k] + 1 + 1);   /* b_l chain and the compare */
        if (ORC_PLANT == 3 ? is[k] <= is0 : is[k] < is0) {
            own = k;
            if (ORC_PLANT != 4) break;
        }
    }
    real out;
    if (own >= 0) {
        OPS(T->m[own] + T->n[own] + 1);       /* the a_l chain */
        out = stencil_dot(T->a[own], T->m[own], T->n[own], f, c, s);
    } else {
        /* Step 3.2: minmod between S_j^{j+1} and S_{j-1}^j, else S_j^j. */
        OPS(7);   /* two slopes, their product, compare, |.| compare, f0 + mm/2 */
        const real da = fp1 - f0;      /* slope towards the downwind neighbour */
        const real db = f0 - fm1;      /* slope towards the upwind neighbour   */
        real mm;
        int pm, pn;
        if (da * db > (real)0) {
            if (ORC_PLANT == 5 ? R_ABS(da) > R_ABS(db) : R_ABS(da) <= R_ABS(db)) { mm = da; pm = 0; pn = 1; }
            else { mm = db; pm = 1; pn = 0; }
        } else {
            mm = (real)0; pm = 0; pn = 0;
        }
        own = T->ncand - 1;
        for (int k = nfull; k < T->ncand; ++k)
            if (T->m[k] == pm && T->n[k] == pn) own = k;
        out = f0 + (real)0.5 * mm;
    }
    *idx = own;
#ifndef ORC_QUAD
    if (ties && ties->follow) {
        const int other = ties->follow[pos];
        if (other != own) {
            const double mu = tie_margin(T, f, ms, c, s, own, other, is, is0);
            tie_record(ties, pos, mu);
            if (fabs(mu) < ties->tol) out = candidate_value(T, f, c, s, other);
        }
    }
#endif
    return out;
}
#undef FR

/*
 * Bare scalar reconstruction over n faces.  f_with_halo has n + 2r - 1
 * entries; face i lies between array cells i + r - 1 and i + r.  Log
 * position of face i: i.
 */
int ORC_FN(orc_recon_faces)(const orc_table *T, int sign, long n, const real *f_with_halo, real *fhat,
                            uint8_t *idx, void *ties)
{
    if (!T || n < 0 || (sign != 1 && sign != -1)) return ORC_EINVAL;
    const int r = T->r;
    ops_off();   /* the operation count covers the Euler operator */
    for (long i = 0; i < n; ++i) {
        int k;
        fhat[i] = recon_face(T, f_with_halo, NULL, i + r - 1, sign, &k, ties, i);
        if (idx) idx[i] = (uint8_t)k;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Boundary handling: ghost index map                                        */
/* ------------------------------------------------------------------------ */

static long map_cell(long i, long n, int bc)
{
    if (bc == ORC_PERIODIC) {
        long k = i % n;
        return k < 0 ? k + n : k;
    }
    /* outflow: zero-gradient copy of the boundary node */
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

/* ------------------------------------------------------------------------ */
/* Scalar conservation law on one line                                       */
/* ------------------------------------------------------------------------ */

static real scalar_flux(int flux, real a, real u)
{
    return flux == ORC_ADVECTION ? a * u : (real)0.5 * u * u;
}

/*
 * Global LF split (Eq. LF_Flux_Split) with alpha = max |f'(u)| over the line,
 * then f-hat = f-hat^+ + f-hat^- at faces f = 0..n (face f between cells f-1
 * and f), and du/dt = -(f-hat_{j+1/2} - f-hat_{j-1/2}) / h (Eq. 1DWENOFD).
 * With split == NONE the flux itself is reconstructed as f^+ (Sec. 4.2).
 * idx (optional): 2 entries per face, [+, -] (log positions 2f, 2f+1).
 */
int ORC_FN(orc_scalar_rhs)(const orc_table *T, int flux, real a, int split, int bc, long n, real ih,
                           const real *u, real *dudt, uint8_t *idx, real *alpha_out, void *ties)
{
    if (!T || n < 2) return ORC_EINVAL;
    const long g = T->r + 1;
    const long nn = n + 2 * g;
    real *fp = (real *)malloc(sizeof(real) * nn);
    real *fm = (real *)malloc(sizeof(real) * nn);
    real *fh = (real *)malloc(sizeof(real) * (n + 1));
    if (!fp || !fm || !fh) { free(fp); free(fm); free(fh); return ORC_EINVAL; }

    real alpha = 0;
    for (long i = 0; i < n; ++i) {
        real d = flux == ORC_ADVECTION ? R_ABS(a) : R_ABS(u[i]);
        if (d > alpha) alpha = d;
    }
    if (alpha_out) *alpha_out = alpha;

    for (long i = 0; i < nn; ++i) {
        real ui = u[map_cell(i - g, n, bc)];
        real fi = scalar_flux(flux, a, ui);
        if (split == ORC_SPLIT_LF) {
            real t = alpha * ui;
            fp[i] = (real)0.5 * (fi + t);
            fm[i] = (real)0.5 * (fi - t);
        } else {
            fp[i] = fi;
            fm[i] = 0;
        }
    }
#pragma omp parallel if (n >= ORC_PAR_FACES)
    {
    ops_off();   /* the operation count covers the Euler operator */
#pragma omp for schedule(static)
    for (long f = 0; f <= n; ++f) {
        long j = f - 1 + g;           /* left cell of face f in the ghosted array */
        int kp, km = 0;
        real hp = recon_face(T, fp, NULL, j, +1, &kp, ties, 2 * (int64_t)f);
        real hm = 0;
        if (split == ORC_SPLIT_LF) hm = recon_face(T, fm, NULL, j, -1, &km, ties, 2 * (int64_t)f + 1);
        fh[f] = hp + hm;
        if (idx) { idx[2 * f] = (uint8_t)kp; idx[2 * f + 1] = (uint8_t)km; }
    }
    }
    for (long i = 0; i < n; ++i) dudt[i] = -((fh[i + 1] - fh[i]) * ih);
    free(fp); free(fm); free(fh);
    return ORC_OK;
}

/*
 * Linear SSP-RK(m, m-1) step for a scalar line (Eq. lSSPRK):
 * u^(s) = u^(s-1) + dt/2 L(u^(s-1)), s = 1..m-1, and
 * u^{n+1} = sum_{k<m-1} a_k u^(k) + a_{m-1} (u^(m-1) + dt/2 L(u^(m-1))).
 * coef holds a_0..a_{m-1} (exact fractions from the caller, Eq. lSSPRK_Coe,
 * each rounded by one division).
 */
static int lssp_run(const orc_table *T, int flux, real a, int split, int bc, long n, real ih, real dt, long nsteps,
                    int m, const real *coef, real *u)
{
    if (m < 2 || m > 32) return ORC_EINVAL;
    real *stages = (real *)malloc(sizeof(real) * n * m);
    real *L = (real *)malloc(sizeof(real) * n);
    real *acc = (real *)malloc(sizeof(real) * n);
    int st = ORC_OK;
    if (!stages || !L || !acc) { st = ORC_EINVAL; goto done; }
    const real hdt = (real)0.5 * dt;
    for (long step = 0; step < nsteps; ++step) {
        memcpy(stages, u, sizeof(real) * n);
        for (int s = 1; s < m; ++s) {
            if ((st = ORC_FN(orc_scalar_rhs)(T, flux, a, split, bc, n, ih, stages + (s - 1) * n, L, NULL, NULL,
                                             NULL)))
                goto done;
            for (long i = 0; i < n; ++i) stages[s * n + i] = stages[(s - 1) * n + i] + hdt * L[i];
        }
        if ((st = ORC_FN(orc_scalar_rhs)(T, flux, a, split, bc, n, ih, stages + (m - 1) * n, L, NULL, NULL, NULL)))
            goto done;
        for (long i = 0; i < n; ++i) acc[i] = 0;
        for (int k = 0; k < m - 1; ++k)
            for (long i = 0; i < n; ++i) acc[i] = acc[i] + coef[k] * stages[k * n + i];
        for (long i = 0; i < n; ++i)
            u[i] = acc[i] + coef[m - 1] * (stages[(m - 1) * n + i] + hdt * L[i]);
    }
done:
    free(stages); free(L); free(acc);
    return st;
}

static int lssp_coefs(int m, const int64_t *cnum, const int64_t *cden, real *coef)
{
    if (m < 2 || m > 32) return ORC_EINVAL;
    for (int k = 0; k < m; ++k) coef[k] = (real)cnum[k] / (real)cden[k];
    return ORC_OK;
}

int ORC_FN(orc_scalar_lssp_run)(const orc_table *T, int flux, real a, int split, int bc, long n, real ih, real dt,
                                long nsteps, int m, const int64_t *cnum, const int64_t *cden, real *u)
{
    real coef[32];
    if (lssp_coefs(m, cnum, cden, coef)) return ORC_EINVAL;
    return lssp_run(T, flux, a, split, bc, n, ih, dt, nsteps, m, coef, u);
}

/*
 * SSP-RK3 stage combination (Eq. TVD3rdRK), elementwise over n values:
 *   stage 1: out = us + dt L
 *   stage 2: out = 3/4 un + 1/4 (us + dt L)
 *   stage 3: out = 1/3 un + 2/3 (us + dt L)
 */
void ORC_FN(orc_ssprk3_combine)(int stage, long n, const real *un, const real *us, const real *L, real dt,
                                real *out)
{
    const real c13 = (real)1 / (real)3, c23 = (real)2 / (real)3;
    ops_enter(ORC_OPS_RK);
    OPS((stage == 1 ? 2 : 5) * n);
    ops_flush();
    for (long i = 0; i < n; ++i) {
        real e = us[i] + dt * L[i];
        if (stage == 1) out[i] = e;
        else if (stage == 2) out[i] = (real)0.75 * un[i] + (real)0.25 * e;
        else out[i] = c13 * un[i] + c23 * e;
    }
}

/*
 * SSP-RK3 run of a scalar line with a fixed step dt; the last step is cut so
 * that the run ends exactly at t_end (if t_end > 0, else nsteps steps).
 */
int ORC_FN(orc_scalar_ssprk3_run)(const orc_table *T, int flux, real a, int split, int bc, long n, real ih, real dt,
                                  real t_end, long nsteps, real *u)
{
    real *un = (real *)malloc(sizeof(real) * n);
    real *us = (real *)malloc(sizeof(real) * n);
    real *L = (real *)malloc(sizeof(real) * n);
    int st = ORC_OK;
    if (!un || !us || !L) { st = ORC_EINVAL; goto done; }
    real t = 0;
    for (long step = 0; t_end > 0 ? t < t_end : step < nsteps; ++step) {
        real h = dt;
        if (t_end > 0 && t + h > t_end) h = t_end - t;
        memcpy(un, u, sizeof(real) * n);
        memcpy(us, u, sizeof(real) * n);
        for (int s = 1; s <= 3; ++s) {
            if ((st = ORC_FN(orc_scalar_rhs)(T, flux, a, split, bc, n, ih, us, L, NULL, NULL, NULL))) goto done;
            ORC_FN(orc_ssprk3_combine)(s, n, un, us, L, h, us);
        }
        memcpy(u, us, sizeof(real) * n);
        t = t + h;
    }
done:
    free(un); free(us); free(L);
    return st;
}

#ifdef ORC_QUAD
/*
 * The linear convergence test of Sec. 4.1 in binary128, start to finish:
 * u0 = lam sin^alpha(pi x) on the n nodes x_j = -1 + (j-1) h, h = 2/n,
 * periodic, linear advection with a = 1, LF split, linear SSP-RK(m, m-1) with
 * dt = h to t = 2 (n steps), after which the exact solution is u0 again.
 * Errors: L1 = mean of |u - u0| over the n+1 points x_1 .. x_{n+1} (the
 * periodic end point counted twice), Linf = max; both rounded to double.
 */
int orc_q_advection_errors(const orc_table *T, int alpha, double lam, long n, int m, const int64_t *cnum,
                           const int64_t *cden, double *l1, double *linf)
{
    if (!T || n < 2 * T->r + 1) return ORC_EINVAL;
    real *u0 = (real *)malloc(sizeof(real) * n);
    real *u = (real *)malloc(sizeof(real) * n);
    if (!u0 || !u) { free(u0); free(u); return ORC_EINVAL; }
    const real h = (real)2 / (real)n;
    for (long j = 0; j < n; ++j) {
        const real x = (real)-1 + (real)j * h;
        real sv = sinq(M_PIq * x), p = 1;
        for (int k = 0; k < alpha; ++k) p = p * sv;
        u0[j] = (real)lam * p;
        u[j] = u0[j];
    }
    int st = ORC_FN(orc_scalar_lssp_run)(T, ORC_ADVECTION, (real)1, ORC_SPLIT_LF, ORC_PERIODIC, n, (real)1 / h, h, n,
                                         m, cnum, cden, u);
    if (!st) {
        real s = 0, mx = 0;
        for (long j = 0; j < n; ++j) {
            const real e = fabsq(u[j] - u0[j]);
            s = s + e;
            if (e > mx) mx = e;
        }
        s = s + fabsq(u[0] - u0[0]);
        *l1 = (double)(s / (real)(n + 1));
        *linf = (double)mx;
    }
    free(u0); free(u);
    return st;
}
#endif

#ifndef ORC_QUAD
/* ------------------------------------------------------------------------ */
/* Euler equations: one line in the face-normal frame                        */
/* ------------------------------------------------------------------------ */

/*
 * A line state holds nv = 3 (rho, m, E) or nv = 4 (rho, m_n, m_t, E)
 * conserved variables, the momentum m_n normal to the faces.
 */
typedef struct {
    double un, ut, p, c, H, sq;
    double F[4];
} cell_prim;

/* Primitive quantities and fluxes of one cell (18 ops for nv = 4, 14 for nv = 3). */
static int primitives(int nv, double gamma, const double *U, cell_prim *q)
{
    const double rho = U[0], mn = U[1], mt = nv == 4 ? U[2] : 0.0, E = U[nv - 1];
    const double un = mn / rho;
    const double ut = nv == 4 ? mt / rho : 0.0;
    const double ke = nv == 4 ? 0.5 * (mn * un + mt * ut) : 0.5 * (mn * un);
    const double p = (gamma - 1.0) * (E - ke);
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(mn)) return ORC_ENONPHYS;
    q->un = un;
    q->ut = ut;
    q->p = p;
    q->c = sqrt(gamma * p / rho);
    q->H = (E + p) / rho;
    q->sq = sqrt(rho);                 /* the cell's Roe weight */
    q->F[0] = mn;
    q->F[1] = mn * un + p;
    if (nv == 4) {
        q->F[2] = mt * un;
        q->F[3] = (E + p) * un;
    } else {
        q->F[2] = (E + p) * un;
    }
    return ORC_OK;
}

/*
 * Roe-averaged eigenvectors at the face between cells with primitives qL, qR
 * (Sec. 4 preamble): the Roe state from sqrt(rho) weights, c^2 = (gamma-1)
 * (H - q^2/2), and the closed-form right eigenvectors of the face-normal flux
 * Jacobian for the fields (u-c, u, [shear,] u+c), with Lm = Rm^{-1} written
 * with k = (gamma-1)/c^2.  Returns nonzero if c^2 is not positive.
 * 42 ops for nv = 4, 34 for nv = 3.
 */
static int roe_eigen(int nv, double gamma, const cell_prim *qL, const cell_prim *qR, double Lm[4][4],
                     double Rm[4][4])
{
    const double sL = qL->sq, sR = qR->sq;
    const double den = sL + sR;
    const double u = ORC_PLANT == 6 ? 0.5 * (qL->un + qR->un) : (sL * qL->un + sR * qR->un) / den;
    const double v = nv == 4 ? (sL * qL->ut + sR * qR->ut) / den : 0.0;
    const double H = (sL * qL->H + sR * qR->H) / den;
    const double q2 = nv == 4 ? u * u + v * v : u * u;
    const double hq2 = 0.5 * q2;
    const double c2 = (gamma - 1.0) * (H - hq2);
    if (!(c2 > 0.0)) return ORC_ENONPHYS;
    const double c = sqrt(c2);
    const double k = (gamma - 1.0) / c2;
    const double hk = 0.5 * k;
    const double hq = hk * q2;
    const double uic = u / c;
    const double ic = 1.0 / c;
    const double ku = k * u;
    const double uc = u * c;
    memset(Lm, 0, sizeof(double) * 16);
    memset(Rm, 0, sizeof(double) * 16);
    if (nv == 4) {
        const double kv = k * v;
        const double lv = -0.5 * kv;
        const double L[4][4] = {
            {0.5 * (hq + uic), (ORC_PLANT == 7 ? 0.5 : -0.5) * (ku + ic), lv, hk},
            {1.0 - hq, ku, kv, -k},
            {-v, 0.0, 1.0, 0.0},
            {0.5 * (hq - uic), -0.5 * (ku - ic), lv, hk},
        };
        const double R[4][4] = {
            {1.0, 1.0, 0.0, 1.0},
            {u - c, u, 0.0, u + c},
            {v, v, 1.0, v},
            {H - uc, hq2, v, H + uc},
        };
        memcpy(Lm, L, sizeof(L));
        memcpy(Rm, R, sizeof(R));
        OPS(42);
    } else {
        const double L[3][3] = {
            {0.5 * (hq + uic), -0.5 * (ku + ic), hk},
            {1.0 - hq, ku, -k},
            {0.5 * (hq - uic), -0.5 * (ku - ic), hk},
        };
        const double R[3][3] = {
            {1.0, 1.0, 1.0},
            {u - c, u, u + c},
            {H - uc, hq2, H + uc},
        };
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                Lm[i][j] = L[i][j];
                Rm[i][j] = R[i][j];
            }
        OPS(34);
    }
    return ORC_OK;
}

/* Exported for the eigenvector tests: L and R at the Roe state of UL, UR. */
int orc_roe_eigen(int nv, double gamma, const double *UL, const double *UR, double *Lout, double *Rout)
{
    cell_prim qL, qR;
    if (primitives(nv, gamma, UL, &qL) || primitives(nv, gamma, UR, &qR)) return ORC_ENONPHYS;
    double Lm[4][4], Rm[4][4];
    int st = roe_eigen(nv, gamma, &qL, &qR, Lm, Rm);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            Lout[i * nv + j] = Lm[i][j];
            Rout[i * nv + j] = Rm[i][j];
        }
    return st;
}

/* sum_i row[i] x[i] as an fma chain over ascending i (nv ops). */
static double row_dot(const double *row, const double *x, int nv)
{
    double acc = row[0] * x[0];
    for (int i = 1; i < nv; ++i) acc = fma(row[i], x[i], acc);
    return acc;
}

/*
 * Largest characteristic speed |u_n| + c over the n cells of a line
 * (alpha of Eq. LF_Flux_Split for the Euler system).
 */
static int line_alpha(int nv, double gamma, long n, const double *Ul, double *alpha)
{
    double amax = 0.0;
    for (long i = 0; i < n; ++i) {
        double U[4];
        for (int v = 0; v < nv; ++v) U[v] = Ul[v * n + i];
        cell_prim q;
        if (primitives(nv, gamma, U, &q)) return ORC_ENONPHYS;
        double s = fabs(q.un) + q.c;
        if (s > amax) amax = s;
    }
    *alpha = amax;
    return ORC_OK;
}

/*
 * Per-field alphas of one line: a[0] = max |u_n - c|, a[1] = max |u_n|,
 * a[2] = max |u_n + c| over its n cells (the characteristic speeds of the
 * fields u-c, u (and the shear field) and u+c).
 */
static int line_alpha_fields(int nv, double gamma, long n, const double *Ul, double a[3])
{
    a[0] = a[1] = a[2] = 0.0;
    for (long i = 0; i < n; ++i) {
        double U[4];
        for (int v = 0; v < nv; ++v) U[v] = Ul[v * n + i];
        cell_prim q;
        if (primitives(nv, gamma, U, &q)) return ORC_ENONPHYS;
        double s0 = fabs(q.un - q.c), s1 = fabs(q.un), s2 = fabs(q.un + q.c);
        if (s0 > a[0]) a[0] = s0;
        if (s1 > a[1]) a[1] = s1;
        if (s2 > a[2]) a[2] = s2;
    }
    return ORC_OK;
}

/* Which of the three per-field alphas field k of an nv-field system uses. */
static int field_speed(int nv, int k)
{
    if (k == 0) return 0;
    if (k == nv - 1) return 2;
    return 1;
}

/* Operator variants (see the header comment). */
typedef struct {
    int componentwise;
    int per_field;
} euler_var;

/*
 * Numerical fluxes at faces f = 0..n of one line (face f between cells f-1
 * and f).  Ul is [nv][n] in the face-normal frame.  Fhat is [n+1][nv].
 * alpha: the line's alpha, or its three per-field alphas (var.per_field).
 * idx (optional) holds nv*2 entries per face: [(field)*2 + (0:+, 1:-)].
 * ties (nullable): the near-tie record; the log position of (face f, field
 * k, sign index sg) is pos0 + f * fstride + 2k + sg.  par: faces in parallel
 * (for a line that is alone; the 2D operator parallelises over lines).
 */
static int euler_line_fluxes(const orc_table *T, int nv, double gamma, int bc, long n, const double *Ul,
                             const double *alpha, euler_var var, double *Fhat, uint8_t *idx, orc_ties *ties,
                             int64_t pos0, int64_t fstride, int par)
{
    const long g = T->r + 1;
    const long nn = n + 2 * g;
    const int W = 2 * T->r - 1;
    double *U = (double *)malloc(sizeof(double) * nn * nv);
    double *Gp = (double *)malloc(sizeof(double) * nn * nv);
    double *Gm = (double *)malloc(sizeof(double) * nn * nv);
    cell_prim *Q = (cell_prim *)malloc(sizeof(cell_prim) * nn);
    int st = ORC_OK;
    const int counting = !var.componentwise && !var.per_field;
    if (!U || !Gp || !Gm || !Q) { st = ORC_EINVAL; goto done; }

    /* Ghosted line, primitive quantities and the LF split G = (F +- alpha U)/2
       (with per-field alphas the split is taken after the projection). */
    for (long i = 0; i < nn; ++i) {
        long src = map_cell(i - g, n, bc);
        for (int v = 0; v < nv; ++v) U[i * nv + v] = Ul[v * n + src];
        if ((st = primitives(nv, gamma, &U[i * nv], &Q[i]))) goto done;
        for (int v = 0; v < nv; ++v) {
            double t = alpha[0] * U[i * nv + v];
            Gp[i * nv + v] = 0.5 * (Q[i].F[v] + t);
            Gm[i * nv + v] = ORC_PLANT == 8 ? 0.5 * (Q[i].F[v] + t) : 0.5 * (Q[i].F[v] - t);
        }
        /* once per cell of the line: the primitives and fluxes, and the split
           (t, the sum and the difference, two halvings: 5 per component) */
        if (counting && i >= g && i < g + n) OPS((nv == 4 ? 18 : 14) + 5 * nv);
    }

    const int cat = t_cat;
#pragma omp parallel if (par)
    {
        ops_enter(cat);
        if (!counting) t_count = 0;
        double *wp = (double *)malloc(sizeof(double) * nn);
        double *wm = (double *)malloc(sizeof(double) * nn);
        if (!wp || !wm) {
#pragma omp atomic write
            st = ORC_EINVAL;
        } else {
#pragma omp for schedule(static)
            for (long f = 0; f <= n; ++f) {
                const long j = f - 1 + g;      /* left cell of the face in the ghosted line */
                /* a periodic line's face n is its face 0 again: counted once */
                t_count = counting && g_count_on && !(bc == ORC_PERIODIC && f == n);
                if (var.componentwise) {
                    for (int k = 0; k < nv; ++k) {
                        for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                            wp[i] = Gp[i * nv + k];
                            wm[i] = Gm[i * nv + k];
                        }
                        int kp, km;
                        const int64_t pk = pos0 + f * fstride + 2 * k;
                        const mag_src msp = {NULL, Gp, NULL, 0, 0.0, nv}, msm = {NULL, Gm, NULL, 0, 0.0, nv};
                        double hp = recon_face(T, wp, &msp, j, +1, &kp, ties, pk);
                        double hm = recon_face(T, wm, &msm, j, -1, &km, ties, pk + 1);
                        Fhat[f * nv + k] = hp + hm;
                        if (idx) {
                            idx[(f * nv + k) * 2 + 0] = (uint8_t)kp;
                            idx[(f * nv + k) * 2 + 1] = (uint8_t)km;
                        }
                    }
                    continue;
                }
                double Lm[4][4], Rm[4][4];
                if (roe_eigen(nv, gamma, &Q[j], &Q[j + 1], Lm, Rm)) {
#pragma omp atomic write
                    st = ORC_ENONPHYS;
                    continue;
                }
                /* the projection of every window cell onto every field: per
                   sign W cells, nv rows of nv terms */
                OPS(2 * W * nv * nv);
                double what[4];
                for (int k = 0; k < nv; ++k) {
                    /* characteristic field k of the split fluxes over the face's window */
                    mag_src msp = {Lm[k], Gp, NULL, 0, 0.0, nv}, msm = {Lm[k], Gm, NULL, 0, 0.0, nv};
                    if (var.per_field) {
                        const double ak = alpha[field_speed(nv, k)];
                        for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                            const double pf = row_dot(Lm[k], Q[i].F, nv);
                            const double t = ak * row_dot(Lm[k], &U[i * nv], nv);
                            wp[i] = 0.5 * (pf + t);
                            wm[i] = 0.5 * (pf - t);
                        }
                        msp.G = msm.G = U;
                        msp.F = msm.F = Q[0].F;
                        msp.fstride = msm.fstride = (long)(sizeof(cell_prim) / sizeof(double));
                        msp.ak = msm.ak = ak;
                    } else {
                        for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                            const int kr = ORC_PLANT == 9 ? (k + 1) % nv : k;
                            wp[i] = row_dot(Lm[kr], &Gp[i * nv], nv);
                            wm[i] = row_dot(Lm[kr], &Gm[i * nv], nv);
                        }
                    }
                    int kp, km;
                    const int64_t pk = pos0 + f * fstride + 2 * k;
                    double hp = recon_face(T, wp, &msp, j, +1, &kp, ties, pk);
                    double hm = recon_face(T, wm, &msm, j, -1, &km, ties, pk + 1);
                    what[k] = ORC_PLANT == 10 ? hp : hp + hm;
                    if (idx) {
                        idx[(f * nv + k) * 2 + 0] = (uint8_t)kp;
                        idx[(f * nv + k) * 2 + 1] = (uint8_t)km;
                    }
                }
                /* back to conserved components: w-hat+ + w-hat-, then F-hat = R w-hat */
                for (int v = 0; v < nv; ++v) Fhat[f * nv + v] = row_dot(Rm[v], what, nv);
                OPS(nv + nv * nv);
            }
        }
        free(wp); free(wm);
        t_count = g_count_on;
        ops_flush();
    }
done:
    free(U); free(Gp); free(Gm); free(Q);
    return st;
}

/* A line's alpha (one value) or per-field alphas (three values). */
static int line_alphas(int nv, double gamma, long n, const double *Ul, euler_var var, double a[3])
{
    if (var.per_field) return line_alpha_fields(nv, gamma, n, Ul, a);
    a[1] = a[2] = 0.0;
    return line_alpha(nv, gamma, n, Ul, &a[0]);
}

/*
 * 1D Euler right-hand side L(U), U and dUdt laid out [3][n], with the
 * variant switches componentwise and per_field (not both).  alpha_out
 * (optional) receives the line's alpha, or its three per-field alphas.
 * idx: [n+1][3][2]; ties (nullable) against a log of that layout.
 */
int orc_euler1d_rhs_var(const orc_table *T, double gamma, int bc, long n, double ih, const double *U, double *dUdt,
                        uint8_t *idx, double *alpha_out, int componentwise, int per_field, orc_ties *ties)
{
    if (!T || n < 2 || (componentwise && per_field)) return ORC_EINVAL;
    euler_var var = {componentwise != 0, per_field != 0};
    double alpha[3];
    int st = line_alphas(3, gamma, n, U, var, alpha);
    if (st) return st;
    if (alpha_out)
        for (int k = 0; k < (per_field ? 3 : 1); ++k) alpha_out[k] = alpha[k];
    double *Fh = (double *)malloc(sizeof(double) * (n + 1) * 3);
    if (!Fh) return ORC_EINVAL;
    ops_enter(ORC_OPS_X);
    st = euler_line_fluxes(T, 3, gamma, bc, n, U, alpha, var, Fh, idx, ties, 0, 6, 1);
    if (!st) {
        for (int v = 0; v < 3; ++v)
            for (long i = 0; i < n; ++i)
                dUdt[v * n + i] = -((Fh[(i + 1) * 3 + v] - Fh[i * 3 + v]) * ih);
        if (!componentwise && !per_field) OPS(2 * 3 * n);   /* the difference: sub, mul */
    }
    ops_flush();
    free(Fh);
    return st;
}

/* 1D Euler right-hand side L(U), U and dUdt laid out [3][n]. */
int orc_euler1d_rhs(const orc_table *T, double gamma, int bc, long n, double ih, const double *U, double *dUdt,
                    uint8_t *idx, double *alpha_out, orc_ties *ties)
{
    return orc_euler1d_rhs_var(T, gamma, bc, n, ih, U, dUdt, idx, alpha_out, 0, 0, ties);
}

/*
 * 2D Euler right-hand side, dimension by dimension (Sec. 2.1):
 * dU/dt = -(F_{i+1/2} - F_{i-1/2})/hx - (G_{j+1/2} - G_{j-1/2})/hy.
 * U, dUdt: [4][ny][nx].  x-lines use (rho, m, n, E); y-lines the permuted
 * state (rho, n, m, E) so that the same normal-frame formulas apply.
 * idx_x (optional): [ny][nx+1][4][2]; idx_y (optional): [ny+1][nx][4][2].
 * ties (nullable): against a log holding the x faces' log followed by the y
 * faces' log, both laid out as idx_x, idx_y.
 * alpha_x[ny], alpha_y[nx] (optional) receive the per-line alphas; with
 * per_field, alpha_x[3][ny] and alpha_y[3][nx] the per-field ones.
 * componentwise, per_field (not both): the variants of the header comment;
 * gravity g != 0 adds the source g [0, 0, rho, rho v] to the result.
 * Lines run in parallel (OpenMP); results do not depend on the thread count.
 */
int orc_euler2d_rhs_var(const orc_table *T, double gamma, int bcx, int bcy, long nx, long ny, double ihx,
                        double ihy, const double *U, double *dUdt, uint8_t *idx_x, uint8_t *idx_y, double *alpha_x,
                        double *alpha_y, int componentwise, int per_field, double gravity, orc_ties *ties)
{
    if (!T || nx < 2 || ny < 2 || (componentwise && per_field)) return ORC_EINVAL;
    euler_var var = {componentwise != 0, per_field != 0};
    const int na = per_field ? 3 : 1;
    const int counting = !componentwise && !per_field;
    const long plane = nx * ny;
    const int64_t nxf = (int64_t)ny * (nx + 1) * 8;
    double *Lx = (double *)malloc(sizeof(double) * 4 * plane);
    int st = ORC_OK;
    if (!Lx) return ORC_EINVAL;

    /* x sweep */
#pragma omp parallel
    {
        double *line = (double *)malloc(sizeof(double) * 4 * nx);
        double *Fh = (double *)malloc(sizeof(double) * 4 * (nx + 1));
        uint8_t *idl = (uint8_t *)malloc(8 * (nx + 1));
        ops_enter(ORC_OPS_X);
        if (!line || !Fh || !idl) {
#pragma omp atomic write
            st = ORC_EINVAL;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (long y = 0; y < ny; ++y) {
                for (int v = 0; v < 4; ++v)
                    for (long x = 0; x < nx; ++x) line[v * nx + x] = U[v * plane + y * nx + x];
                double alpha[3];
                int ls = line_alphas(4, gamma, nx, line, var, alpha);
                if (!ls && alpha_x)
                    for (int k = 0; k < na; ++k) alpha_x[k * ny + y] = alpha[k];
                if (!ls)
                    ls = euler_line_fluxes(T, 4, gamma, bcx, nx, line, alpha, var, Fh, idx_x ? idl : NULL, ties,
                                           (int64_t)y * (nx + 1) * 8, 8, 0);
                if (ls) {
#pragma omp atomic write
                    st = ls;
                    continue;
                }
                if (idx_x) memcpy(idx_x + (size_t)y * (nx + 1) * 8, idl, (size_t)(nx + 1) * 8);
                for (int v = 0; v < 4; ++v)
                    for (long x = 0; x < nx; ++x)
                        Lx[v * plane + y * nx + x] = -((Fh[(x + 1) * 4 + v] - Fh[x * 4 + v]) * ihx);
                if (counting) OPS(2 * 4 * nx);
            }
        }
        free(line); free(Fh); free(idl);
        ops_flush();
    }
    if (st) goto done;
    /* y sweep on the permuted state, then the sum */
#pragma omp parallel
    {
        static const int perm[4] = {0, 2, 1, 3};
        double *line = (double *)malloc(sizeof(double) * 4 * ny);
        double *Fh = (double *)malloc(sizeof(double) * 4 * (ny + 1));
        uint8_t *idl = (uint8_t *)malloc(8 * (ny + 1));
        ops_enter(ORC_OPS_Y);
        if (!line || !Fh || !idl) {
#pragma omp atomic write
            st = ORC_EINVAL;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (long x = 0; x < nx; ++x) {
                for (int v = 0; v < 4; ++v)
                    for (long y = 0; y < ny; ++y) line[v * ny + y] = U[perm[v] * plane + y * nx + x];
                double alpha[3];
                int ls = line_alphas(4, gamma, ny, line, var, alpha);
                if (!ls && alpha_y)
                    for (int k = 0; k < na; ++k) alpha_y[k * nx + x] = alpha[k];
                if (!ls)
                    ls = euler_line_fluxes(T, 4, gamma, bcy, ny, line, alpha, var, Fh, idx_y ? idl : NULL, ties,
                                           nxf + (int64_t)x * 8, (int64_t)nx * 8, 0);
                if (ls) {
#pragma omp atomic write
                    st = ls;
                    continue;
                }
                if (idx_y)
                    for (long f = 0; f <= ny; ++f) memcpy(idx_y + ((size_t)f * nx + x) * 8, idl + f * 8, 8);
                for (int v = 0; v < 4; ++v)
                    for (long y = 0; y < ny; ++y) {
                        int cv = perm[v];
                        double ly = -((Fh[(y + 1) * 4 + v] - Fh[y * 4 + v]) * ihy);
                        dUdt[cv * plane + y * nx + x] = Lx[cv * plane + y * nx + x] + ly;
                    }
                if (counting) {
                    OPS(2 * 4 * ny);               /* the difference */
                    t_cat = ORC_OPS_SUM;
                    OPS(4 * ny);                   /* L_x + L_y */
                    t_cat = ORC_OPS_Y;
                }
            }
        }
        free(line); free(Fh); free(idl);
        ops_flush();
    }
    /* source term of the Rayleigh-Taylor problem (Sec. 4.4): rho g in the
       y-momentum, rho v g in the energy equation */
    if (!st && gravity != 0.0)
        for (long i = 0; i < plane; ++i) {
            dUdt[2 * plane + i] = dUdt[2 * plane + i] + gravity * U[i];
            dUdt[3 * plane + i] = dUdt[3 * plane + i] + gravity * U[2 * plane + i];
        }
done:
    free(Lx);
    return st;
}

int orc_euler2d_rhs(const orc_table *T, double gamma, int bcx, int bcy, long nx, long ny, double ihx, double ihy,
                    const double *U, double *dUdt, uint8_t *idx_x, uint8_t *idx_y, double *alpha_x,
                    double *alpha_y, orc_ties *ties)
{
    return orc_euler2d_rhs_var(T, gamma, bcx, bcy, nx, ny, ihx, ihy, U, dUdt, idx_x, idx_y, alpha_x, alpha_y, 0, 0,
                               0.0, ties);
}

/* ------------------------------------------------------------------------ */
/* Time step                                                                 */
/* ------------------------------------------------------------------------ */

/* Largest |u_n| + c over a [nv][n] array of cells (normal = component 1). */
int orc_euler_maxspeed(int nv, double gamma, long n, const double *U, double *smax)
{
    return line_alpha(nv, gamma, n, U, smax);
}

/* 2D: largest |u| + c and |v| + c over the grid. */
int orc_euler2d_maxspeeds(double gamma, long nx, long ny, const double *U, double *sx, double *sy)
{
    const long plane = nx * ny;
    double ax = 0.0, ay = 0.0;
    for (long i = 0; i < plane; ++i) {
        double Uc[4] = {U[i], U[plane + i], U[2 * plane + i], U[3 * plane + i]};
        cell_prim q;
        if (primitives(4, gamma, Uc, &q)) return ORC_ENONPHYS;
        double a = fabs(q.un) + q.c;
        double b = fabs(q.ut) + q.c;
        if (a > ax) ax = a;
        if (b > ay) ay = b;
    }
    *sx = ax;
    *sy = ay;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Frozen-stencil 1D Euler operator with its tangent (dual numbers)          */
/* ------------------------------------------------------------------------ */

/*
 * With the stencil choices (idx), the line's alpha and therefore every
 * branch fixed, L(U) is a smooth function of U.  Each quantity below carries
 * its value (computed with exactly the operations of the forward operator
 * above, so the value part equals L(U) when idx and alpha are the ones the
 * forward chose) and its directional derivative along dU.
 */
typedef struct {
    double v, d;
} dual;

static dual D(double v) { dual r = {v, 0.0}; return r; }
static dual dadd(dual a, dual b) { dual r = {a.v + b.v, a.d + b.d}; return r; }
static dual dsub(dual a, dual b) { dual r = {a.v - b.v, a.d - b.d}; return r; }
static dual dmul(dual a, dual b) { dual r = {a.v * b.v, a.d * b.v + a.v * b.d}; return r; }
static dual dscale(double c, dual a) { dual r = {c * a.v, c * a.d}; return r; }
static dual ddiv(dual a, dual b) { dual r = {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; return r; }
static dual dsqrt(dual a) { double s = sqrt(a.v); dual r = {s, a.d / (2.0 * s)}; return r; }
static dual dfma(dual a, dual b, dual c) { dual r = {fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d}; return r; }

/* row_dot() in dual arithmetic */
static dual ddot(const dual *c, const dual *x, int n)
{
    dual acc = dmul(c[0], x[0]);
    for (int i = 1; i < n; ++i) acc = dfma(c[i], x[i], acc);
    return acc;
}

/* candidate_value() of a frozen choice k in dual arithmetic (frame as in recon_face) */
static dual recon_frozen(const orc_table *T, const dual *f, long j, int sign, int k)
{
    const int s = sign > 0 ? 1 : -1;
    const long c = sign > 0 ? j : j + 1;
#define FD(l) (f[c + (long)s * (l)])
    const int m = T->m[k], n = T->n[k];
    if (m >= 1 && n >= 1) {
        int l = (s > 0) ? -m : n;
        const int dl = (s > 0) ? 1 : -1;
        dual acc = dmul(D(T->a[k][l + m]), FD(l));
        for (int q = 1; q < m + n + 1; ++q) {
            l += dl;
            acc = dfma(D(T->a[k][l + m]), FD(l), acc);
        }
        return acc;
    }
    dual f0 = FD(0), mm;
    if (m == 0 && n == 1) mm = dsub(FD(1), f0);          /* S_j^{j+1} branch */
    else if (m == 1 && n == 0) mm = dsub(f0, FD(-1));    /* S_{j-1}^j branch */
    else mm = D(0.0);                                     /* S_j^j */
#undef FD
    return dadd(f0, dscale(0.5, mm));
}

/*
 * Frozen operator and tangent: L = L(U; idx, alpha), dL = dL/dU . dU.
 * U, dU, L, dL: [3][n]; idx: [n+1][3][2] as from orc_euler1d_rhs.  dU and dL
 * may be NULL (value only).
 */
int orc_euler1d_rhs_frozen(const orc_table *T, double gamma, int bc, long n, double ih, const double *U,
                           const double *dU, const uint8_t *idx, double alpha, double *L, double *dL)
{
    if (!T || n < 2 || !idx) return ORC_EINVAL;
    const long g = T->r + 1;
    const long nn = n + 2 * g;
    const double gm1 = gamma - 1.0;
    dual *Gp = (dual *)malloc(sizeof(dual) * nn * 3);
    dual *Gm = (dual *)malloc(sizeof(dual) * nn * 3);
    dual *un = (dual *)malloc(sizeof(dual) * nn);
    dual *H = (dual *)malloc(sizeof(dual) * nn);
    dual *sq = (dual *)malloc(sizeof(dual) * nn);
    dual *wp = (dual *)malloc(sizeof(dual) * nn);
    dual *wm = (dual *)malloc(sizeof(dual) * nn);
    dual *Fh = (dual *)malloc(sizeof(dual) * (n + 1) * 3);
    int st = ORC_OK;
    if (!Gp || !Gm || !un || !H || !sq || !wp || !wm || !Fh) { st = ORC_EINVAL; goto done; }
    for (long i = 0; i < nn; ++i) {
        long src = map_cell(i - g, n, bc);
        dual rho = {U[src], dU ? dU[src] : 0.0};
        dual mn = {U[n + src], dU ? dU[n + src] : 0.0};
        dual E = {U[2 * n + src], dU ? dU[2 * n + src] : 0.0};
        dual u = ddiv(mn, rho);
        dual ke = dscale(0.5, dmul(mn, u));
        dual p = dscale(gm1, dsub(E, ke));
        if (!(rho.v > 0.0) || !(p.v > 0.0)) { st = ORC_ENONPHYS; goto done; }
        dual Ep = dadd(E, p);
        dual F[3] = {mn, dadd(dmul(mn, u), p), dmul(Ep, u)};
        dual Ucs[3] = {rho, mn, E};
        for (int v = 0; v < 3; ++v) {
            dual t = dscale(alpha, Ucs[v]);
            Gp[i * 3 + v] = dscale(0.5, dadd(F[v], t));
            Gm[i * 3 + v] = dscale(0.5, dsub(F[v], t));
        }
        un[i] = u;
        H[i] = ddiv(Ep, rho);
        sq[i] = dsqrt(rho);
    }
    for (long f = 0; f <= n; ++f) {
        long j = f - 1 + g;
        /* Roe eigenvectors, the formulas of roe_eigen() in dual arithmetic */
        dual den = dadd(sq[j], sq[j + 1]);
        dual u = ddiv(dadd(dmul(sq[j], un[j]), dmul(sq[j + 1], un[j + 1])), den);
        dual Hr = ddiv(dadd(dmul(sq[j], H[j]), dmul(sq[j + 1], H[j + 1])), den);
        dual q2 = dmul(u, u);
        dual hq2 = dscale(0.5, q2);
        dual c2 = dscale(gm1, dsub(Hr, hq2));
        if (!(c2.v > 0.0)) { st = ORC_ENONPHYS; goto done; }
        dual c = dsqrt(c2);
        dual k = ddiv(D(gm1), c2);
        dual hk = dscale(0.5, k);
        dual hq = dmul(hk, q2);
        dual uic = ddiv(u, c);
        dual ic = ddiv(D(1.0), c);
        dual ku = dmul(k, u);
        dual uc = dmul(u, c);
        dual Lm[3][3] = {
            {dscale(0.5, dadd(hq, uic)), dscale(-0.5, dadd(ku, ic)), hk},
            {dsub(D(1.0), hq), ku, dscale(-1.0, k)},
            {dscale(0.5, dsub(hq, uic)), dscale(-0.5, dsub(ku, ic)), hk},
        };
        dual Rm[3][3] = {
            {D(1.0), D(1.0), D(1.0)},
            {dsub(u, c), u, dadd(u, c)},
            {dsub(Hr, uc), hq2, dadd(Hr, uc)},
        };
        dual what[3];
        for (int q = 0; q < 3; ++q) {
            for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                wp[i] = ddot(Lm[q], &Gp[i * 3], 3);
                wm[i] = ddot(Lm[q], &Gm[i * 3], 3);
            }
            int kp = idx[(f * 3 + q) * 2 + 0], km = idx[(f * 3 + q) * 2 + 1];
            if (kp >= T->ncand || km >= T->ncand) { st = ORC_EINVAL; goto done; }
            dual hp = recon_frozen(T, wp, j, +1, kp);
            dual hm = recon_frozen(T, wm, j, -1, km);
            what[q] = dadd(hp, hm);
        }
        for (int v = 0; v < 3; ++v) Fh[f * 3 + v] = ddot(Rm[v], what, 3);
    }
    for (int v = 0; v < 3; ++v)
        for (long i = 0; i < n; ++i) {
            dual d = dsub(Fh[(i + 1) * 3 + v], Fh[i * 3 + v]);
            L[v * n + i] = -(d.v * ih);
            if (dL) dL[v * n + i] = -(d.d * ih);
        }
done:
    free(Gp); free(Gm); free(un); free(H); free(sq); free(wp); free(wm); free(Fh);
    return st;
}
#endif /* !ORC_QUAD */
