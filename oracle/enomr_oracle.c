/*
 * CPU oracle for the ENO-MR finite-difference scheme (H. Shen, arXiv 2311.15504).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * table with the GPU library: the stencil coefficients arrive as arguments,
 * computed in exact rational arithmetic by oracle/coeffs.py.
 *
 * Everything is FP64.  Built with -ffp-contract=off: every operation is rounded
 * separately, except where fma() is written out.  The evaluation order of each
 * formula is part of the specification (the paper leaves it open); the GPU
 * kernels follow the same order so that stencil choices agree bit for bit.
 *
 *   - dot products (fluxes, the full stencil's IS, R w-hat): first term a
 *     plain product, then fma() terms, in ascending physical cell (or
 *     component) order;
 *   - projections L G: the same chain from the last component to the first
 *     (rows u-c and u+c then share their last two terms);
 *   - the full stencil of a characteristic field (candidate 0): its indicator
 *     and flux are the projection of the stencil sums of the split fluxes,
 *     l_k.(sum_l b_l G_l) and l_k.(sum_l a_l G_l), each component's sum in
 *     ascending cell order (the same values as sum_l b_l (l_k.G_l) in exact
 *     arithmetic, since the projection is linear);
 *   - IS of every other candidate: the (m+n)-th undivided difference of its
 *     cells in ascending order, by repeated differencing f_{i+1} - f_i;
 *   - IS0 second differences: (f_c - 2 f_{c-1}) + f_{c-2};
 *   - one reciprocal per cell (1/rho) and per face (1/(sqrt(rho_L)+sqrt(rho_R)))
 *     multiplies instead of repeated divisions.
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
 *     a field-wise reading of the maximum of Eq. (LF_Flux_Split);
 *     w+-_k = (l_k.F +- alpha_k l_k.U) / 2, each product l_k.x by the
 *     projection chain, then t = alpha_k (l_k.U), w+- = 0.5 (l_k.F +- t);
 *   gravity: the source g [0, 0, rho, rho v] of the Rayleigh-Taylor problem
 *     (Sec. 4.4) added to the 2D right-hand side after the two sweeps.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Operation counter                                                          */
/* ------------------------------------------------------------------------ */

/*
 * Algorithmic operation count of the Euler operator, taken as the method's
 * steps run (the early exit of Step 3.1 included): FP64 flops with fma = 2;
 * add, sub, mul, div, sqrt, min, max and compare = 1; |x|, negation and
 * products or sums with a structural 0 or 1 of the eigenvectors are free.
 * A shared subexpression counts once (the last two terms of the u-c and u+c
 * rows of L, E + p of a cell).  The indicators of the candidates after a
 * failed full stencil count as the cheaper of two ways to obtain them up to
 * the accepted candidate: one b_l chain per candidate scanned, or one
 * difference table of the window ((2r-2)(2r-1)/2 - 1 subtractions) with one
 * compare per candidate.  The wave speeds, alpha and dt (a separate step) and
 * the RK stage combination are not part of the operator count.
 */
static double g_ops;
static int g_counting;

void orc_ops_begin(void) { g_ops = 0.0; g_counting = 1; }
double orc_ops_end(void) { g_counting = 0; return g_ops; }
#define OPS(n) do { if (g_counting) g_ops += (double)(n); } while (0)

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
    double a[ORC_MAXC][ORC_MAXW];   /* a[c][l+m], l = -m..n */
    double b[ORC_MAXC][ORC_MAXW];   /* b[c][l+m] */
} orc_table;

orc_table *orc_table_new(int order, int ncand, const int *mn, const double *a, const double *b)
{
    if (ncand < 1 || ncand > ORC_MAXC) return NULL;
    orc_table *t = (orc_table *)calloc(1, sizeof(orc_table));
    if (!t) return NULL;
    t->order = order;
    t->r = (order + 1) / 2;
    t->ncand = ncand;
    for (int c = 0; c < ncand; ++c) {
        t->m[c] = mn[2 * c];
        t->n[c] = mn[2 * c + 1];
        for (int l = 0; l < ORC_MAXW; ++l) {
            t->a[c][l] = a[c * ORC_MAXW + l];
            t->b[c][l] = b[c * ORC_MAXW + l];
        }
    }
    return t;
}

void orc_table_free(orc_table *t) { free(t); }

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
static double stencil_dot(const double *coef, int m, int n, const double *f, long c, int s)
{
    /* cells covered: offsets -m..n; ascending cell order means offsets
       ascending for s = +1 and descending for s = -1. */
    int l0 = (s > 0) ? -m : n;
    int dl = (s > 0) ? 1 : -1;
    int cnt = m + n + 1;
    int l = l0;
    double acc = coef[l + m] * FR(l);
    for (int k = 1; k < cnt; ++k) {
        l += dl;
        acc = fma(coef[l + m], FR(l), acc);
    }
    return acc;
}

/*
 * The d-th undivided difference of f at cells first .. first+d (ascending):
 * d rounds of replacing neighbours by f_{i+1} - f_i.  Eq. (CurrentIS) defines
 * IS as h^{m+n} times the (m+n)-th derivative of the stencil's polynomial,
 * which is this difference; the b_l of Table ISCoe are its binomial expansion.
 */
static double undivided_difference(const double *f, long first, int d)
{
    double t[ORC_MAXW];
    for (int i = 0; i <= d; ++i) t[i] = f[first + i];
    for (int lev = 1; lev <= d; ++lev)
        for (int i = 0; i + lev <= d; ++i) t[i] = t[i + 1] - t[i];
    return t[0];
}

/*
 * The full stencil (candidate 0) of a characteristic field, evaluated by the
 * caller: is_sum = l_k.(sum b_l G_l) (the indicator before |.|), flux =
 * l_k.(sum a_l G_l), and the operations the field's window projection costs
 * when the reconstruction has to go past candidate 0.
 */
typedef struct {
    double is_sum, flux, fallback_ops;
} full_stencil;

/*
 * Reconstruct f-hat at face j+1/2 from cell values f (indexable from
 * j-r+1 to j+r).  sign = +1: f^+ (upwind on the left); sign = -1: f^-.
 * Writes the chosen candidate's position in the candidate list to *idx.
 * pre (optional): candidate 0's indicator and flux, already evaluated.
 */
static double recon_face(const orc_table *T, const double *f, long j, int sign, int *idx,
                         const full_stencil *pre)
{
    const int s = sign > 0 ? 1 : -1;
    const long c = sign > 0 ? j : j + 1;

    /* Step 1: baseline indicator IS0 = min(IS_L, IS_R), Eq. (Baseline_IS). */
    double f0 = FR(0), fm1 = FR(-1), fm2 = FR(-2), fp1 = FR(1), fp2 = FR(2);
    double isl = fmax(fabs(f0 - fm1), fabs((f0 - 2.0 * fm1) + fm2));
    double isr = fmax(fabs(f0 - fp1), fabs((f0 - 2.0 * fp1) + fp2));
    double is0 = fmin(isl, isr);
    OPS(11);   /* two sides of (sub, mul, sub, add, max), then min */

    /* Step 2: IS of every candidate, Eqs. (CurrentIS), (ISCoe): for the full
       stencil |sum b_l f_{j+l}|, for the others the undivided difference over
       the stencil's cells (leftmost physical cell c-m for f^+, c-n for f^-).
       (The paper only needs them up to the first accepted one; computing all of
       them and then scanning gives the same choice.) */
    double is[ORC_MAXC];
    for (int k = 0; k < T->ncand; ++k) {
        const int m = T->m[k], n = T->n[k];
        if (m >= 1 && n >= 1)
            is[k] = k == 0 ? fabs(pre ? pre->is_sum : stencil_dot(T->b[k], m, n, f, c, s))
                           : fabs(undivided_difference(f, s > 0 ? c - m : c - n, m + n));
        else
            is[k] = 0.0;
    }

    /* Step 3.1: first candidate in list order with m, n >= 1 and IS < IS0. */
    double scan = 0.0;     /* ops of the b_l chains of candidates 1.. scanned so far */
    int tested = 0;        /* candidates 1.. tested so far */
    const int r = T->r;
    const double table = (double)((2 * r - 2) * (2 * r - 1) / 2 - 1);
    for (int k = 0; k < T->ncand; ++k) {
        if (T->m[k] >= 1 && T->n[k] >= 1) {
            const int d = T->m[k] + T->n[k];
            if (k == 0) OPS(pre ? 1 : 2 * d + 1 + 1);     /* (b_l chain and) compare */
            else { scan += 2 * d + 1 + 1; ++tested; }
            if (is[k] < is0) {
                if (k > 0) OPS(scan < table + tested ? scan : table + tested);
                *idx = k;
                if (k == 0 && pre) return pre->flux;
                OPS(2 * d + 1);                 /* a_l chain */
                return stencil_dot(T->a[k], T->m[k], T->n[k], f, c, s);
            }
            /* past candidate 0: the field's window must be projected */
            if (k == 0 && pre) OPS(pre->fallback_ops);
        }
    }
    OPS(scan < table + tested ? scan : table + tested);
    OPS(7);   /* minmod: two slopes, their product, compare, |.| compare, f0 + mm/2 */

    /* Step 3.2: minmod between S_j^{j+1} and S_{j-1}^j, else S_j^j. */
    double da = fp1 - f0;      /* slope towards the downwind neighbour */
    double db = f0 - fm1;      /* slope towards the upwind neighbour   */
    double mm;
    int pick_m, pick_n;
    if (da * db > 0.0) {
        if (fabs(da) <= fabs(db)) { mm = da; pick_m = 0; pick_n = 1; }
        else { mm = db; pick_m = 1; pick_n = 0; }
    } else {
        mm = 0.0; pick_m = 0; pick_n = 0;
    }
    *idx = T->ncand - 1;
    for (int k = 0; k < T->ncand; ++k)
        if (T->m[k] == pick_m && T->n[k] == pick_n) *idx = k;
    return f0 + 0.5 * mm;
}
#undef FR

/*
 * Bare scalar reconstruction over n faces.  f_with_halo has n + 2r - 1
 * entries; face i lies between array cells i + r - 1 and i + r.
 */
int orc_recon_faces(const orc_table *T, int sign, long n, const double *f_with_halo,
                    double *fhat, uint8_t *idx)
{
    if (!T || n < 0 || (sign != 1 && sign != -1)) return ORC_EINVAL;
    const int r = T->r;
    for (long i = 0; i < n; ++i) {
        int k;
        fhat[i] = recon_face(T, f_with_halo, i + r - 1, sign, &k, NULL);
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

static double scalar_flux(int flux, double a, double u)
{
    return flux == ORC_ADVECTION ? a * u : 0.5 * u * u;
}

/*
 * Global LF split (Eq. LF_Flux_Split) with alpha = max |f'(u)| over the line,
 * then f-hat = f-hat^+ + f-hat^- at faces f = 0..n (face f between cells f-1
 * and f), and du/dt = -(f-hat_{j+1/2} - f-hat_{j-1/2}) / h (Eq. 1DWENOFD).
 * With split == NONE the flux itself is reconstructed as f^+ (Sec. 4.2).
 * idx (optional): 2 entries per face, [+, -].
 */
int orc_scalar_rhs(const orc_table *T, int flux, double a, int split, int bc, long n,
                   double ih, const double *u, double *dudt, uint8_t *idx, double *alpha_out)
{
    if (!T || n < 2) return ORC_EINVAL;
    const long g = T->r + 1;
    const long nn = n + 2 * g;
    double *fp = (double *)malloc(sizeof(double) * nn);
    double *fm = (double *)malloc(sizeof(double) * nn);
    double *fh = (double *)malloc(sizeof(double) * (n + 1));
    if (!fp || !fm || !fh) { free(fp); free(fm); free(fh); return ORC_EINVAL; }

    double alpha = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = flux == ORC_ADVECTION ? fabs(a) : fabs(u[i]);
        if (d > alpha) alpha = d;
    }
    if (alpha_out) *alpha_out = alpha;

    for (long i = 0; i < nn; ++i) {
        double ui = u[map_cell(i - g, n, bc)];
        double fi = scalar_flux(flux, a, ui);
        if (split == ORC_SPLIT_LF) {
            double t = alpha * ui;
            fp[i] = 0.5 * (fi + t);
            fm[i] = 0.5 * (fi - t);
        } else {
            fp[i] = fi;
            fm[i] = 0.0;
        }
    }
    for (long f = 0; f <= n; ++f) {
        long j = f - 1 + g;           /* left cell of face f in the ghosted array */
        int kp, km;
        double hp = recon_face(T, fp, j, +1, &kp, NULL);
        double hm = 0.0;
        km = 0;
        if (split == ORC_SPLIT_LF) hm = recon_face(T, fm, j, -1, &km, NULL);
        fh[f] = hp + hm;
        if (idx) { idx[2 * f] = (uint8_t)kp; idx[2 * f + 1] = (uint8_t)km; }
    }
    for (long i = 0; i < n; ++i) dudt[i] = -((fh[i + 1] - fh[i]) * ih);
    free(fp); free(fm); free(fh);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Euler equations: one line in the face-normal frame                        */
/* ------------------------------------------------------------------------ */

/*
 * A line state holds nv = 3 (rho, m, E) or nv = 4 (rho, m_n, m_t, E)
 * conserved variables, the momentum m_n normal to the faces.
 */
typedef struct {
    double un, ut, p, c, H;
    double F[4];
} cell_prim;

static int primitives(int nv, double gamma, const double *U, cell_prim *q)
{
    double rho = U[0], mn = U[1], mt = nv == 4 ? U[2] : 0.0, E = U[nv - 1];
    double ir = 1.0 / rho;
    double un = mn * ir;
    double ut = nv == 4 ? mt * ir : 0.0;
    double ke = nv == 4 ? 0.5 * (mn * un + mt * ut) : 0.5 * (mn * un);
    double p = (gamma - 1.0) * (E - ke);
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(mn)) return ORC_ENONPHYS;
    q->un = un;
    q->ut = ut;
    q->p = p;
    q->c = sqrt((gamma * p) * ir);
    q->H = (E + p) * ir;
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
 * Roe-averaged eigenvectors at the face between states UL and UR
 * (Sec. 4 preamble).  Fields are ordered (u-c, u, [shear,] u+c); Lm is the
 * inverse of Rm.  Returns nonzero if the averaged sound speed is not real.
 */
static int roe_eigen(int nv, double gamma, const double *UL, const cell_prim *qL,
                     const double *UR, const cell_prim *qR, double Lm[4][4], double Rm[4][4])
{
    double sL = sqrt(UL[0]);
    double sR = sqrt(UR[0]);
    double id = 1.0 / (sL + sR);
    double u = (sL * qL->un + sR * qR->un) * id;
    double v = nv == 4 ? (sL * qL->ut + sR * qR->ut) * id : 0.0;
    double H = (sL * qL->H + sR * qR->H) * id;
    double q2 = nv == 4 ? u * u + v * v : u * u;
    double c2 = (gamma - 1.0) * (H - 0.5 * q2);
    if (!(c2 > 0.0)) return ORC_ENONPHYS;
    double c = sqrt(c2);
    double k = (gamma - 1.0) / c2;
    double ic = 1.0 / c;
    double hq = 0.5 * k * q2;
    double ku = k * u;
    double uic = u * ic;
    double uc = u * c;
    if (nv == 4) {
        double kv = k * v;
        double L[4][4] = {
            {0.5 * (hq + uic), -0.5 * (ku + ic), -0.5 * kv, 0.5 * k},
            {1.0 - hq, ku, kv, -k},
            {-v, 0.0, 1.0, 0.0},
            {0.5 * (hq - uic), -0.5 * (ku - ic), -0.5 * kv, 0.5 * k},
        };
        double R[4][4] = {
            {1.0, 1.0, 0.0, 1.0},
            {u - c, u, 0.0, u + c},
            {v, v, 1.0, v},
            {H - uc, 0.5 * q2, v, H + uc},
        };
        memcpy(Lm, L, sizeof(L));
        memcpy(Rm, R, sizeof(R));
    } else {
        double L[4][4] = {
            {0.5 * (hq + uic), -0.5 * (ku + ic), 0.5 * k, 0.0},
            {1.0 - hq, ku, -k, 0.0},
            {0.5 * (hq - uic), -0.5 * (ku - ic), 0.5 * k, 0.0},
            {0.0, 0.0, 0.0, 0.0},
        };
        double R[4][4] = {
            {1.0, 1.0, 1.0, 0.0},
            {u - c, u, u + c, 0.0},
            {H - uc, 0.5 * q2, H + uc, 0.0},
            {0.0, 0.0, 0.0, 0.0},
        };
        memcpy(Lm, L, sizeof(L));
        memcpy(Rm, R, sizeof(R));
    }
    return ORC_OK;
}

/* Exported for the eigenvector tests: L and R at the Roe state of UL, UR. */
int orc_roe_eigen(int nv, double gamma, const double *UL, const double *UR, double *Lout, double *Rout)
{
    cell_prim qL, qR;
    if (primitives(nv, gamma, UL, &qL) || primitives(nv, gamma, UR, &qR)) return ORC_ENONPHYS;
    double Lm[4][4], Rm[4][4];
    int st = roe_eigen(nv, gamma, UL, &qL, UR, &qR, Lm, Rm);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            Lout[i * nv + j] = Lm[i][j];
            Rout[i * nv + j] = Rm[i][j];
        }
    return st;
}

static double row_dot(const double *row, const double *x, int nv)
{
    double acc = row[0] * x[0];
    for (int i = 1; i < nv; ++i) acc = fma(row[i], x[i], acc);
    return acc;
}

/* A row of L applied to a split flux: the chain from the last component down. */
static double project_dot(const double *row, const double *x, int nv)
{
    double acc = row[nv - 1] * x[nv - 1];
    for (int i = nv - 2; i >= 0; --i) acc = fma(row[i], x[i], acc);
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

static const euler_var k_default_var = {0, 0};

/*
 * Numerical fluxes at faces f = 0..n of one line (face f between cells f-1
 * and f).  Ul is [nv][n] in the face-normal frame.  Fhat is [n+1][nv].
 * alpha: the line's alpha, or its three per-field alphas (var.per_field).
 * idx (optional) holds nv*2 entries per face: [(field)*2 + (0:+, 1:-)].
 */
static int euler_line_fluxes(const orc_table *T, int nv, double gamma, int bc, long n,
                             const double *Ul, const double *alpha, euler_var var, double *Fhat,
                             uint8_t *idx)
{
    const long g = T->r + 1;
    const long nn = n + 2 * g;
    double *U = (double *)malloc(sizeof(double) * nn * nv);
    double *Gp = (double *)malloc(sizeof(double) * nn * nv);
    double *Gm = (double *)malloc(sizeof(double) * nn * nv);
    cell_prim *Q = (cell_prim *)malloc(sizeof(cell_prim) * nn);
    double *wp = (double *)malloc(sizeof(double) * nn);
    double *wm = (double *)malloc(sizeof(double) * nn);
    int st = ORC_OK;
    const int counting = g_counting;
    /* the operation counter covers the default operator only */
    if (var.componentwise || var.per_field) g_counting = 0;
    if (!U || !Gp || !Gm || !Q || !wp || !wm) { st = ORC_EINVAL; goto done; }

    /* Ghosted line, primitive quantities and the LF split G = (F +- alpha U)/2
       (with per-field alphas the split is taken after the projection). */
    for (long i = 0; i < nn; ++i) {
        long src = map_cell(i - g, n, bc);
        for (int v = 0; v < nv; ++v) U[i * nv + v] = Ul[v * n + src];
        if ((st = primitives(nv, gamma, &U[i * nv], &Q[i]))) goto done;
        for (int v = 0; v < nv; ++v) {
            double t = alpha[0] * U[i * nv + v];
            Gp[i * nv + v] = 0.5 * (Q[i].F[v] + t);
            Gm[i * nv + v] = 0.5 * (Q[i].F[v] - t);
        }
        /* once per cell of the line (ghosts are copies): 1/rho, velocities,
           kinetic energy, p, E + p, H, fluxes, the split (5 per component) and
           sqrt(rho) of the Roe average */
        if (i >= g && i < g + n) OPS(nv == 4 ? 36 : 27);
    }

    for (long f = 0; f <= n; ++f) {
        long j = f - 1 + g;      /* left cell of the face in the ghosted line */
        double Lm[4][4], Rm[4][4];
        /* a periodic line's face n is its face 0 again: counted once */
        g_counting = counting && !var.componentwise && !var.per_field && !(bc == ORC_PERIODIC && f == n);
        if (var.componentwise) {
            /* G+- of each component reconstructed as they are */
            for (int k = 0; k < nv; ++k) {
                for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                    wp[i] = Gp[i * nv + k];
                    wm[i] = Gm[i * nv + k];
                }
                int kp, km;
                double hp = recon_face(T, wp, j, +1, &kp, NULL);
                double hm = recon_face(T, wm, j, -1, &km, NULL);
                Fhat[f * nv + k] = hp + hm;
                if (idx) {
                    idx[(f * nv + k) * 2 + 0] = (uint8_t)kp;
                    idx[(f * nv + k) * 2 + 1] = (uint8_t)km;
                }
            }
            continue;
        }
        if ((st = roe_eigen(nv, gamma, &U[j * nv], &Q[j], &U[(j + 1) * nv], &Q[j + 1], Lm, Rm)))
            goto done;
        /* Roe average and the entries of L and R used below (0.5 q^2 is shared
           by c^2 and R) */
        OPS(nv == 4 ? 44 : 36);
        const int W = 2 * T->r - 1;
        const double proj = nv == 4 ? 20 : 14;
        /* the full stencil of every field by linearity: per sign the a_l and
           b_l sums of each split-flux component, then their projections */
        full_stencil pre[4][2];
        if (!var.per_field) {
            double A[2][4], B[2][4];
            for (int sg = 0; sg < 2; ++sg) {
                const double *G = sg == 0 ? Gp : Gm;
                const long cc = sg == 0 ? j : j + 1;
                const int ss = sg == 0 ? 1 : -1;
                for (int v = 0; v < nv; ++v) {
                    for (long i = j - T->r + 1; i <= j + T->r; ++i) wp[i] = G[i * nv + v];
                    A[sg][v] = stencil_dot(T->a[0], T->m[0], T->n[0], wp, cc, ss);
                    B[sg][v] = stencil_dot(T->b[0], T->m[0], T->n[0], wp, cc, ss);
                }
            }
            for (int k = 0; k < nv; ++k)
                for (int sg = 0; sg < 2; ++sg) {
                    pre[k][sg].is_sum = project_dot(Lm[k], B[sg], nv);
                    pre[k][sg].flux = project_dot(Lm[k], A[sg], nv);
                    /* one row of L over the window cells beyond the five
                       centre cells IS0 uses: u-c, u+c and u rows 3 fma and a
                       product (2 fma and a product in 1D), the shear row one fma */
                    pre[k][sg].fallback_ops = (W - 5) * (nv == 4 ? (k == 2 ? 2 : 7) : 5);
                }
            /* per sign: L G at the five centre cells, 2 nv chains of W terms,
               and the projection of the a_l and b_l sums */
            OPS(2 * (5 * proj + 2 * nv * (2 * W - 1) + 2 * proj));
        } else {
            /* L F and L U over each window (2r-1 cells per sign) */
            OPS(2 * W * proj);
        }
        double what[4];
        for (int k = 0; k < nv; ++k) {
            /* characteristic field k of the split fluxes over the face's window */
            if (var.per_field) {
                const double ak = alpha[field_speed(nv, k)];
                for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                    double pf = project_dot(Lm[k], Q[i].F, nv);
                    double t = ak * project_dot(Lm[k], &U[i * nv], nv);
                    wp[i] = 0.5 * (pf + t);
                    wm[i] = 0.5 * (pf - t);
                }
            } else {
                for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                    wp[i] = project_dot(Lm[k], &Gp[i * nv], nv);
                    wm[i] = project_dot(Lm[k], &Gm[i * nv], nv);
                }
            }
            int kp, km;
            double hp = recon_face(T, wp, j, +1, &kp, var.per_field ? NULL : &pre[k][0]);
            double hm = recon_face(T, wm, j, -1, &km, var.per_field ? NULL : &pre[k][1]);
            what[k] = hp + hm;
            if (idx) {
                idx[(f * nv + k) * 2 + 0] = (uint8_t)kp;
                idx[(f * nv + k) * 2 + 1] = (uint8_t)km;
            }
        }
        /* back to conserved components: F-hat = R w-hat (w-hat+ + w-hat- first) */
        for (int v = 0; v < nv; ++v) Fhat[f * nv + v] = row_dot(Rm[v], what, nv);
        OPS(nv == 4 ? 4 + 20 : 3 + 12);
    }
done:
    g_counting = counting;
    free(U); free(Gp); free(Gm); free(Q); free(wp); free(wm);
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
 */
int orc_euler1d_rhs_var(const orc_table *T, double gamma, int bc, long n, double ih,
                        const double *U, double *dUdt, uint8_t *idx, double *alpha_out,
                        int componentwise, int per_field)
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
    st = euler_line_fluxes(T, 3, gamma, bc, n, U, alpha, var, Fh, idx);
    if (!st)
        for (int v = 0; v < 3; ++v)
            for (long i = 0; i < n; ++i)
                dUdt[v * n + i] = -((Fh[(i + 1) * 3 + v] - Fh[i * 3 + v]) * ih);
    free(Fh);
    return st;
}

/* 1D Euler right-hand side L(U), U and dUdt laid out [3][n]. */
int orc_euler1d_rhs(const orc_table *T, double gamma, int bc, long n, double ih,
                    const double *U, double *dUdt, uint8_t *idx, double *alpha_out)
{
    return orc_euler1d_rhs_var(T, gamma, bc, n, ih, U, dUdt, idx, alpha_out, 0, 0);
}

/*
 * 2D Euler right-hand side, dimension by dimension (Sec. 2.1):
 * dU/dt = -(F_{i+1/2} - F_{i-1/2})/hx - (G_{j+1/2} - G_{j-1/2})/hy.
 * U, dUdt: [4][ny][nx].  x-lines use (rho, m, n, E); y-lines the permuted
 * state (rho, n, m, E) so that the same normal-frame formulas apply.
 * idx_x (optional): [ny][nx+1][4][2]; idx_y (optional): [ny+1][nx][4][2].
 * alpha_x[ny], alpha_y[nx] (optional) receive the per-line alphas; with
 * per_field, alpha_x[3][ny] and alpha_y[3][nx] the per-field ones.
 * componentwise, per_field (not both): the variants of the header comment;
 * gravity g != 0 adds the source g [0, 0, rho, rho v] to the result.
 */
int orc_euler2d_rhs_var(const orc_table *T, double gamma, int bcx, int bcy, long nx, long ny,
                        double ihx, double ihy, const double *U, double *dUdt,
                        uint8_t *idx_x, uint8_t *idx_y, double *alpha_x, double *alpha_y,
                        int componentwise, int per_field, double gravity)
{
    if (!T || nx < 2 || ny < 2 || (componentwise && per_field)) return ORC_EINVAL;
    euler_var var = {componentwise != 0, per_field != 0};
    const int na = per_field ? 3 : 1;
    const long plane = nx * ny;
    long nmax = nx > ny ? nx : ny;
    double *line = (double *)malloc(sizeof(double) * 4 * nmax);
    double *Fh = (double *)malloc(sizeof(double) * 4 * (nmax + 1));
    uint8_t *idl = (uint8_t *)malloc(8 * (nmax + 1));
    double *Lx = (double *)malloc(sizeof(double) * 4 * plane);
    int st = ORC_OK;
    if (!line || !Fh || !idl || !Lx) { st = ORC_EINVAL; goto done; }

    /* x sweep */
    for (long y = 0; y < ny; ++y) {
        for (int v = 0; v < 4; ++v)
            for (long x = 0; x < nx; ++x) line[v * nx + x] = U[v * plane + y * nx + x];
        double alpha[3];
        if ((st = line_alphas(4, gamma, nx, line, var, alpha))) goto done;
        if (alpha_x)
            for (int k = 0; k < na; ++k) alpha_x[k * ny + y] = alpha[k];
        if ((st = euler_line_fluxes(T, 4, gamma, bcx, nx, line, alpha, var, Fh, idx_x ? idl : NULL)))
            goto done;
        if (idx_x) memcpy(idx_x + (size_t)y * (nx + 1) * 8, idl, (size_t)(nx + 1) * 8);
        for (int v = 0; v < 4; ++v)
            for (long x = 0; x < nx; ++x)
                Lx[v * plane + y * nx + x] = -((Fh[(x + 1) * 4 + v] - Fh[x * 4 + v]) * ihx);
        OPS(8 * nx);
    }
    /* y sweep on the permuted state, then combine */
    static const int perm[4] = {0, 2, 1, 3};
    for (long x = 0; x < nx; ++x) {
        for (int v = 0; v < 4; ++v)
            for (long y = 0; y < ny; ++y) line[v * ny + y] = U[perm[v] * plane + y * nx + x];
        double alpha[3];
        if ((st = line_alphas(4, gamma, ny, line, var, alpha))) goto done;
        if (alpha_y)
            for (int k = 0; k < na; ++k) alpha_y[k * nx + x] = alpha[k];
        if ((st = euler_line_fluxes(T, 4, gamma, bcy, ny, line, alpha, var, Fh, idx_y ? idl : NULL)))
            goto done;
        if (idx_y)
            for (long f = 0; f <= ny; ++f) memcpy(idx_y + ((size_t)f * nx + x) * 8, idl + f * 8, 8);
        for (int v = 0; v < 4; ++v)
            for (long y = 0; y < ny; ++y) {
                int cv = perm[v];
                double ly = -((Fh[(y + 1) * 4 + v] - Fh[y * 4 + v]) * ihy);
                dUdt[cv * plane + y * nx + x] = Lx[cv * plane + y * nx + x] + ly;
            }
        OPS(12 * ny);
    }
    /* source term of the Rayleigh-Taylor problem (Sec. 4.4): rho g in the
       y-momentum, rho v g in the energy equation */
    if (gravity != 0.0)
        for (long i = 0; i < plane; ++i) {
            dUdt[2 * plane + i] = dUdt[2 * plane + i] + gravity * U[i];
            dUdt[3 * plane + i] = dUdt[3 * plane + i] + gravity * U[2 * plane + i];
        }
done:
    free(line); free(Fh); free(idl); free(Lx);
    return st;
}

int orc_euler2d_rhs(const orc_table *T, double gamma, int bcx, int bcy, long nx, long ny,
                    double ihx, double ihy, const double *U, double *dUdt,
                    uint8_t *idx_x, uint8_t *idx_y, double *alpha_x, double *alpha_y)
{
    return orc_euler2d_rhs_var(T, gamma, bcx, bcy, nx, ny, ihx, ihy, U, dUdt, idx_x, idx_y, alpha_x,
                               alpha_y, 0, 0, 0.0);
}

/*
 * L(U) at selected cells of a 2D grid only (for spot checks of large runs).
 * cells: ncell (x, y) pairs; out: [ncell][4].  Each cell needs its row's and
 * column's alpha, computed here over the whole line.
 */
int orc_euler2d_rhs_cells(const orc_table *T, double gamma, int bcx, int bcy, long nx, long ny,
                          double ihx, double ihy, const double *U, long ncell, const long *cells,
                          double *out)
{
    if (!T || nx < 2 || ny < 2) return ORC_EINVAL;
    const long plane = nx * ny;
    const long w = T->r + 2;   /* cells each side needed by two faces */
    long nmax = nx > ny ? nx : ny;
    double *line = (double *)malloc(sizeof(double) * 4 * nmax);
    double *seg = (double *)malloc(sizeof(double) * 4 * (2 * w + 1));
    double *Fh = (double *)malloc(sizeof(double) * 4 * (2 * w + 2));
    int st = ORC_OK;
    static const int perm[4] = {0, 2, 1, 3};
    if (!line || !seg || !Fh) { st = ORC_EINVAL; goto done; }
    for (long q = 0; q < ncell; ++q) {
        long cx = cells[2 * q], cy = cells[2 * q + 1];
        double res[4];
        for (int dir = 0; dir < 2; ++dir) {
            long n = dir == 0 ? nx : ny;
            long ci = dir == 0 ? cx : cy;
            int bc = dir == 0 ? bcx : bcy;
            for (int v = 0; v < 4; ++v)
                for (long i = 0; i < n; ++i) {
                    long gx = dir == 0 ? i : cx, gy = dir == 0 ? cy : i;
                    int sv = dir == 0 ? v : perm[v];
                    line[v * n + i] = U[sv * plane + gy * nx + gx];
                }
            double alpha[3] = {0.0, 0.0, 0.0};
            if ((st = line_alpha(4, gamma, n, line, &alpha[0]))) goto done;
            /* fluxes at the cell's two faces: evaluate on the whole line (plain) */
            double *Fl = (double *)malloc(sizeof(double) * 4 * (n + 1));
            if (!Fl) { st = ORC_EINVAL; goto done; }
            st = euler_line_fluxes(T, 4, gamma, bc, n, line, alpha, k_default_var, Fl, NULL);
            if (st) { free(Fl); goto done; }
            for (int v = 0; v < 4; ++v) {
                double ih = dir == 0 ? ihx : ihy;
                double d = -((Fl[(ci + 1) * 4 + v] - Fl[ci * 4 + v]) * ih);
                int cv = dir == 0 ? v : perm[v];
                if (dir == 0) res[cv] = d;
                else res[cv] = res[cv] + d;
            }
            free(Fl);
        }
        for (int v = 0; v < 4; ++v) out[q * 4 + v] = res[v];
    }
done:
    free(line); free(seg); free(Fh);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Time step and Runge-Kutta updates                                         */
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

/*
 * SSP-RK3 stage combination (Eq. TVD3rdRK), elementwise over n values:
 *   stage 1: out = us + dt L
 *   stage 2: out = 3/4 un + 1/4 (us + dt L)
 *   stage 3: out = 1/3 un + 2/3 (us + dt L)
 */
void orc_ssprk3_combine(int stage, long n, const double *un, const double *us, const double *L,
                        double dt, double *out)
{
    const double c13 = 1.0 / 3.0, c23 = 2.0 / 3.0;
    for (long i = 0; i < n; ++i) {
        double e = us[i] + dt * L[i];
        if (stage == 1) out[i] = e;
        else if (stage == 2) out[i] = 0.75 * un[i] + 0.25 * e;
        else out[i] = c13 * un[i] + c23 * e;
    }
}

/*
 * Linear SSP-RK(m, m-1) step for a scalar line (Eq. lSSPRK):
 * u^(s) = u^(s-1) + dt/2 L(u^(s-1)), s = 1..m-1, and
 * u^{n+1} = sum_{k<m-1} a_k u^(k) + a_{m-1} (u^(m-1) + dt/2 L(u^(m-1))).
 * coef holds a_0..a_{m-1} (computed exactly by the caller, Eq. lSSPRK_Coe).
 */
int orc_scalar_lssp_run(const orc_table *T, int flux, double a, int split, int bc, long n,
                        double ih, double dt, long nsteps, int m, const double *coef, double *u)
{
    if (m < 2 || m > 32) return ORC_EINVAL;
    double *stages = (double *)malloc(sizeof(double) * n * m);
    double *L = (double *)malloc(sizeof(double) * n);
    double *acc = (double *)malloc(sizeof(double) * n);
    int st = ORC_OK;
    if (!stages || !L || !acc) { st = ORC_EINVAL; goto done; }
    const double hdt = 0.5 * dt;
    for (long step = 0; step < nsteps; ++step) {
        memcpy(stages, u, sizeof(double) * n);
        for (int s = 1; s < m; ++s) {
            if ((st = orc_scalar_rhs(T, flux, a, split, bc, n, ih, stages + (s - 1) * n, L, NULL, NULL)))
                goto done;
            for (long i = 0; i < n; ++i) stages[s * n + i] = stages[(s - 1) * n + i] + hdt * L[i];
        }
        if ((st = orc_scalar_rhs(T, flux, a, split, bc, n, ih, stages + (m - 1) * n, L, NULL, NULL)))
            goto done;
        for (long i = 0; i < n; ++i) acc[i] = 0.0;
        for (int k = 0; k < m - 1; ++k)
            for (long i = 0; i < n; ++i) acc[i] = acc[i] + coef[k] * stages[k * n + i];
        for (long i = 0; i < n; ++i)
            u[i] = acc[i] + coef[m - 1] * (stages[(m - 1) * n + i] + hdt * L[i]);
    }
done:
    free(stages); free(L); free(acc);
    return st;
}

/*
 * SSP-RK3 run of a scalar line with a fixed step dt; the last step is cut so
 * that the run ends exactly at t_end (if t_end > 0, else nsteps steps).
 */
int orc_scalar_ssprk3_run(const orc_table *T, int flux, double a, int split, int bc, long n,
                          double ih, double dt, double t_end, long nsteps, double *u)
{
    double *un = (double *)malloc(sizeof(double) * n);
    double *us = (double *)malloc(sizeof(double) * n);
    double *L = (double *)malloc(sizeof(double) * n);
    int st = ORC_OK;
    if (!un || !us || !L) { st = ORC_EINVAL; goto done; }
    double t = 0.0;
    for (long step = 0; t_end > 0.0 ? t < t_end : step < nsteps; ++step) {
        double h = dt;
        if (t_end > 0.0 && t + h > t_end) h = t_end - t;
        memcpy(un, u, sizeof(double) * n);
        memcpy(us, u, sizeof(double) * n);
        for (int s = 1; s <= 3; ++s) {
            if ((st = orc_scalar_rhs(T, flux, a, split, bc, n, ih, us, L, NULL, NULL))) goto done;
            orc_ssprk3_combine(s, n, un, us, L, h, us);
        }
        memcpy(u, us, sizeof(double) * n);
        t = t + h;
    }
done:
    free(un); free(us); free(L);
    return st;
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
static dual dinv(dual a) { dual r = {1.0 / a.v, -a.d / (a.v * a.v)}; return r; }
static dual dsqrt(dual a) { double s = sqrt(a.v); dual r = {s, a.d / (2.0 * s)}; return r; }
static dual dfma(dual a, dual b, dual c) { dual r = {fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d}; return r; }

/* chain acc = c[0] x[0]; acc = fma(c[i], x[i], acc) */
static dual ddot(const dual *c, const dual *x, int n)
{
    dual acc = dmul(c[0], x[0]);
    for (int i = 1; i < n; ++i) acc = dfma(c[i], x[i], acc);
    return acc;
}

/* project_dot() in dual arithmetic */
static dual dproject(const dual *c, const dual *x, int n)
{
    dual acc = dmul(c[n - 1], x[n - 1]);
    for (int i = n - 2; i >= 0; --i) acc = dfma(c[i], x[i], acc);
    return acc;
}

/* recon of one window with a frozen choice k (frame as in recon_face) */
static dual recon_frozen(const orc_table *T, const dual *f, long j, int sign, int k)
{
    const int s = sign > 0 ? 1 : -1;
    const long c = sign > 0 ? j : j + 1;
#define FD(l) (f[c + (long)s * (l)])
    const int m = T->m[k], n = T->n[k];
    if (m >= 1 && n >= 1) {
        int l0 = (s > 0) ? -m : n, dl = (s > 0) ? 1 : -1, l = l0;
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

/* The full stencil's a_l sum of component v of the split fluxes G ([cell][3]),
   frame and cell order as in recon_face (dual arithmetic). */
static dual full_sum_frozen(const orc_table *T, const dual *G, long j, int sign, int v)
{
    const int s = sign > 0 ? 1 : -1;
    const long c = sign > 0 ? j : j + 1;
    const int m = T->m[0], n = T->n[0];
    int l = (s > 0) ? -m : n;
    const int dl = (s > 0) ? 1 : -1;
    dual acc = dmul(D(T->a[0][l + m]), G[(c + (long)s * l) * 3 + v]);
    for (int q = 1; q < m + n + 1; ++q) {
        l += dl;
        acc = dfma(D(T->a[0][l + m]), G[(c + (long)s * l) * 3 + v], acc);
    }
    return acc;
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
    dual *Uc = (dual *)malloc(sizeof(dual) * nn * 3);
    dual *Gp = (dual *)malloc(sizeof(dual) * nn * 3);
    dual *Gm = (dual *)malloc(sizeof(dual) * nn * 3);
    dual *un = (dual *)malloc(sizeof(dual) * nn);
    dual *H = (dual *)malloc(sizeof(dual) * nn);
    dual *sq = (dual *)malloc(sizeof(dual) * nn);
    dual *wp = (dual *)malloc(sizeof(dual) * nn);
    dual *wm = (dual *)malloc(sizeof(dual) * nn);
    dual *Fh = (dual *)malloc(sizeof(dual) * (n + 1) * 3);
    int st = ORC_OK;
    if (!Uc || !Gp || !Gm || !un || !H || !sq || !wp || !wm || !Fh) { st = ORC_EINVAL; goto done; }
    for (long i = 0; i < nn; ++i) {
        long src = map_cell(i - g, n, bc);
        dual rho = {U[src], dU ? dU[src] : 0.0};
        dual mn = {U[n + src], dU ? dU[n + src] : 0.0};
        dual E = {U[2 * n + src], dU ? dU[2 * n + src] : 0.0};
        dual ir = dinv(rho);
        dual u = dmul(mn, ir);
        dual ke = dscale(0.5, dmul(mn, u));
        dual p = dscale(gm1, dsub(E, ke));
        if (!(rho.v > 0.0) || !(p.v > 0.0)) { st = ORC_ENONPHYS; goto done; }
        dual F[3] = {mn, dadd(dmul(mn, u), p), dmul(dadd(E, p), u)};
        dual Ucs[3] = {rho, mn, E};
        for (int v = 0; v < 3; ++v) {
            dual t = dscale(alpha, Ucs[v]);
            Uc[i * 3 + v] = Ucs[v];
            Gp[i * 3 + v] = dscale(0.5, dadd(F[v], t));
            Gm[i * 3 + v] = dscale(0.5, dsub(F[v], t));
        }
        un[i] = u;
        H[i] = dmul(dadd(E, p), ir);
        sq[i] = dsqrt(rho);
    }
    for (long f = 0; f <= n; ++f) {
        long j = f - 1 + g;
        /* Roe eigenvectors, the formulas of roe_eigen() in dual arithmetic */
        dual id = dinv(dadd(sq[j], sq[j + 1]));
        dual u = dmul(dadd(dmul(sq[j], un[j]), dmul(sq[j + 1], un[j + 1])), id);
        dual Hr = dmul(dadd(dmul(sq[j], H[j]), dmul(sq[j + 1], H[j + 1])), id);
        dual q2 = dmul(u, u);
        dual c2 = dscale(gm1, dsub(Hr, dscale(0.5, q2)));
        if (!(c2.v > 0.0)) { st = ORC_ENONPHYS; goto done; }
        dual c = dsqrt(c2);
        dual k = dscale(gm1, dinv(c2));
        k.v = gm1 / c2.v;                     /* the forward divides once */
        dual ic = dinv(c);
        dual hq = dmul(dscale(0.5, k), q2);
        dual ku = dmul(k, u);
        dual uic = dmul(u, ic);
        dual uc = dmul(u, c);
        dual Lm[3][3] = {
            {dscale(0.5, dadd(hq, uic)), dscale(-0.5, dadd(ku, ic)), dscale(0.5, k)},
            {dsub(D(1.0), hq), ku, dscale(-1.0, k)},
            {dscale(0.5, dsub(hq, uic)), dscale(-0.5, dsub(ku, ic)), dscale(0.5, k)},
        };
        dual Rm[3][3] = {
            {D(1.0), D(1.0), D(1.0)},
            {dsub(u, c), u, dadd(u, c)},
            {dsub(Hr, uc), dscale(0.5, q2), dadd(Hr, uc)},
        };
        /* the full stencil's flux is the projection of the a_l sums (as in
           euler_line_fluxes) */
        dual Ap[3], Am[3];
        for (int v = 0; v < 3; ++v) {
            Ap[v] = full_sum_frozen(T, Gp, j, +1, v);
            Am[v] = full_sum_frozen(T, Gm, j, -1, v);
        }
        dual what[3];
        for (int q = 0; q < 3; ++q) {
            for (long i = j - T->r + 1; i <= j + T->r; ++i) {
                wp[i] = dproject(Lm[q], &Gp[i * 3], 3);
                wm[i] = dproject(Lm[q], &Gm[i * 3], 3);
            }
            int kp = idx[(f * 3 + q) * 2 + 0], km = idx[(f * 3 + q) * 2 + 1];
            if (kp >= T->ncand || km >= T->ncand) { st = ORC_EINVAL; goto done; }
            dual hp = kp == 0 ? dproject(Lm[q], Ap, 3) : recon_frozen(T, wp, j, +1, kp);
            dual hm = km == 0 ? dproject(Lm[q], Am, 3) : recon_frozen(T, wm, j, -1, km);
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
    free(Uc); free(Gp); free(Gm); free(un); free(H); free(sq); free(wp); free(wm); free(Fh);
    return st;
}
