/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * Plain FP64 CPU reference of the pseudopotential LBM with a shaped
 * equation of state.  Loops are written for clarity, not speed: no
 * blocking, no fusion, no reordering beyond what the equations state.
 *
 * Readings taken where the paper is silent, ambiguous or garbled:
 *  R1  Sec. III.D region 2: the printed cubic coefficients (d2 = p_max,
 *      c2 = 0, b2 = 3(p_min-p_max), a2 = 2(p_max-p_min)) only interpolate
 *      the two knots with zero end slopes when the variable runs over a
 *      unit interval, so the cubic is evaluated in
 *      t = (rho-rho_max)/(rho_min-rho_max).
 *  R2  Sec. III.D region 3: the undefined p_2, rho_2 are p_min, rho_min
 *      (mirror of region 1; gives p(rho_min)=p_min with zero slope).
 *  R3  Eq. LiFS: the printed vector is the moment-space source S; it is
 *      applied as M^-1 (I - Lambda/2) S, the same (I - Lambda/2) factor
 *      Eq. GFS carries (at sigma = 0 the two coincide).
 *  R4  Eq. LiFS |F|^2/psi^2 is evaluated literally; at psi = 0 the limit
 *      |F~|^2 with F = psi F~ is used.
 *  R5  Critical temperature from the exact critical point of the EOS
 *      (the paper's Tc ~ 0.3773 a/(bR) is a rounded value).
 *  R6  Raised vapor slope (Sec. III.D): the vapor branch is k_vap times the
 *      base EOS at the same reduced temperature (C-S with a_v at the same
 *      Tr is a_v/a times C-S with a); the liquid branch is the base EOS
 *      plus dP = (k_vap-1) p_sat; Maxwell densities are unchanged.
 *  R7  alpha is taken relative to the base EOS:
 *      p_min = p_sat_new - alpha (p_sat - p_min_base).
 *  R8  Eq. RelaxationTime outside [rho_v, rho_l]: tau is clamped to
 *      [min(tau_v,tau_l), max(tau_v,tau_l)].
 *  R9  Walls (Sec. IV): half-way bounce-back; the solid node one lattice
 *      unit outside the first/last fluid row enters Eq. ShanChenForce with
 *      psi(rho_wall_lo) below and psi(rho_wall_hi) above.
 *  R10 Peng-Robinson is the textbook EOS; its critical point is found the
 *      same way as for C-S (alpha(Tc) = 1).
 *
 * Quadratures: composite Simpson in the variable s = ln(rho), split at the
 * knots of the shaped EOS (Sec. III.A states Simpson's rule).
 *
 * Threads: built with -DOR_OMP -fopenmp, the three node loops of a time step
 * (fields, collision, streaming) are split over rows by OpenMP.  Every node
 * still runs the same arithmetic on the same inputs, and no sum crosses nodes,
 * so the threaded build gives the same bits as the single-threaded one.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef OR_OMP
#include <omp.h>
#define OR_PARALLEL_ROWS _Pragma("omp parallel for schedule(static)")
#define OR_PARALLEL_ROWS_FLAG _Pragma("omp parallel for schedule(static) reduction(|:flag)")
#else
#define OR_PARALLEL_ROWS
#define OR_PARALLEL_ROWS_FLAG
#endif

/* ---------------------------------------------------------------- */
/* D2Q9 (Eq. VelocitySet), weights (Sec. II.A), M (Eq. MatrixMRT)   */
/* ---------------------------------------------------------------- */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double MROWS[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};
static const double CS2 = 1.0 / 3.0;

static int opposite(int i)
{
    for (int k = 0; k < 9; ++k)
        if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
    return -1;
}

/* Gauss-Jordan inverse of the printed M, computed once. */
static double MINV[9][9];
static int minv_ready = 0;
static void build_minv(void)
{
    if (minv_ready) return;
    double A[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c) A[r][c] = c < 9 ? MROWS[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        for (int c = 0; c < 18; ++c) {
            double t = A[col][c];
            A[col][c] = A[piv][c];
            A[piv][c] = t;
        }
        double d = A[col][col];
        for (int c = 0; c < 18; ++c) A[col][c] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == col) continue;
            double m = A[r][col];
            for (int c = 0; c < 18; ++c) A[r][c] -= m * A[col][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) MINV[r][c] = A[r][c + 9];
    minv_ready = 1;
}

void or_matrix(double* M, double* Minv)
{
    build_minv();
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            M[r * 9 + c] = MROWS[r][c];
            Minv[r * 9 + c] = MINV[r][c];
        }
}

/* ---------------------------------------------------------------- */
/* Base equations of state                                          */
/* ---------------------------------------------------------------- */
/* C-S compressibility pieces in eta = b rho / 4 (Eq. CS):
 *   q(eta)   = eta (1+eta+eta^2-eta^3)/(1-eta)^3
 *   q'(eta)  = (1+4eta+4eta^2-4eta^3+eta^4)/(1-eta)^4
 *   q''(eta) = (8+20eta-4eta^2)/(1-eta)^5                      */
static double cs_q1(double e) { return (1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e) / pow(1 - e, 4); }
static double cs_q2(double e) { return (8 + 20 * e - 4 * e * e) / pow(1 - e, 5); }

double or_cs_critical_eta(void)
{
    /* critical point: dp/drho = d2p/drho2 = 0  <=>  q'(eta) = eta q''(eta) */
    double lo = 1e-6, hi = 0.5;
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi);
        double h = cs_q1(mid) - mid * cs_q2(mid);
        if (h > 0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Peng-Robinson in x = b rho:  p = (RT/b) x/(1-x) - (a alpha/b^2) x^2/(1+2x-x^2).
 * Critical point with alpha = 1: B/A = g1(x) = g2(x) with
 *   g1 = 2x(1+x)(1-x)^2/D^2,  g2 = (1-x)^3 d/dx[2x(1+x)/D^2] / 2,  D = 1+2x-x^2. */
static double pr_g1(double x)
{
    double D = 1 + 2 * x - x * x;
    return 2 * x * (1 + x) * (1 - x) * (1 - x) / (D * D);
}
static double pr_g2(double x)
{
    double D = 1 + 2 * x - x * x, Dp = 2 - 2 * x;
    double N = 2 * x + 2 * x * x, Np = 2 + 4 * x;
    double gp = (Np * D - 2 * N * Dp) / (D * D * D);
    return 0.5 * pow(1 - x, 3) * gp;
}
static double pr_critical_ratio(void)
{
    double lo = 0.05, hi = 0.6;
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi);
        double h = pr_g1(mid) - pr_g2(mid);
        double hlo = pr_g1(lo) - pr_g2(lo);
        if ((h > 0) == (hlo > 0)) lo = mid; else hi = mid;
    }
    return pr_g1(0.5 * (lo + hi)); /* Tc = (a/(bR)) * this */
}

static double pr_alpha(const or_eos* e)
{
    double kappa = 0.37464 + 1.54226 * e->omega - 0.26992 * e->omega * e->omega;
    double s = 1.0 + kappa * (1.0 - sqrt(e->T / e->Tc));
    return s * s;
}

double or_base_p(const or_eos* e, double rho)
{
    if (e->base == OR_BASE_CS) {
        double eta = e->b * rho / 4.0;
        double num = 1.0 + eta + eta * eta - eta * eta * eta;
        double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
        return e->scale * (rho * e->R * e->T * num / den - e->a * rho * rho);
    }
    double al = pr_alpha(e);
    double b = e->b;
    return e->scale * (rho * e->R * e->T / (1.0 - b * rho) -
                       e->a * al * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho));
}

double or_base_dp(const or_eos* e, double rho)
{
    if (e->base == OR_BASE_CS) {
        double eta = e->b * rho / 4.0;
        return e->scale * (e->R * e->T * cs_q1(eta) - 2.0 * e->a * rho);
    }
    double al = pr_alpha(e);
    double b = e->b;
    double D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    return e->scale * (e->R * e->T / ((1.0 - b * rho) * (1.0 - b * rho)) -
                       e->a * al * 2.0 * rho * (1.0 + b * rho) / (D * D));
}

static double rho_upper(const or_eos* e) { return e->base == OR_BASE_CS ? 4.0 / e->b : 1.0 / e->b; }

/* ---------------------------------------------------------------- */
/* Shaped EOS (Sec. III.D Smooth; Eq. PengEOS)                      */
/* ---------------------------------------------------------------- */
double or_eos_p(const or_eos* e, double rho)
{
    if (e->shape == OR_SHAPE_NONE) return or_base_p(e, rho);
    if (rho <= e->rho_v) return e->k_vap * or_base_p(e, rho);
    if (rho >= e->rho_l) return or_base_p(e, rho) + e->dP_liq;
    if (e->shape == OR_SHAPE_PENG)
        return e->p_sat + e->theta * (rho - e->rho_v) * (rho - e->rho_l) * (rho - e->rho_m);
    if (rho <= e->rho_max) {
        double d = rho - e->rho_max;
        return e->p_max - e->b1 + e->b1 * sqrt(1.0 - d * d / e->a1sq);
    }
    if (rho < e->rho_min) {
        /* R1: printed coefficients in the normalised variable t */
        double a2 = 2.0 * (e->p_max - e->p_min), b2 = 3.0 * (e->p_min - e->p_max), c2 = 0.0, d2 = e->p_max;
        double t = (rho - e->rho_max) / (e->rho_min - e->rho_max);
        return a2 * t * t * t + b2 * t * t + c2 * t + d2;
    }
    {
        /* R2: p_2 = p_min, rho_2 = rho_min */
        double d = rho - e->rho_min;
        return e->p_min + e->b3 - e->b3 * sqrt(1.0 - d * d / e->a3sq);
    }
}

double or_eos_dp(const or_eos* e, double rho)
{
    if (e->shape == OR_SHAPE_NONE) return or_base_dp(e, rho);
    if (rho <= e->rho_v) return e->k_vap * or_base_dp(e, rho);
    if (rho >= e->rho_l) return or_base_dp(e, rho);
    if (e->shape == OR_SHAPE_PENG) {
        double A = rho - e->rho_v, B = rho - e->rho_l, C = rho - e->rho_m;
        return e->theta * (B * C + A * C + A * B);
    }
    if (rho <= e->rho_max) {
        double d = rho - e->rho_max;
        return -e->b1 * d / (e->a1sq * sqrt(1.0 - d * d / e->a1sq));
    }
    if (rho < e->rho_min) {
        double a2 = 2.0 * (e->p_max - e->p_min), b2 = 3.0 * (e->p_min - e->p_max);
        double L = e->rho_min - e->rho_max;
        double t = (rho - e->rho_max) / L;
        return (3.0 * a2 * t * t + 2.0 * b2 * t) / L;
    }
    {
        double d = rho - e->rho_min;
        return e->b3 * d / (e->a3sq * sqrt(1.0 - d * d / e->a3sq));
    }
}

/* ---------------------------------------------------------------- */
/* Generic root finding and quadrature                              */
/* ---------------------------------------------------------------- */
typedef double (*fn1)(double x, const void* ctx);

static double bisect(fn1 f, const void* ctx, double lo, double hi, int* ok)
{
    double flo = f(lo, ctx), fhi = f(hi, ctx);
    if (flo == 0.0) return lo;
    if (fhi == 0.0) return hi;
    if (!((flo > 0) != (fhi > 0))) {
        *ok = 0;
        return NAN;
    }
    for (int it = 0; it < 500; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double fm = f(mid, ctx);
        if (fm == 0.0) return mid;
        if ((fm > 0) == (flo > 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

/* integral of g over [lo,hi] by composite Simpson in s = ln(rho) */
static double simpson_log(fn1 g, const void* ctx, double lo, double hi, int n)
{
    if (!(hi > lo)) return 0.0;
    double s0 = log(lo), s1 = log(hi), h = (s1 - s0) / n, sum = 0.0;
    for (int k = 0; k <= n; ++k) {
        double rho = k == 0 ? lo : (k == n ? hi : exp(s0 + k * h));
        double w = (k == 0 || k == n) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        sum += w * g(rho, ctx) * rho;
    }
    return sum * h / 3.0;
}

#define NQUAD (1 << 15)

/* ---------------------------------------------------------------- */
/* Maxwell rule (Eq. MaxwellRule)                                   */
/* ---------------------------------------------------------------- */
typedef struct {
    const or_eos* e;
    double p0;
    int shaped;
} maxw_ctx;

static double maxwell_integrand(double rho, const void* v)
{
    const maxw_ctx* c = (const maxw_ctx*)v;
    double p = c->shaped ? or_eos_p(c->e, rho) : or_base_p(c->e, rho);
    return (c->p0 - p) / (rho * rho);
}

double or_maxwell_residual(const or_eos* e, double p0, double rho_lo, double rho_hi, int shaped)
{
    maxw_ctx c = {e, p0, shaped};
    if (!shaped || e->shape == OR_SHAPE_NONE)
        return simpson_log(maxwell_integrand, &c, rho_lo, rho_hi, NQUAD);
    /* split at the knots of the shaped loop */
    double knots[4] = {rho_lo, e->rho_max, e->rho_min, rho_hi};
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double a = knots[k] > rho_lo ? knots[k] : rho_lo;
        double b = knots[k + 1] < rho_hi ? knots[k + 1] : rho_hi;
        if (b > a) s += simpson_log(maxwell_integrand, &c, a, b, NQUAD);
    }
    return s;
}

typedef struct {
    const or_eos* e;
    double p0;
} pctx;
static double base_minus_p0(double rho, const void* v)
{
    const pctx* c = (const pctx*)v;
    return or_base_p(c->e, rho) - c->p0;
}

typedef struct {
    or_eos* e;
    double rv, rl;
} maxsolve;
static void coexist_for(const or_eos* e, double p0, double* rv, double* rl)
{
    pctx c = {e, p0};
    int ok = 1;
    *rv = bisect(base_minus_p0, &c, 0.0, e->rho_max, &ok);
    *rl = bisect(base_minus_p0, &c, e->rho_min, rho_upper(e) * (1.0 - 1e-12), &ok);
}
static double maxwell_of_logp(double lp, const void* v)
{
    maxsolve* m = (maxsolve*)v;
    double p0 = exp(lp);
    coexist_for(m->e, p0, &m->rv, &m->rl);
    return or_maxwell_residual(m->e, p0, m->rv, m->rl, 0);
}

/* ---------------------------------------------------------------- */
/* Mechanical stability condition (Eq. VaporLiqEq)                  */
/* ---------------------------------------------------------------- */
typedef struct {
    const or_eos* e;
    double p0, eps, G;
    int with_log; /* 1: integrand times -ln(psi) (d/d eps) */
    int bad;
} mech_ctx;

static double mech_integrand(double rho, const void* v)
{
    mech_ctx* c = (mech_ctx*)v;
    double p = or_eos_p(c->e, rho);
    double dp = or_eos_dp(c->e, rho);
    double arg = 2.0 * (p - rho * CS2) / c->G; /* Eq. InteractionPotential with c = 1 */
    if (!(arg > 0)) {
        c->bad = 1;
        return 0.0;
    }
    double psi = sqrt(arg);
    double dpsi = (dp - CS2) / (c->G * psi);
    double val = (c->p0 - p) * dpsi * pow(psi, -1.0 - c->eps);
    if (c->with_log) val *= -log(psi);
    return val;
}

static double mech_integral(const or_eos* e, double eps, double G, int with_log, int* bad)
{
    double p0 = (e->shape == OR_SHAPE_NONE || e->shape == OR_SHAPE_PENG) ? e->p_sat : e->p_sat_new;
    mech_ctx c = {e, p0, eps, G, with_log, 0};
    double s = 0.0;
    if (e->shape == OR_SHAPE_SMOOTH || e->shape == OR_SHAPE_MODSMOOTH) {
        s += simpson_log(mech_integrand, &c, e->rho_v, e->rho_max, NQUAD);
        s += simpson_log(mech_integrand, &c, e->rho_max, e->rho_min, NQUAD);
        s += simpson_log(mech_integrand, &c, e->rho_min, e->rho_l, NQUAD);
    } else if (e->shape == OR_SHAPE_PENG) {
        s += simpson_log(mech_integrand, &c, e->rho_v, e->rho_m, NQUAD);
        s += simpson_log(mech_integrand, &c, e->rho_m, e->rho_l, NQUAD);
    } else {
        s += simpson_log(mech_integrand, &c, e->rho_v, e->rho_max, NQUAD);
        s += simpson_log(mech_integrand, &c, e->rho_max, e->rho_min, NQUAD);
        s += simpson_log(mech_integrand, &c, e->rho_min, e->rho_l, NQUAD);
    }
    if (bad) *bad = c.bad;
    return s;
}

double or_mech_residual(const or_eos* e, double eps, double G) { return mech_integral(e, eps, G, 0, NULL); }

/* ---------------------------------------------------------------- */
/* Smooth loop coefficients (Sec. III.D)                            */
/* ---------------------------------------------------------------- */
static void region1_coeffs(or_eos* e)
{
    double D = e->rho_max - e->rho_v;
    double dpv = e->p_max - e->p_sat_new;
    double k = dpv * D / e->slope_v - D * D;
    e->a1sq = -k * k / (2.0 * k + D * D);
    e->b1 = dpv / (1.0 - sqrt(1.0 - D * D / e->a1sq));
}
static void region3_coeffs(or_eos* e)
{
    double D = e->rho_l - e->rho_min;
    double dpl = e->p_sat_new - e->p_min;
    double k = dpl * D / e->slope_l - D * D;
    e->a3sq = -k * k / (2.0 * k + D * D);
    e->b3 = dpl / (1.0 - sqrt(1.0 - D * D / e->a3sq));
}

/* Replace the four interior knots of a built Smooth loop and refit both
 * ellipses (Sec. III.D).  Used to differentiate by finite differences with
 * the knots treated as independent parameters. */
int or_eos_set_knots(or_eos* e, double rho_max, double p_max, double rho_min, double p_min)
{
    if (e->shape != OR_SHAPE_SMOOTH && e->shape != OR_SHAPE_MODSMOOTH) return OR_EINVAL;
    if (!(e->rho_v < rho_max && rho_max < rho_min && rho_min < e->rho_l)) return OR_EINVAL;
    e->rho_max = rho_max;
    e->p_max = p_max;
    e->rho_min = rho_min;
    e->p_min = p_min;
    region1_coeffs(e);
    region3_coeffs(e);
    if (!(e->a1sq > 0) || !(e->a3sq > 0) || !isfinite(e->b1) || !isfinite(e->b3)) return OR_EINVAL;
    return OR_OK;
}

static double smooth_maxwell_of_pmax(double pmax, const void* v)
{
    or_eos* e = (or_eos*)v;
    e->p_max = pmax;
    region1_coeffs(e);
    return or_maxwell_residual(e, e->p_sat_new, e->rho_v, e->rho_l, 1);
}
typedef struct {
    or_eos* e;
    double G;
} modctx;
static double smooth_mech_of_pmax(double pmax, const void* v)
{
    const modctx* m = (const modctx*)v;
    m->e->p_max = pmax;
    region1_coeffs(m->e);
    return mech_integral(m->e, 0.0, m->G, 0, NULL);
}
static double peng_mech_of_rhom(double rhom, const void* v)
{
    const modctx* m = (const modctx*)v;
    or_eos* e = m->e;
    e->rho_m = rhom;
    /* Eq. PengTheta */
    e->theta = (1.0 - e->r_theta) / ((e->rho_v - rhom) * (e->rho_v - e->rho_l)) * e->slope_v +
               e->r_theta / ((e->rho_l - rhom) * (e->rho_l - e->rho_v)) * e->slope_l;
    return mech_integral(e, 0.0, m->G, 0, NULL);
}

int or_eos_build(or_eos* e, double G, double* sigma_out)
{
    if (!(G < 0) || !(e->Tr > 0) || !(e->Tr < 1) || !(e->a > 0) || !(e->b > 0) || !(e->R > 0))
        return OR_EINVAL;
    if (e->scale == 0.0) e->scale = 1.0;
    if (e->k_vap == 0.0) e->k_vap = 1.0;
    if (e->shape == OR_SHAPE_PENG && e->k_vap != 1.0) return OR_EINVAL;
    /* critical temperature (R5, R10) */
    if (e->base == OR_BASE_CS) {
        double ec = or_cs_critical_eta();
        e->Tc = 8.0 * e->a / (e->R * e->b * cs_q2(ec));
    } else {
        e->Tc = e->a / (e->b * e->R) * pr_critical_ratio();
    }
    e->T = e->Tr * e->Tc;
    /* spinodals: sign changes of dp/drho of the base EOS */
    {
        int n = 400000;
        double up = rho_upper(e);
        double prev = or_base_dp(e, up * 1e-9);
        double xprev = up * 1e-9;
        int found = 0;
        for (int k = 1; k < n; ++k) {
            double x = up * k / (double)n;
            double d = or_base_dp(e, x);
            if (found == 0 && prev > 0 && d <= 0) {
                double lo = xprev, hi = x;
                for (int it = 0; it < 200; ++it) {
                    double m = 0.5 * (lo + hi);
                    if (or_base_dp(e, m) > 0) lo = m; else hi = m;
                }
                e->rho_max = 0.5 * (lo + hi);
                found = 1;
            } else if (found == 1 && prev < 0 && d >= 0) {
                double lo = xprev, hi = x;
                for (int it = 0; it < 200; ++it) {
                    double m = 0.5 * (lo + hi);
                    if (or_base_dp(e, m) < 0) lo = m; else hi = m;
                }
                e->rho_min = 0.5 * (lo + hi);
                found = 2;
                break;
            }
            prev = d;
            xprev = x;
        }
        if (found != 2) return OR_ENOROOT;
        e->p_max_base = or_base_p(e, e->rho_max);
        e->p_min_base = or_base_p(e, e->rho_min);
    }
    /* Maxwell coexistence of the base EOS (Eq. MaxwellRule), bisection in ln p0 */
    {
        double plo = e->p_min_base > 0 ? e->p_min_base : e->p_max_base * 1e-30;
        maxsolve m = {e, 0, 0};
        int ok = 1;
        double lp = bisect(maxwell_of_logp, &m, log(plo) + 1e-13, log(e->p_max_base) - 1e-13, &ok);
        if (!ok) return OR_ENOROOT;
        e->p_sat = exp(lp);
        coexist_for(e, e->p_sat, &e->rho_v, &e->rho_l);
    }
    /* shaped branches */
    e->p_sat_new = e->p_sat;
    e->dP_liq = 0.0;
    e->slope_v = or_base_dp(e, e->rho_v);
    e->slope_l = or_base_dp(e, e->rho_l);
    e->p_max = e->p_max_base;
    e->p_min = e->p_min_base;
    e->a1sq = e->b1 = e->a3sq = e->b3 = 0.0;
    e->rho_m = e->theta = 0.0;
    if (e->shape == OR_SHAPE_SMOOTH || e->shape == OR_SHAPE_MODSMOOTH) {
        e->p_sat_new = e->k_vap * e->p_sat;
        e->dP_liq = (e->k_vap - 1.0) * e->p_sat;
        e->slope_v = e->k_vap * or_base_dp(e, e->rho_v);
        e->p_min = e->p_sat_new - e->alpha * (e->p_sat - e->p_min_base);
        /* realness of a3 (stated beside region 1 for a1; mirrored) */
        if (!(e->slope_l > 2.0 * (e->p_sat_new - e->p_min) / (e->rho_l - e->rho_min))) return OR_EINVAL;
        region3_coeffs(e);
        double hi = e->p_sat_new + 0.5 * e->slope_v * (e->rho_max - e->rho_v);
        double lo = e->p_sat_new;
        double span = hi - lo;
        int ok = 1;
        /* p_max -> p_sat_new flattens ellipse 1 onto its chord: a1^2 -> D^2 with a margin of
         * order (dp/(S_v D))^2, so the lower end stays 1e-6 of the span inside to keep the
         * ellipse real in FP64 */
        if (e->shape == OR_SHAPE_SMOOTH) {
            e->p_max = bisect(smooth_maxwell_of_pmax, e, lo + span * 1e-6, hi - span * 1e-9, &ok);
        } else {
            modctx m = {e, G};
            e->p_max = bisect(smooth_mech_of_pmax, &m, lo + span * 1e-6, hi - span * 1e-9, &ok);
        }
        if (!ok) return OR_ENOROOT;
        region1_coeffs(e);
    } else if (e->shape == OR_SHAPE_PENG) {
        modctx m = {e, G};
        int ok = 1;
        double span = e->rho_l - e->rho_v;
        double rm = bisect(peng_mech_of_rhom, &m, e->rho_v + span * 1e-6, e->rho_l - span * 1e-6, &ok);
        if (!ok) return OR_ENOROOT;
        peng_mech_of_rhom(rm, &m);
    }
    /* eps from Eq. VaporLiqEq by Newton from eps = 2 (Sec. III.A); sigma = -eps/(16 G) */
    e->eps = 0.0;
    if (e->shape == OR_SHAPE_NONE || e->shape == OR_SHAPE_SMOOTH) {
        double eps = 2.0;
        int conv = 0;
        for (int it = 0; it < 200; ++it) {
            int bad = 0;
            double r = mech_integral(e, eps, G, 0, &bad);
            double dr = mech_integral(e, eps, G, 1, &bad);
            if (bad) return OR_EINVAL;
            double step = r / dr;
            eps -= step;
            if (fabs(step) < 1e-13 * (1.0 + fabs(eps))) {
                conv = 1;
                break;
            }
        }
        if (!conv) return OR_ENOROOT;
        e->eps = eps;
    }
    if (sigma_out) *sigma_out = -e->eps / (16.0 * G);
    return OR_OK;
}

/* ---------------------------------------------------------------- */
/* Lattice Boltzmann step                                           */
/* ---------------------------------------------------------------- */
void or_feq(double rho, double ux, double uy, double* feq)
{
    /* Eq. EquilibriumDistribution */
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double second = 0.0;
        double c[2] = {CX[i], CY[i]}, u[2] = {ux, uy};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                second += (c[a] * c[b] - CS2 * (a == b)) * rho * u[a] * u[b];
        feq[i] = WT[i] * (rho + cu * rho / CS2 + second / (2.0 * CS2 * CS2));
    }
}

static double tau_of_rho(const or_params* p, double rho)
{
    /* Eq. RelaxationTime, clamped (R8) */
    double t = p->tau_l * (rho - p->rho_v_tau) / (p->rho_l_tau - p->rho_v_tau) +
               p->tau_v * (rho - p->rho_l_tau) / (p->rho_v_tau - p->rho_l_tau);
    double lo = p->tau_l < p->tau_v ? p->tau_l : p->tau_v;
    double hi = p->tau_l < p->tau_v ? p->tau_v : p->tau_l;
    if (t < lo) t = lo;
    if (t > hi) t = hi;
    return t;
}

void or_collide_node(const or_params* p, const double* f, double Fx, double Fy, double psi,
                     double Ftx, double Fty, double* fout)
{
    build_minv();
    /* Eq. Density, Eq. Momentum */
    double rho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
    }
    double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    /* Eq. RelaxationMatrix */
    double tau[9];
    for (int k = 0; k < 9; ++k) tau[k] = p->tau[k];
    if (p->var_tau) tau[7] = tau[8] = tau_of_rho(p, rho);
    double lam[9];
    for (int k = 0; k < 9; ++k) lam[k] = 1.0 / tau[k];
    /* Eq. OperatorMRT: Omega = -M^-1 Lambda M (f - feq) */
    double feq[9], d[9], md[9], omega[9];
    or_feq(rho, ux, uy, feq);
    for (int i = 0; i < 9; ++i) d[i] = f[i] - feq[i];
    for (int k = 0; k < 9; ++k) {
        md[k] = 0;
        for (int i = 0; i < 9; ++i) md[k] += MROWS[k][i] * d[i];
        md[k] *= lam[k];
    }
    for (int i = 0; i < 9; ++i) {
        omega[i] = 0;
        for (int k = 0; k < 9; ++k) omega[i] -= MINV[i][k] * md[k];
    }
    /* forcing term F' */
    double S[9], Fp[9];
    if (p->forcing == OR_FORCING_GUO) {
        /* Eq. GFS: M^-1 (I - Lambda/2) M applied to w_j (c.F/cs2 + (cc - cs2 I):F u/cs4) */
        double br[9];
        for (int j = 0; j < 9; ++j) {
            double c[2] = {CX[j], CY[j]}, F[2] = {Fx, Fy}, u[2] = {ux, uy};
            double t1 = 0, t2 = 0;
            for (int a = 0; a < 2; ++a) {
                t1 += c[a] * F[a] / CS2;
                for (int b = 0; b < 2; ++b) t2 += (c[a] * c[b] - CS2 * (a == b)) * F[a] * u[b] / (CS2 * CS2);
            }
            br[j] = WT[j] * (t1 + t2);
        }
        for (int k = 0; k < 9; ++k) {
            S[k] = 0;
            for (int j = 0; j < 9; ++j) S[k] += MROWS[k][j] * br[j];
        }
    } else {
        /* Eq. LiFS (moment space), R4 for |F|^2/psi^2 */
        double F2 = Fx * Fx + Fy * Fy;
        double F2overpsi2 = psi != 0.0 ? F2 / (psi * psi) : (Ftx * Ftx + Fty * Fty);
        double uF = ux * Fx + uy * Fy;
        S[0] = 0.0;
        S[1] = 6.0 * uF + 12.0 * p->sigma * F2overpsi2 / (tau[1] - 0.5);
        S[2] = -6.0 * uF - 12.0 * p->sigma * F2overpsi2 / (tau[2] - 0.5);
        S[3] = Fx;
        S[4] = -Fx;
        S[5] = Fy;
        S[6] = -Fy;
        S[7] = 2.0 * (ux * Fx - uy * Fy);
        S[8] = ux * Fy + uy * Fx;
    }
    for (int k = 0; k < 9; ++k) S[k] *= (1.0 - 0.5 * lam[k]); /* R3 */
    for (int i = 0; i < 9; ++i) {
        Fp[i] = 0;
        for (int k = 0; k < 9; ++k) Fp[i] += MINV[i][k] * S[k];
    }
    /* Eq. LBE right-hand side */
    for (int i = 0; i < 9; ++i) fout[i] = f[i] + omega[i] + Fp[i];
}

struct or_lattice {
    or_params P;
    double* f;    /* f_i(t, x): [9][ny][nx] */
    double* fs;   /* post-collision */
    double* rho;
    double* psi;
    double psi_lo, psi_hi;
    long long step;
    long long fail_step;
};

#define IDX(i, x, y) ((size_t)(i) * (size_t)L->P.ny * (size_t)L->P.nx + (size_t)(y) * (size_t)L->P.nx + (size_t)(x))

static double psi_of(const or_params* P, double rho, int* bad)
{
    double p = or_eos_p(&P->eos, rho);
    double arg = 2.0 * (p - rho * CS2) / P->G; /* Eq. InteractionPotential, c = 1 */
    if (!(arg >= 0.0)) {
        *bad = 1;
        return 0.0;
    }
    return sqrt(arg);
}

or_lattice* or_lattice_new(const or_params* p)
{
    if (p->nx < 1 || p->ny < 1) return NULL;
    or_lattice* L = (or_lattice*)calloc(1, sizeof(or_lattice));
    L->P = *p;
    size_t n = (size_t)p->nx * p->ny;
    L->f = (double*)calloc(9 * n, sizeof(double));
    L->fs = (double*)calloc(9 * n, sizeof(double));
    L->rho = (double*)calloc(n, sizeof(double));
    L->psi = (double*)calloc(n, sizeof(double));
    int bad = 0;
    L->psi_lo = p->walls ? psi_of(p, p->rho_wall_lo, &bad) : 0.0;
    L->psi_hi = p->walls ? psi_of(p, p->rho_wall_hi, &bad) : 0.0;
    L->fail_step = -1;
    build_minv();
    return L;
}

void or_lattice_free(or_lattice* L)
{
    if (!L) return;
    free(L->f);
    free(L->fs);
    free(L->rho);
    free(L->psi);
    free(L);
}

void or_init_eq(or_lattice* L, const double* rho, const double* ux, const double* uy)
{
    int nx = L->P.nx, ny = L->P.ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double feq[9];
            or_feq(rho[c], ux ? ux[c] : 0.0, uy ? uy[c] : 0.0, feq);
            for (int i = 0; i < 9; ++i) L->f[IDX(i, x, y)] = feq[i];
        }
    L->step = 0;
    L->fail_step = -1;
}

void or_set_f(or_lattice* L, const double* f) { memcpy(L->f, f, sizeof(double) * 9 * L->P.nx * L->P.ny); }
void or_get_f(const or_lattice* L, double* f) { memcpy(f, L->f, sizeof(double) * 9 * L->P.nx * L->P.ny); }
long long or_fail_step(const or_lattice* L) { return L->fail_step; }

/* psi at node (x, y) with periodic x and, for walls, ghost solid rows (R9) */
static double psi_at(const or_lattice* L, int x, int y)
{
    int nx = L->P.nx, ny = L->P.ny;
    x = ((x % nx) + nx) % nx;
    if (L->P.walls) {
        if (y < 0) return L->psi_lo;
        if (y >= ny) return L->psi_hi;
    } else {
        y = ((y % ny) + ny) % ny;
    }
    return L->psi[(size_t)y * nx + x];
}

/* macroscopic fields at time t; returns nonzero if psi is not real somewhere */
/* rho and psi of every node; 1 if some node has psi^2 < 0.  poison: such a node's
 * psi is NaN instead (see or_run_window) */
static int fields(or_lattice* L, int poison)
{
    int nx = L->P.nx, ny = L->P.ny, flag = 0; /* some node has psi^2 < 0 */
    OR_PARALLEL_ROWS_FLAG
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double r = 0;
            int b = 0;
            for (int i = 0; i < 9; ++i) r += L->f[IDX(i, x, y)];
            L->rho[(size_t)y * nx + x] = r;
            double ps = psi_of(&L->P, r, &b);
            if (b && poison) ps = NAN;
            L->psi[(size_t)y * nx + x] = ps;
            flag |= b;
        }
    return flag;
}

/* Eq. ShanChenForce divided by psi(x): F~ = -G sum_i w(|c_i|^2) psi(x+c_i) c_i */
static void force_tilde(const or_lattice* L, int x, int y, double* Ftx, double* Fty)
{
    double sx = 0, sy = 0;
    for (int i = 1; i < 9; ++i) {
        double w = (CX[i] * CX[i] + CY[i] * CY[i]) == 1 ? 1.0 / 3.0 : 1.0 / 12.0;
        double ps = psi_at(L, x + CX[i], y + CY[i]);
        sx += w * ps * CX[i];
        sy += w * ps * CY[i];
    }
    *Ftx = -L->P.G * sx;
    *Fty = -L->P.G * sy;
}

/* Eq. ShanChenForce divided by psi(x) on a caller-given psi field (algebra tests) */
void or_force_tilde_field(int nx, int ny, const double* psi, int walls, double psi_lo, double psi_hi,
                          double G, double* Ftx, double* Fty)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0, sy = 0;
            for (int i = 1; i < 9; ++i) {
                double w = (CX[i] * CX[i] + CY[i] * CY[i]) == 1 ? 1.0 / 3.0 : 1.0 / 12.0;
                int xx = ((x + CX[i]) % nx + nx) % nx, yy = y + CY[i];
                double ps;
                if (walls && yy < 0) ps = psi_lo;
                else if (walls && yy >= ny) ps = psi_hi;
                else ps = psi[(size_t)(((yy % ny) + ny) % ny) * nx + xx];
                sx += w * ps * CX[i];
                sy += w * ps * CY[i];
            }
            Ftx[(size_t)y * nx + x] = -G * sx;
            Fty[(size_t)y * nx + x] = -G * sy;
        }
}

static int one_step(or_lattice* L, int poison)
{
    int nx = L->P.nx, ny = L->P.ny, flag = 0; /* some post-collision value is not finite */
    if (fields(L, poison) && !poison) return OR_EUNSTABLE;
    OR_PARALLEL_ROWS_FLAG
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double f[9], fo[9], Ftx, Fty;
            for (int i = 0; i < 9; ++i) f[i] = L->f[IDX(i, x, y)];
            force_tilde(L, x, y, &Ftx, &Fty);
            double ps = L->psi[(size_t)y * nx + x];
            or_collide_node(&L->P, f, ps * Ftx, ps * Fty, ps, Ftx, Fty, fo);
            for (int i = 0; i < 9; ++i) {
                flag |= !isfinite(fo[i]);
                L->fs[IDX(i, x, y)] = fo[i];
            }
        }
    if (flag && !poison) return OR_EUNSTABLE;
    /* streaming, Eq. LBE left-hand side; bounce-back at the walls */
    OR_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int tx = ((x + CX[i]) % nx + nx) % nx;
                int ty = y + CY[i];
                double v = L->fs[IDX(i, x, y)];
                if (L->P.walls && (ty < 0 || ty >= ny)) {
                    L->f[IDX(opposite(i), x, y)] = v;
                } else {
                    ty = ((ty % ny) + ny) % ny;
                    L->f[IDX(i, tx, ty)] = v;
                }
            }
    L->step++;
    return OR_OK;
}

int or_threads(void)
{
#ifdef OR_OMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_run(or_lattice* L, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) {
        int st = one_step(L, 0);
        if (st != OR_OK) {
            L->fail_step = L->step;
            return st;
        }
    }
    return OR_OK;
}

/* The same steps on a periodic window cut out of a larger lattice, for checking the
 * window's centre: the cut joins unrelated states at the window's edges, where a node
 * may reach psi^2 < 0.  Such a node's psi is NaN and the run goes on; NaN spreads at
 * most two nodes per step (the pull and the psi stencil of Eq. ShanChenForce), as any
 * information does, so a finite centre was never reached by the cut. */
int or_run_window(or_lattice* L, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) one_step(L, 1);
    return OR_OK;
}

int or_macros(or_lattice* L, double* rho, double* ux, double* uy, double* psi, double* p,
              double* Fx, double* Fy)
{
    int nx = L->P.nx, ny = L->P.ny;
    int bad = fields(L, 0);
    OR_PARALLEL_ROWS
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double r = L->rho[c], jx = 0, jy = 0, Ftx, Fty;
            for (int i = 0; i < 9; ++i) {
                jx += L->f[IDX(i, x, y)] * CX[i];
                jy += L->f[IDX(i, x, y)] * CY[i];
            }
            force_tilde(L, x, y, &Ftx, &Fty);
            double fx = L->psi[c] * Ftx, fy = L->psi[c] * Fty;
            if (rho) rho[c] = r;
            if (ux) ux[c] = (jx + 0.5 * fx) / r;
            if (uy) uy[c] = (jy + 0.5 * fy) / r;
            if (psi) psi[c] = L->psi[c];
            if (p) p[c] = or_eos_p(&L->P.eos, r);
            if (Fx) Fx[c] = fx;
            if (Fy) Fy[c] = fy;
        }
    return bad ? OR_EUNSTABLE : OR_OK;
}
