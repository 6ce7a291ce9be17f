/*
 * fd_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * Plain FP64 CPU reference of the finite-difference solver the paper uses as
 * the reference for its dynamic tests (Appendix "Finite Difference Method"):
 * mass and momentum equations in the form of Eq. FDmomentum, viscous stress of
 * Eq. StressTensor with the viscosities of Eq. DynamicViscosity (tau_nu from
 * Eq. RelaxationTime, its density derivative as in Eq. FDviscosityDerivative),
 * and the pseudopotential pressure tensor through Eq. FDforce, integrated with
 * the MacCormack predictor-corrector:
 *   Q* = Q^n + dt R+(Q^n),   Q^{n+1} = (Q^n + Q* + dt R-(Q*)) / 2,
 * where R+ uses first-order forward differences for the first derivatives of
 * the convective, pressure and viscous terms, R- backward differences, and all
 * second and third derivatives (and every derivative inside Eq. FDforce) are
 * second-order central differences.  Mesh of spacing h (LBM units, c = 1,
 * c_s^2 = 1/3), periodic in x; in y periodic, or walls as in the appendix's
 * grid study: below row 0 the layer b1 on the wall (rho and psi extrapolated
 * from rows 0 and 1, u = v = 0) and the solid layer b2 (Eq. B2, psi only);
 * row ny-1 lies on the top wall and the layers above mirror rows ny-2 and
 * ny-3 (velocities reversed).  Written node by node for checkability.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_fd {
    or_fd_params P;
    double *rho, *u, *v;        /* state Q^n */
    double *rs, *us, *vs;       /* predictor state Q* */
    double *psi, *p;            /* psi and p_EOS of the state being differentiated */
    double *dr, *du, *dv;       /* right-hand side */
};

static int idx(const or_fd* F, int i, int j)
{
    const int nx = F->P.nx, ny = F->P.ny;
    i = ((i % nx) + nx) % nx;
    j = ((j % ny) + ny) % ny;
    return j * nx + i;
}

enum { FD_RHO, FD_U, FD_V, FD_PSI, FD_P };

/* value of a field at (i, j), including the wall layers j = -2, -1, ny, ny + 1 */
static double val(const or_fd* F, int kind, const double* f, const double* rho, int i, int j)
{
    const int ny = F->P.ny;
    if (!F->P.walls || (j >= 0 && j < ny)) return f[idx(F, i, j)];
    if (j >= ny) {
        /* reflexive top: t1 mirrors ny-2, t2 mirrors ny-3 (velocities reversed) */
        const int m = 2 * (ny - 1) - j;
        const double s = (kind == FD_U || kind == FD_V) ? -1.0 : 1.0;
        return s * f[idx(F, i, m)];
    }
    /* bottom: b1 (j = -1) on the wall, b2 (j = -2) inside it */
    if (kind == FD_U || kind == FD_V) return 0.0;
    if (kind == FD_RHO) return 2.0 * f[idx(F, i, 0)] - f[idx(F, i, 1)];
    if (kind == FD_P) return or_eos_p(&F->P.eos, 2.0 * rho[idx(F, i, 0)] - rho[idx(F, i, 1)]);
    const double b1 = 2.0 * f[idx(F, i, 0)] - f[idx(F, i, 1)];
    if (j == -1) return b1;
    return b1 + 2.0 * F->P.h * (F->P.psi_wall - b1); /* Eq. B2 */
}

or_fd* or_fd_new(const or_fd_params* P)
{
    if (P->nx < 3 || P->ny < 3 || !(P->h > 0) || !(P->dt > 0)) return NULL;
    or_fd* F = (or_fd*)calloc(1, sizeof(or_fd));
    F->P = *P;
    const size_t n = (size_t)P->nx * P->ny;
    double** arr[] = {&F->rho, &F->u, &F->v, &F->rs, &F->us, &F->vs, &F->psi, &F->p, &F->dr, &F->du, &F->dv};
    for (size_t k = 0; k < sizeof(arr) / sizeof(arr[0]); ++k) *arr[k] = (double*)calloc(n, sizeof(double));
    return F;
}

void or_fd_free(or_fd* F)
{
    if (!F) return;
    free(F->rho); free(F->u); free(F->v); free(F->rs); free(F->us); free(F->vs);
    free(F->psi); free(F->p); free(F->dr); free(F->du); free(F->dv);
    free(F);
}

void or_fd_set(or_fd* F, const double* rho, const double* u, const double* v)
{
    const size_t n = (size_t)F->P.nx * F->P.ny;
    memcpy(F->rho, rho, n * sizeof(double));
    for (size_t k = 0; k < n; ++k) {
        F->u[k] = u ? u[k] : 0.0;
        F->v[k] = v ? v[k] : 0.0;
    }
}

void or_fd_get(const or_fd* F, double* rho, double* u, double* v)
{
    const size_t n = (size_t)F->P.nx * F->P.ny;
    if (rho) memcpy(rho, F->rho, n * sizeof(double));
    if (u) memcpy(u, F->u, n * sizeof(double));
    if (v) memcpy(v, F->v, n * sizeof(double));
}

/* Eq. RelaxationTime for tau_nu (clamped, R8) and its density derivative */
static void tau_nu_of(const or_fd_params* P, double rho, double* t, double* dt)
{
    if (!P->var_tau) {
        *t = P->tau_nu;
        *dt = 0.0;
        return;
    }
    const double s = (P->tau_l - P->tau_v) / (P->rho_l_tau - P->rho_v_tau);
    double x = P->tau_v + s * (rho - P->rho_v_tau);
    const double lo = P->tau_l < P->tau_v ? P->tau_l : P->tau_v;
    const double hi = P->tau_l < P->tau_v ? P->tau_v : P->tau_l;
    *dt = s;
    if (x <= lo) { x = lo; *dt = 0.0; }
    if (x >= hi) { x = hi; *dt = 0.0; }
    *t = x;
}

/* p_EOS and psi = sqrt(2 (p - rho c_s^2) / G) (Eq. InteractionPotential) of a field */
static int fields(or_fd* F, const double* rho)
{
    const size_t n = (size_t)F->P.nx * F->P.ny;
    for (size_t k = 0; k < n; ++k) {
        const double r = rho[k];
        if (!(r > 0) || !isfinite(r)) return OR_EUNSTABLE;
        const double p = or_eos_p(&F->P.eos, r);
        const double q = 2.0 * (p - r / 3.0) / F->P.G;
        if (!(q >= 0)) return OR_EUNSTABLE;
        F->p[k] = p;
        F->psi[k] = sqrt(q);
    }
    return OR_OK;
}

/* first derivative along axis (0 = x, 1 = y): dir +1 forward, -1 backward, 0 central */
static double d1(const or_fd* F, int kind, const double* f, const double* rho, int i, int j, int axis, int dir)
{
    const double h = F->P.h;
    const int di = axis == 0, dj = axis == 1;
    if (dir > 0) return (val(F, kind, f, rho, i + di, j + dj) - val(F, kind, f, rho, i, j)) / h;
    if (dir < 0) return (val(F, kind, f, rho, i, j) - val(F, kind, f, rho, i - di, j - dj)) / h;
    return (val(F, kind, f, rho, i + di, j + dj) - val(F, kind, f, rho, i - di, j - dj)) / (2.0 * h);
}

/* central second derivatives d^2 f / dx_a dx_b */
static double d2(const or_fd* F, int kind, const double* f, const double* rho, int i, int j, int a, int b)
{
    const double h = F->P.h;
    if (a == b) {
        const int di = a == 0, dj = a == 1;
        return (val(F, kind, f, rho, i + di, j + dj) - 2.0 * val(F, kind, f, rho, i, j) +
                val(F, kind, f, rho, i - di, j - dj)) / (h * h);
    }
    return (val(F, kind, f, rho, i + 1, j + 1) - val(F, kind, f, rho, i + 1, j - 1) -
            val(F, kind, f, rho, i - 1, j + 1) + val(F, kind, f, rho, i - 1, j - 1)) / (4.0 * h * h);
}

static double lap(const or_fd* F, const double* f, const double* rho, int i, int j)
{
    return d2(F, FD_PSI, f, rho, i, j, 0, 0) + d2(F, FD_PSI, f, rho, i, j, 1, 1);
}

/* right-hand sides of the mass and momentum equations at every node */
static void rhs(or_fd* F, const double* rho, const double* u, const double* v, int dir)
{
    const or_fd_params* P = &F->P;
    const double cs2 = 1.0 / 3.0, G = P->G, eps = P->eps;
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            const int k = idx(F, i, j);
            const double r = rho[k], ux = u[k], uy = v[k];
            /* first derivatives, one-sided per stage */
            const double rx = d1(F, FD_RHO, rho, rho, i, j, 0, dir), ry = d1(F, FD_RHO, rho, rho, i, j, 1, dir);
            const double uxx1 = d1(F, FD_U, u, rho, i, j, 0, dir), uxy1 = d1(F, FD_U, u, rho, i, j, 1, dir);
            const double vx1 = d1(F, FD_V, v, rho, i, j, 0, dir), vy1 = d1(F, FD_V, v, rho, i, j, 1, dir);
            const double px = d1(F, FD_P, F->p, rho, i, j, 0, dir), py = d1(F, FD_P, F->p, rho, i, j, 1, dir);
            const double div = uxx1 + vy1;
            /* mass */
            F->dr[k] = -(r * div + ux * rx + uy * ry);
            /* viscosities (Eq. DynamicViscosity) and their gradients (Eq. FDviscosityDerivative) */
            double tn, dtn;
            tau_nu_of(P, r, &tn, &dtn);
            const double mu = r * cs2 * (tn - 0.5), dmu = cs2 * (tn - 0.5) + r * cs2 * dtn;
            const double muB = r * cs2 * (P->tau_e - tn), dmuB = cs2 * (P->tau_e - tn) - r * cs2 * dtn;
            const double mux = dmu * rx, muy = dmu * ry, mBx = dmuB * rx, mBy = dmuB * ry;
            /* central second derivatives of the velocity */
            const double u_xx = d2(F, FD_U, u, rho, i, j, 0, 0), u_yy = d2(F, FD_U, u, rho, i, j, 1, 1);
            const double u_xy = d2(F, FD_U, u, rho, i, j, 0, 1);
            const double v_xx = d2(F, FD_V, v, rho, i, j, 0, 0), v_yy = d2(F, FD_V, v, rho, i, j, 1, 1);
            const double v_xy = d2(F, FD_V, v, rho, i, j, 0, 1);
            /* divergence of the viscous stress (Eq. FDstressTensor) */
            const double Sx = mux * (2.0 * uxx1) + muy * (vx1 + uxy1) + mu * (2.0 * u_xx + u_yy + v_xy) + mBx * div +
                              muB * (u_xx + v_xy);
            const double Sy = mux * (uxy1 + vx1) + muy * (2.0 * vy1) + mu * (v_xx + 2.0 * v_yy + u_xy) + mBy * div +
                              muB * (u_xy + v_yy);
            /* divergence of the non-ideal pressure tensor (Eq. FDforce), central differences */
            const double* s = F->psi;
            const double ps = s[k];
            const double sx = d1(F, FD_PSI, s, rho, i, j, 0, 0), sy = d1(F, FD_PSI, s, rho, i, j, 1, 0);
            const double sxx = d2(F, FD_PSI, s, rho, i, j, 0, 0), syy = d2(F, FD_PSI, s, rho, i, j, 1, 1);
            const double sxy = d2(F, FD_PSI, s, rho, i, j, 0, 1);
            const double L = sxx + syy;
            const double Lx = (lap(F, s, rho, i + 1, j) - lap(F, s, rho, i - 1, j)) / (2.0 * P->h);
            const double Ly = (lap(F, s, rho, i, j + 1) - lap(F, s, rho, i, j - 1)) / (2.0 * P->h);
            const double gx = sx * sxx + sy * sxy, gy = sx * sxy + sy * syy;  /* (d_g psi)(d_a d_g psi) */
            const double Px = -eps * G / 4.0 * gx + G / 12.0 * sx * L + G / 6.0 * gx + G / 4.0 * ps * Lx;
            const double Py = -eps * G / 4.0 * gy + G / 12.0 * sy * L + G / 6.0 * gy + G / 4.0 * ps * Ly;
            /* momentum (Eq. FDmomentum) */
            F->du[k] = -(ux * uxx1 + uy * uxy1) - px / r - Px / r + Sx / r;
            F->dv[k] = -(ux * vx1 + uy * vy1) - py / r - Py / r + Sy / r;
        }
}

int or_fd_run(or_fd* F, long long nsteps)
{
    const size_t n = (size_t)F->P.nx * F->P.ny;
    const double dt = F->P.dt;
    for (long long t = 0; t < nsteps; ++t) {
        /* predictor: forward differences */
        if (fields(F, F->rho) != OR_OK) return OR_EUNSTABLE;
        rhs(F, F->rho, F->u, F->v, +1);
        for (size_t k = 0; k < n; ++k) {
            F->rs[k] = F->rho[k] + dt * F->dr[k];
            F->us[k] = F->u[k] + dt * F->du[k];
            F->vs[k] = F->v[k] + dt * F->dv[k];
        }
        /* corrector: backward differences on the predicted state */
        if (fields(F, F->rs) != OR_OK) return OR_EUNSTABLE;
        rhs(F, F->rs, F->us, F->vs, -1);
        for (size_t k = 0; k < n; ++k) {
            F->rho[k] = 0.5 * (F->rho[k] + F->rs[k] + dt * F->dr[k]);
            F->u[k] = 0.5 * (F->u[k] + F->us[k] + dt * F->du[k]);
            F->v[k] = 0.5 * (F->v[k] + F->vs[k] + dt * F->dv[k]);
        }
    }
    return OR_OK;
}
