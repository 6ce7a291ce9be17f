// Host FP64 thermodynamics of the shaped equation of state (lbm_eos_build).
//
// Sec. III.A: Maxwell coexistence (Eq. MaxwellRule) and eps from the
// mechanical stability condition (Eq. VaporLiqEq), sigma = -eps/(16 G)
// (Sec. II.C).  Sec. III.D: the Smooth vdW-loop replacement (ellipse /
// cubic / ellipse through four knots).  Eq. PengEOS / Eq. PengTheta, and the
// Modified Smooth loop of Sec. IV.C.
//
// Numerics chosen for this library: closed-form antiderivatives of p/rho^2
// for the base EOS, Brent's method for every scalar root, and composite
// 8-point Gauss-Legendre quadrature in ln(rho) for integrals over the
// shaped loop.
#include <cmath>
#include <complex>
#include <cstring>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

constexpr double kCs2 = 1.0 / 3.0;

// ----------------------------------------------------------------- base EOS
double pr_alpha(const lbm_eos& e)
{
    const double kap = 0.37464 + 1.54226 * e.omega - 0.26992 * e.omega * e.omega;
    const double t = 1.0 + kap * (1.0 - std::sqrt(e.T / e.Tc));
    return t * t;
}

// unscaled base pressure and derivatives at temperature T with a given a*alpha
double cs_p(double a, double b, double RT, double rho)
{
    const double n = 0.25 * b * rho, m = 1.0 - n;
    return RT * rho * (1.0 + n * (1.0 + n * (1.0 - n))) / (m * m * m) - a * rho * rho;
}
double cs_dp(double a, double b, double RT, double rho)
{
    const double n = 0.25 * b * rho, m = 1.0 - n;
    const double m2 = m * m;
    return RT * (1.0 + n * (4.0 + n * (4.0 + n * (-4.0 + n)))) / (m2 * m2) - 2.0 * a * rho;
}
double cs_d2p(double a, double b, double RT, double rho)
{
    const double n = 0.25 * b * rho, m = 1.0 - n;
    const double m5 = m * m * m * m * m;
    return RT * 0.25 * b * (8.0 + n * (20.0 - 4.0 * n)) / m5 - 2.0 * a;
}
double pr_p(double aal, double b, double RT, double rho)
{
    const double D = 1.0 + b * rho * (2.0 - b * rho);
    return RT * rho / (1.0 - b * rho) - aal * rho * rho / D;
}
double pr_dp(double aal, double b, double RT, double rho)
{
    const double D = 1.0 + b * rho * (2.0 - b * rho);
    const double m = 1.0 - b * rho;
    return RT / (m * m) - 2.0 * aal * rho * (1.0 + b * rho) / (D * D);
}
double pr_d2p(double aal, double b, double RT, double rho)
{
    const double D = 1.0 + b * rho * (2.0 - b * rho);
    const double Dp = 2.0 * b * (1.0 - b * rho);
    const double m = 1.0 - b * rho;
    const double N = rho * (1.0 + b * rho), Np = 1.0 + 2.0 * b * rho;
    return 2.0 * b * RT / (m * m * m) - 2.0 * aal * (Np * D - 2.0 * N * Dp) / (D * D * D);
}

double a_eff(const lbm_eos& e) { return e.base == LBM_BASE_PR ? e.a * pr_alpha(e) : e.a; }

double basep(const lbm_eos& e, double rho)
{
    const double RT = e.R * e.T;
    return e.scale * (e.base == LBM_BASE_PR ? pr_p(a_eff(e), e.b, RT, rho) : cs_p(e.a, e.b, RT, rho));
}
double basedp(const lbm_eos& e, double rho)
{
    const double RT = e.R * e.T;
    return e.scale * (e.base == LBM_BASE_PR ? pr_dp(a_eff(e), e.b, RT, rho) : cs_dp(e.a, e.b, RT, rho));
}
double rho_cap(const lbm_eos& e) { return e.base == LBM_BASE_PR ? 1.0 / e.b : 4.0 / e.b; }

// closed-form antiderivative of p/rho^2 (scaled base EOS)
double base_prim(const lbm_eos& e, double rho)
{
    const double RT = e.R * e.T;
    if (e.base == LBM_BASE_PR) {
        const double s2 = std::sqrt(2.0), br = e.b * rho;
        return e.scale * (RT * std::log(rho / (1.0 - br)) -
                          a_eff(e) / (2.0 * s2 * e.b) * std::log((s2 - 1.0 + br) / (s2 + 1.0 - br)));
    }
    const double n = 0.25 * e.b * rho;
    return e.scale * (RT * (std::log(rho) + n * (4.0 - 3.0 * n) / ((1.0 - n) * (1.0 - n))) - e.a * rho);
}

// ----------------------------------------------------------------- Brent
template <class F>
double brent(F f, double a, double b, bool* ok, double rtol = 4e-16)
{
    double fa = f(a), fb = f(b);
    if (fa == 0.0) return a;
    if (fb == 0.0) return b;
    if ((fa > 0) == (fb > 0) || !std::isfinite(fa) || !std::isfinite(fb)) {
        *ok = false;
        return NAN;
    }
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0) == (fc > 0)) {
            c = a;
            fc = fa;
            d = e = b - a;
        }
        if (std::fabs(fc) < std::fabs(fb)) {
            a = b; b = c; c = a;
            fa = fb; fb = fc; fc = fa;
        }
        const double tol = 2.0 * rtol * std::fabs(b) + 1e-300;
        const double m = 0.5 * (c - b);
        if (std::fabs(m) <= tol || fb == 0.0) return b;
        if (std::fabs(e) >= tol && std::fabs(fa) > std::fabs(fb)) {
            double p, q, r;
            const double s = fb / fa;
            if (a == c) {
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else {
                q = fa / fc;
                r = fb / fc;
                p = s * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
                q = (q - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0) q = -q; else p = -p;
            if (2.0 * p < std::fmin(3.0 * m * q - std::fabs(tol * q), std::fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = m;
                e = m;
            }
        } else {
            d = m;
            e = m;
        }
        a = b;
        fa = fb;
        b += std::fabs(d) > tol ? d : (m > 0 ? tol : -tol);
        fb = f(b);
    }
    return b;
}

// ----------------------------------------------------------------- quadrature
const double kGLx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                        0.1834346424956498,  0.5255324099163290,  0.7966664774136267,  0.9602898564975363};
const double kGLw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                        0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

// int_lo^hi g(rho) d rho with rho = exp(s), composite 8-point Gauss-Legendre
template <class F>
double gl_log(F g, double lo, double hi, int panels = 768)
{
    if (!(hi > lo)) return 0.0;
    const double s0 = std::log(lo), s1 = std::log(hi), h = (s1 - s0) / panels;
    double acc = 0.0;
    for (int k = 0; k < panels; ++k) {
        const double c = s0 + (k + 0.5) * h;
        double part = 0.0;
        for (int q = 0; q < 8; ++q) {
            const double r = std::exp(c + 0.5 * h * kGLx[q]);
            part += kGLw[q] * g(r) * r;
        }
        acc += part;
    }
    return 0.5 * h * acc;
}

// ----------------------------------------------------------------- shaped loop
// ellipse coefficients (a^2, b) of a region joining the saturated knot
// (rho_s, p_s), where the slope is S, to the knot (rho_k, p_k) of zero slope;
// with D = rho_k - rho_s, dp = p_k - p_s and r = dp/(S D):
// a^2 = D^2 (1-r)^2/(1-2r), b = |dp| (1-r)/(1-2r) (Sec. III.D, regions 1 and 3)
template <class R>
void ellipse_coeffs(R rho_k, R p_k, double rho_s, double p_s, double S, R* asq, R* b)
{
    const R D = rho_k - rho_s, dp = p_k - p_s;
    const R r = dp / (S * D);
    *asq = D * D * (1.0 - r) * (1.0 - r) / (1.0 - 2.0 * r);
    *b = (std::real(dp) < 0.0 ? -dp : dp) * (1.0 - r) / (1.0 - 2.0 * r);
}

void fill_region1(lbm_eos& e) { ellipse_coeffs<double>(e.rho_max, e.p_max, e.rho_v, e.p_sat_new, e.slope_v, &e.a1sq, &e.b1); }
void fill_region3(lbm_eos& e) { ellipse_coeffs<double>(e.rho_min, e.p_min, e.rho_l, e.p_sat_new, e.slope_l, &e.a3sq, &e.b3); }

double mech_residual(const lbm_eos& e, double eps, double G, bool* bad)
{
    const double p0 = (e.shape == LBM_SHAPE_NONE || e.shape == LBM_SHAPE_PENG) ? e.p_sat : e.p_sat_new;
    auto g = [&](double r) {
        const double p = lbm_eos_pressure(&e, r), dp = lbm_eos_slope(&e, r);
        const double q = 2.0 * (p - kCs2 * r) / G;
        if (!(q > 0.0)) {
            *bad = true;
            return 0.0;
        }
        const double psi = std::sqrt(q);
        // (p0 - p) psi' psi^(-1-eps), psi' = (p' - 1/3)/(G psi)
        return (p0 - p) * (dp - kCs2) / G * std::pow(psi, -2.0 - eps);
    };
    double knots[4];
    int nk = 0;
    knots[nk++] = e.rho_v;
    if (e.shape == LBM_SHAPE_PENG) {
        knots[nk++] = e.rho_m;
    } else {
        knots[nk++] = e.rho_max;
        knots[nk++] = e.rho_min;
    }
    knots[nk++] = e.rho_l;
    double s = 0.0;
    for (int k = 0; k + 1 < nk; ++k) s += gl_log(g, knots[k], knots[k + 1]);
    return s;
}

double shaped_maxwell(const lbm_eos& e)
{
    auto g = [&](double r) { return (e.p_sat_new - lbm_eos_pressure(&e, r)) / (r * r); };
    return gl_log(g, e.rho_v, e.rho_max) + gl_log(g, e.rho_max, e.rho_min) + gl_log(g, e.rho_min, e.rho_l);
}

thread_local char g_msg[256];

}  // namespace

void lbm_set_error(const char* msg)
{
    std::strncpy(g_msg, msg, sizeof(g_msg) - 1);
    g_msg[sizeof(g_msg) - 1] = 0;
}

extern "C" const char* lbm_last_error(void) { return g_msg; }

// d(b1, a1^2)/d(rho_max, p_max) and d(b3, a3^2)/d(rho_min, p_min) by complex-step
// differentiation of the coefficient formulas (exact to rounding)
void lbm_knot_jacobians(const lbm_eos* ep, double J1[2][2], double J3[2][2])
{
    const lbm_eos& e = *ep;
    using C = std::complex<double>;
    const double h = 1e-30;
    for (int k = 0; k < 2; ++k) {
        const double sr = k == 0 ? h * std::fabs(e.rho_max) : h * std::fabs(e.p_max);
        C a, b;
        ellipse_coeffs<C>(C(e.rho_max, k == 0 ? sr : 0.0), C(e.p_max, k == 1 ? sr : 0.0), e.rho_v, e.p_sat_new, e.slope_v,
                          &a, &b);
        J1[0][k] = b.imag() / sr;
        J1[1][k] = a.imag() / sr;
        const double s3 = k == 0 ? h * std::fabs(e.rho_min) : h * std::fabs(e.p_min);
        ellipse_coeffs<C>(C(e.rho_min, k == 0 ? s3 : 0.0), C(e.p_min, k == 1 ? s3 : 0.0), e.rho_l, e.p_sat_new, e.slope_l,
                          &a, &b);
        J3[0][k] = b.imag() / s3;
        J3[1][k] = a.imag() / s3;
    }
}

extern "C" int lbm_eos_set_knots(lbm_eos* ep, double rho_max, double p_max, double rho_min, double p_min)
{
    lbm_eos& e = *ep;
    if (e.shape != LBM_SHAPE_SMOOTH && e.shape != LBM_SHAPE_MODSMOOTH) {
        lbm_set_error("lbm_eos_set_knots: only the Smooth loops have four knots");
        return LBM_EINVAL;
    }
    if (!(e.rho_v < rho_max && rho_max < rho_min && rho_min < e.rho_l) ||
        !(2.0 * (p_max - e.p_sat_new) < e.slope_v * (rho_max - e.rho_v)) || !(p_max > e.p_sat_new) ||
        !(2.0 * (e.p_sat_new - p_min) < e.slope_l * (e.rho_l - rho_min)) || !(p_min < e.p_sat_new)) {
        lbm_set_error("lbm_eos_set_knots: knots out of order or an ellipse would not be real");
        return LBM_EINVAL;
    }
    e.rho_max = rho_max;
    e.p_max = p_max;
    e.rho_min = rho_min;
    e.p_min = p_min;
    fill_region1(e);
    fill_region3(e);
    return LBM_OK;
}

extern "C" double lbm_eos_pressure(const lbm_eos* ep, double rho)
{
    const lbm_eos& e = *ep;
    if (e.shape == LBM_SHAPE_NONE) return basep(e, rho);
    if (rho <= e.rho_v) return e.k_vap * basep(e, rho);
    if (rho >= e.rho_l) return basep(e, rho) + e.dP_liq;
    if (e.shape == LBM_SHAPE_PENG) return e.p_sat + e.theta * (rho - e.rho_v) * (rho - e.rho_l) * (rho - e.rho_m);
    if (rho <= e.rho_max) {
        const double d = rho - e.rho_max;
        return e.p_max - e.b1 * (1.0 - std::sqrt(1.0 - d * d / e.a1sq));
    }
    if (rho < e.rho_min) {
        const double t = (rho - e.rho_max) / (e.rho_min - e.rho_max);
        return e.p_max + (e.p_min - e.p_max) * t * t * (3.0 - 2.0 * t);
    }
    const double d = rho - e.rho_min;
    return e.p_min + e.b3 * (1.0 - std::sqrt(1.0 - d * d / e.a3sq));
}

extern "C" double lbm_eos_slope(const lbm_eos* ep, double rho)
{
    const lbm_eos& e = *ep;
    if (e.shape == LBM_SHAPE_NONE) return basedp(e, rho);
    if (rho <= e.rho_v) return e.k_vap * basedp(e, rho);
    if (rho >= e.rho_l) return basedp(e, rho);
    if (e.shape == LBM_SHAPE_PENG) {
        const double u = rho - e.rho_v, v = rho - e.rho_l, w = rho - e.rho_m;
        return e.theta * (u * v + v * w + w * u);
    }
    if (rho <= e.rho_max) {
        const double d = rho - e.rho_max;
        return -e.b1 * d / (e.a1sq * std::sqrt(1.0 - d * d / e.a1sq));
    }
    if (rho < e.rho_min) {
        const double L = e.rho_min - e.rho_max, t = (rho - e.rho_max) / L;
        return (e.p_min - e.p_max) * 6.0 * t * (1.0 - t) / L;
    }
    const double d = rho - e.rho_min;
    return e.b3 * d / (e.a3sq * std::sqrt(1.0 - d * d / e.a3sq));
}

extern "C" int lbm_eos_build(lbm_eos* ep, double G, double* sigma_out)
{
    lbm_eos& e = *ep;
    if (!(G < 0.0) || !(e.Tr > 0.0 && e.Tr < 1.0) || !(e.a > 0.0) || !(e.b > 0.0) || !(e.R > 0.0) ||
        (e.base != LBM_BASE_CS && e.base != LBM_BASE_PR) || e.shape < 0 || e.shape > 3) {
        lbm_set_error("lbm_eos_build: invalid EOS inputs (need G<0, 0<Tr<1, a,b,R>0)");
        return LBM_EINVAL;
    }
    if (e.scale == 0.0) e.scale = 1.0;
    if (e.k_vap == 0.0) e.k_vap = 1.0;
    if (e.shape == LBM_SHAPE_PENG && e.k_vap != 1.0) {
        lbm_set_error("lbm_eos_build: the Peng loop keeps the base vapor branch (k_vap must be 1)");
        return LBM_EINVAL;
    }
    bool ok = true;
    // critical point: p' = T A1(rho) - B1(rho) = 0 and p'' = T A2(rho) - B2(rho) = 0 (alpha(Tc) = 1);
    // eliminate T and find rho_c with Brent, then Tc = B1/A1.
    {
        const double a = e.a, b = e.b, R = e.R;
        auto A1 = [&](double r) { return e.base == LBM_BASE_PR ? pr_dp(0.0, b, R, r) : cs_dp(0.0, b, R, r); };
        auto B1 = [&](double r) { return e.base == LBM_BASE_PR ? -pr_dp(a, b, 0.0, r) : -cs_dp(a, b, 0.0, r); };
        auto A2 = [&](double r) { return e.base == LBM_BASE_PR ? pr_d2p(0.0, b, R, r) : cs_d2p(0.0, b, R, r); };
        auto B2 = [&](double r) { return e.base == LBM_BASE_PR ? -pr_d2p(a, b, 0.0, r) : -cs_d2p(a, b, 0.0, r); };
        auto g = [&](double r) { return B1(r) * A2(r) / A1(r) - B2(r); };
        const double cap = rho_cap(e);
        const double rc = brent(g, 0.05 * cap, 0.6 * cap, &ok);
        if (!ok) {
            lbm_set_error("lbm_eos_build: critical point not bracketed");
            return LBM_ENOROOT;
        }
        e.Tc = B1(rc) / A1(rc);
    }
    e.T = e.Tr * e.Tc;
    // spinodals: first maximum and following minimum of the base EOS (geometric scan + Brent)
    {
        const double cap = rho_cap(e);
        double prev_r = cap * 1e-8, prev_d = basedp(e, prev_r);
        int found = 0;
        const int n = 20000;
        for (int k = 1; k <= n && found < 2; ++k) {
            const double r = cap * 1e-8 * std::pow((1.0 - 1e-9) / 1e-8, double(k) / n);
            const double d = basedp(e, r);
            if (found == 0 && prev_d > 0 && d <= 0) {
                e.rho_max = brent([&](double x) { return basedp(e, x); }, prev_r, r, &ok);
                found = 1;
            } else if (found == 1 && prev_d < 0 && d >= 0) {
                e.rho_min = brent([&](double x) { return basedp(e, x); }, prev_r, r, &ok);
                found = 2;
            }
            prev_r = r;
            prev_d = d;
        }
        if (found != 2 || !ok) {
            lbm_set_error("lbm_eos_build: no van der Waals loop (spinodals not found)");
            return LBM_ENOROOT;
        }
        e.p_max_base = basep(e, e.rho_max);
        e.p_min_base = basep(e, e.rho_min);
    }
    // Maxwell coexistence with the closed-form antiderivative, Brent in ln p0
    {
        double rv = 0, rl = 0;
        auto roots = [&](double p0) {
            bool k = true;
            rv = brent([&](double x) { return basep(e, x) - p0; }, 0.0, e.rho_max, &k);
            rl = brent([&](double x) { return basep(e, x) - p0; }, e.rho_min, rho_cap(e) * (1.0 - 1e-13), &k);
            return k;
        };
        auto resid = [&](double lp) {
            const double p0 = std::exp(lp);
            roots(p0);
            return p0 * (1.0 / rv - 1.0 / rl) - (base_prim(e, rl) - base_prim(e, rv));
        };
        const double plo = e.p_min_base > 0.0 ? e.p_min_base * (1.0 + 1e-12) : e.p_max_base * 1e-30;
        const double lp = brent(resid, std::log(plo), std::log(e.p_max_base * (1.0 - 1e-12)), &ok);
        if (!ok) {
            lbm_set_error("lbm_eos_build: Maxwell root not bracketed");
            return LBM_ENOROOT;
        }
        e.p_sat = std::exp(lp);
        roots(e.p_sat);
        e.rho_v = rv;
        e.rho_l = rl;
    }
    e.p_sat_new = e.p_sat;
    e.dP_liq = 0.0;
    e.slope_v = basedp(e, e.rho_v);
    e.slope_l = basedp(e, e.rho_l);
    e.p_max = e.p_max_base;
    e.p_min = e.p_min_base;
    e.a1sq = e.b1 = e.a3sq = e.b3 = 0.0;
    e.rho_m = e.theta = 0.0;
    e.eps = 0.0;
    if (e.shape == LBM_SHAPE_SMOOTH || e.shape == LBM_SHAPE_MODSMOOTH) {
        e.p_sat_new = e.k_vap * e.p_sat;
        e.dP_liq = (e.k_vap - 1.0) * e.p_sat;
        e.slope_v *= e.k_vap;
        e.p_min = e.p_sat_new - e.alpha * (e.p_sat - e.p_min_base);
        if (!(2.0 * (e.p_sat_new - e.p_min) < e.slope_l * (e.rho_l - e.rho_min))) {
            lbm_set_error("lbm_eos_build: region-3 ellipse not real for this alpha");
            return LBM_EINVAL;
        }
        fill_region3(e);
        const double lo = e.p_sat_new, hi = e.p_sat_new + 0.5 * e.slope_v * (e.rho_max - e.rho_v);
        const double span = hi - lo;
        auto fmax = [&](double pm) {
            e.p_max = pm;
            fill_region1(e);
            if (e.shape == LBM_SHAPE_SMOOTH) return shaped_maxwell(e);
            bool bad = false;
            return mech_residual(e, 0.0, G, &bad);
        };
        e.p_max = brent(fmax, lo + 1e-9 * span, hi - 1e-9 * span, &ok, 1e-15);
        if (!ok) {
            lbm_set_error("lbm_eos_build: p_max root not bracketed");
            return LBM_ENOROOT;
        }
        fill_region1(e);
    } else if (e.shape == LBM_SHAPE_PENG) {
        auto fm = [&](double rm) {
            e.rho_m = rm;
            e.theta = (1.0 - e.r_theta) * e.slope_v / ((e.rho_v - rm) * (e.rho_v - e.rho_l)) +
                      e.r_theta * e.slope_l / ((e.rho_l - rm) * (e.rho_l - e.rho_v));
            bool bad = false;
            return mech_residual(e, 0.0, G, &bad);
        };
        const double span = e.rho_l - e.rho_v;
        const double rm = brent(fm, e.rho_v + 1e-6 * span, e.rho_l - 1e-6 * span, &ok, 1e-15);
        if (!ok) {
            lbm_set_error("lbm_eos_build: Peng rho_m root not bracketed");
            return LBM_ENOROOT;
        }
        fm(rm);
    }
    if (e.shape == LBM_SHAPE_NONE || e.shape == LBM_SHAPE_SMOOTH) {
        bool bad = false;
        auto fe = [&](double eps) { return mech_residual(e, eps, G, &bad); };
        double lo = 0.0, hi = 4.0;
        double flo = fe(lo), fhi = fe(hi);
        for (int k = 0; k < 20 && (flo > 0) == (fhi > 0); ++k) {
            lo -= 2.0;
            hi += 2.0;
            flo = fe(lo);
            fhi = fe(hi);
        }
        e.eps = brent(fe, lo, hi, &ok, 1e-15);
        if (!ok || bad) {
            lbm_set_error("lbm_eos_build: eps root of the mechanical stability condition not found");
            return bad ? LBM_EINVAL : LBM_ENOROOT;
        }
    }
    if (sigma_out) *sigma_out = -e.eps / (16.0 * G);
    return LBM_OK;
}
