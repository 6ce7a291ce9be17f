// liblbm.so: the finite-difference reference solver of the paper's appendix
// ("Finite Difference Method"), FP64; periodic in x, in y periodic or with the
// wall layers of the appendix's grid study.
//
// State: rho, u, v on an nx x ny mesh of spacing h (LBM units, c = 1,
// c_s^2 = 1/3).  One time step is the MacCormack predictor-corrector
//   Q* = Q^n + dt R+(Q^n),   Q^{n+1} = (Q^n + Q* + dt R-(Q*)) / 2
// with R the right-hand sides of the mass equation and Eq. FDmomentum: first
// derivatives of the convective, pressure and viscous terms are one-sided
// (forward in R+, backward in R-), second derivatives and every derivative of
// psi in Eq. FDforce are central; viscosities from Eq. DynamicViscosity with
// tau_nu(rho) of Eq. RelaxationTime (Eq. FDviscosityDerivative).
// Two launches per step (predictor, corrector in place over Q^n: the corrector
// reads Q^n only at its own node).  Each workgroup owns a 32 x 8 tile and first
// evaluates p_EOS and psi of its tile plus a two-node halo into LDS (Eq. FDforce
// reaches two nodes out through the Laplacian of psi), then every thread forms
// its node's right-hand side from LDS (psi, p) and the state (radius one).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

struct lbm_fd_ctx {
    lbm_fd_params P;
    lbmk::DevEos eos;
    double psi_wall;
    size_t n;
    double *rho, *u, *v, *rs, *us, *vs;
    unsigned* err;
    long long step;
};

namespace {

using namespace lbmk;

struct FdArgs {
    int nx, ny, var_tau, walls;
    double psi_wall;      // psi_l of Eq. B2
    double h, inv_h, inv_2h, inv_h2, inv_4h2, dt, G, two_inv_G, eps;
    double tau_e, tau_nu, tau_v, tau_lo, tau_hi, dtau, rho_v_tau;
    DevEos eos;
    unsigned* err;
    long long step;
};

__device__ __forceinline__ void fd_flag(const FdArgs& A)
{
    if (atomicCAS(A.err, 0u, 1u) == 0u) A.err[1] = (unsigned)A.step;
}

__device__ __forceinline__ double fd_psi(const FdArgs& A, double r)
{
    const double q = (dev_eos_p(A.eos, r) - r * (1.0 / 3.0)) * A.two_inv_G;
    return q > 0.0 ? sqrt(q) : 0.0;
}

constexpr int kTx = 32, kTy = 8, kHalo = 2;
constexpr int kLx = kTx + 2 * kHalo, kLy = kTy + 2 * kHalo;

// out = a * base + b * (Q + dt R_DIR(Q)) at every node
template <int DIR>
__global__ __launch_bounds__(kTx * kTy) void k_fd_stage(FdArgs A, const double* rho, const double* u, const double* v,
                                                        const double* base_r, const double* base_u,
                                                        const double* base_v, double wa, double wb, double* o_r,
                                                        double* o_u, double* o_v)
{
    __shared__ double spsi[kLy][kLx], spe[kLy][kLx];
    const int tid = threadIdx.y * kTx + threadIdx.x;
    const int i0 = blockIdx.x * kTx, j0 = blockIdx.y * kTy;
    // p_EOS and psi (Eq. InteractionPotential) of the tile and its halo
    for (int q = tid; q < kLx * kLy; q += kTx * kTy) {
        const int ti = q % kLx, tj = q / kLx;
        int gi = (i0 + ti - kHalo) % A.nx;
        gi = gi < 0 ? gi + A.nx : gi;
        int gj = j0 + tj - kHalo;
        if (A.walls && gj < 0) {
            // b1 on the bottom wall (psi, rho extrapolated from rows 0 and 1), b2 inside it (Eq. B2)
            const double r0 = rho[gi], r1 = rho[(size_t)A.nx + gi];
            const double b1 = 2.0 * fd_psi(A, r0) - fd_psi(A, r1);
            spe[tj][ti] = dev_eos_p(A.eos, 2.0 * r0 - r1);
            spsi[tj][ti] = gj == -1 ? b1 : b1 + 2.0 * A.h * (A.psi_wall - b1);
            continue;
        }
        if (A.walls && gj >= A.ny) gj = max(2 * (A.ny - 1) - gj, 0);  // reflexive top layers
        gj %= A.ny;
        gj = gj < 0 ? gj + A.ny : gj;
        const double r = rho[(size_t)gj * A.nx + gi];
        const double pe = dev_eos_p(A.eos, r);
        const double qq = (pe - r * (1.0 / 3.0)) * A.two_inv_G;
        const int rj = j0 + tj - kHalo;
        if ((!A.walls || (rj >= 0 && rj < A.ny)) && (!(r > 0.0) || !(qq >= 0.0))) fd_flag(A);
        spe[tj][ti] = pe;
        spsi[tj][ti] = qq > 0.0 ? sqrt(qq) : 0.0;
    }
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= A.nx || j >= A.ny) return;
    const int li = threadIdx.x + kHalo, lj = threadIdx.y + kHalo;
    // neighbours: periodic in x; in y periodic or the wall layers (b1 below row 0: u = v = 0 and rho
    // extrapolated; above row ny-1 the mirror of row ny-2 with u, v reversed)
    const bool wbot = A.walls && j == 0, wtop = A.walls && j == A.ny - 1;
    const int ip = i + 1 == A.nx ? 0 : i + 1, im = i == 0 ? A.nx - 1 : i - 1;
    const int jp = wtop ? A.ny - 2 : (j + 1 == A.ny ? 0 : j + 1), jm = wbot ? 0 : (j == 0 ? A.ny - 1 : j - 1);
    const double fm = wbot ? 0.0 : 1.0, fp = wtop ? -1.0 : 1.0;
    const size_t nxs = (size_t)A.nx;
    const size_t c = j * nxs + i, xp = j * nxs + ip, xm = j * nxs + im, yp = jp * nxs + i, ym = jm * nxs + i;
    const size_t pp = jp * nxs + ip, pm = jm * nxs + ip, mp = jp * nxs + im, mm = jm * nxs + im;
    const double cs2 = 1.0 / 3.0;
    const double r = rho[c], ux = u[c], uy = v[c];
    const double r_yp = rho[yp], r_ym = wbot ? 2.0 * r - rho[nxs + i] : rho[ym];
    const double u_yp = fp * u[yp], u_ym = fm * u[ym], v_yp = fp * v[yp], v_ym = fm * v[ym];
    // one-sided first derivatives
    const double rx = (DIR > 0 ? rho[xp] - r : r - rho[xm]) * A.inv_h;
    const double ry = (DIR > 0 ? r_yp - r : r - r_ym) * A.inv_h;
    const double u_x = (DIR > 0 ? u[xp] - ux : ux - u[xm]) * A.inv_h, u_y = (DIR > 0 ? u_yp - ux : ux - u_ym) * A.inv_h;
    const double v_x = (DIR > 0 ? v[xp] - uy : uy - v[xm]) * A.inv_h, v_y = (DIR > 0 ? v_yp - uy : uy - v_ym) * A.inv_h;
    const double px = (DIR > 0 ? spe[lj][li + 1] - spe[lj][li] : spe[lj][li] - spe[lj][li - 1]) * A.inv_h;
    const double py = (DIR > 0 ? spe[lj + 1][li] - spe[lj][li] : spe[lj][li] - spe[lj - 1][li]) * A.inv_h;
    const double div = u_x + v_y;
    const double dr = -(r * div + ux * rx + uy * ry);
    // Eq. DynamicViscosity, Eq. RelaxationTime and Eq. FDviscosityDerivative
    double tn = A.tau_nu, dtn = 0.0;
    if (A.var_tau) {
        tn = A.tau_v + A.dtau * (r - A.rho_v_tau);
        dtn = A.dtau;
        if (tn <= A.tau_lo) { tn = A.tau_lo; dtn = 0.0; }
        if (tn >= A.tau_hi) { tn = A.tau_hi; dtn = 0.0; }
    }
    const double mu = r * cs2 * (tn - 0.5), dmu = cs2 * (tn - 0.5) + r * cs2 * dtn;
    const double muB = r * cs2 * (A.tau_e - tn), dmuB = cs2 * (A.tau_e - tn) - r * cs2 * dtn;
    const double mux = dmu * rx, muy = dmu * ry, mBx = dmuB * rx, mBy = dmuB * ry;
    // central second derivatives of the velocity
    const double u_xx = (u[xp] - 2.0 * ux + u[xm]) * A.inv_h2, u_yy = (u_yp - 2.0 * ux + u_ym) * A.inv_h2;
    const double v_xx = (v[xp] - 2.0 * uy + v[xm]) * A.inv_h2, v_yy = (v_yp - 2.0 * uy + v_ym) * A.inv_h2;
    const double u_xy = (fp * u[pp] - fm * u[pm] - fp * u[mp] + fm * u[mm]) * A.inv_4h2;
    const double v_xy = (fp * v[pp] - fm * v[pm] - fp * v[mp] + fm * v[mm]) * A.inv_4h2;
    // divergence of the viscous stress (Eq. FDstressTensor)
    const double Sx = mux * (2.0 * u_x) + muy * (v_x + u_y) + mu * (2.0 * u_xx + u_yy + v_xy) + mBx * div +
                      muB * (u_xx + v_xy);
    const double Sy = mux * (u_y + v_x) + muy * (2.0 * v_y) + mu * (v_xx + 2.0 * v_yy + u_xy) + mBy * div +
                      muB * (u_xy + v_yy);
    // Eq. FDforce, central differences of psi (the Laplacian at x+-1, y+-1 reaches two nodes out)
    const double s0 = spsi[lj][li], sxp = spsi[lj][li + 1], sxm = spsi[lj][li - 1];
    const double syp = spsi[lj + 1][li], sym = spsi[lj - 1][li];
    const double spp = spsi[lj + 1][li + 1], spm = spsi[lj - 1][li + 1], smp = spsi[lj + 1][li - 1];
    const double smm = spsi[lj - 1][li - 1];
    const double sx = (sxp - sxm) * A.inv_2h, sy = (syp - sym) * A.inv_2h;
    const double sxx = (sxp - 2.0 * s0 + sxm) * A.inv_h2, syy = (syp - 2.0 * s0 + sym) * A.inv_h2;
    const double sxy = (spp - spm - smp + smm) * A.inv_4h2;
    const double L = sxx + syy;
    const double Lxp = (spsi[lj][li + 2] - 2.0 * sxp + s0) * A.inv_h2 + (spp - 2.0 * sxp + spm) * A.inv_h2;
    const double Lxm = (s0 - 2.0 * sxm + spsi[lj][li - 2]) * A.inv_h2 + (smp - 2.0 * sxm + smm) * A.inv_h2;
    const double Lyp = (spp - 2.0 * syp + smp) * A.inv_h2 + (spsi[lj + 2][li] - 2.0 * syp + s0) * A.inv_h2;
    const double Lym = (spm - 2.0 * sym + smm) * A.inv_h2 + (s0 - 2.0 * sym + spsi[lj - 2][li]) * A.inv_h2;
    const double Lx = (Lxp - Lxm) * A.inv_2h, Ly = (Lyp - Lym) * A.inv_2h;
    const double gx = sx * sxx + sy * sxy, gy = sx * sxy + sy * syy;
    const double G = A.G;
    const double Px = -A.eps * G * 0.25 * gx + G * (1.0 / 12.0) * sx * L + G * (1.0 / 6.0) * gx + G * 0.25 * s0 * Lx;
    const double Py = -A.eps * G * 0.25 * gy + G * (1.0 / 12.0) * sy * L + G * (1.0 / 6.0) * gy + G * 0.25 * s0 * Ly;
    // Eq. FDmomentum
    const double inv_r = 1.0 / r;
    const double du = -(ux * u_x + uy * u_y) + (Sx - px - Px) * inv_r;
    const double dv = -(ux * v_x + uy * v_y) + (Sy - py - Py) * inv_r;
    const double nr = r + A.dt * dr, nu = ux + A.dt * du, nv = uy + A.dt * dv;
    if (base_r) {
        o_r[c] = wa * base_r[c] + wb * nr;
        o_u[c] = wa * base_u[c] + wb * nu;
        o_v[c] = wa * base_v[c] + wb * nv;
    } else {
        o_r[c] = nr;
        o_u[c] = nu;
        o_v[c] = nv;
    }
}

FdArgs fd_args(const lbm_fd_ctx* c)
{
    const lbm_fd_params& P = c->P;
    FdArgs A;
    std::memset(&A, 0, sizeof(A));
    A.nx = P.nx;
    A.ny = P.ny;
    A.var_tau = P.var_tau;
    A.walls = P.walls;
    A.psi_wall = c->psi_wall;
    A.h = P.h;
    A.inv_h = 1.0 / P.h;
    A.inv_2h = 0.5 / P.h;
    A.inv_h2 = 1.0 / (P.h * P.h);
    A.inv_4h2 = 0.25 / (P.h * P.h);
    A.dt = P.dt;
    A.G = P.G;
    A.two_inv_G = 2.0 / P.G;
    A.eps = P.eps;
    A.tau_e = P.tau_e;
    A.tau_nu = P.tau_nu;
    A.tau_v = P.tau_v;
    A.tau_lo = P.tau_l < P.tau_v ? P.tau_l : P.tau_v;
    A.tau_hi = P.tau_l < P.tau_v ? P.tau_v : P.tau_l;
    A.dtau = P.var_tau ? (P.tau_l - P.tau_v) / (P.rho_l_tau - P.rho_v_tau) : 0.0;
    A.rho_v_tau = P.rho_v_tau;
    A.eos = c->eos;
    A.err = c->err;
    A.step = c->step;
    return A;
}

bool ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    lbm_set_error(buf);
    return false;
}

constexpr size_t kFdArrays = 6;

}  // namespace

extern "C" {

int lbm_fd_layout(const lbm_fd_params* p, size_t* bytes)
{
    if (!p || p->nx < 3 || p->ny < 3 || !(p->h > 0) || !(p->dt > 0) || !(p->G < 0)) {
        lbm_set_error("lbm_fd_layout: need nx, ny >= 3, h > 0, dt > 0 and G < 0");
        return LBM_EINVAL;
    }
    if (bytes) *bytes = 256 + kFdArrays * (((size_t)p->nx * p->ny * sizeof(double) + 255) & ~(size_t)255);
    return LBM_OK;
}

int lbm_fd_init(lbm_fd_ctx** out, const lbm_fd_params* p, void* buf, size_t buf_bytes, const double* rho0,
                const double* u0, const double* v0, void* stream)
{
    size_t need = 0;
    if (!out || !buf || !rho0) return LBM_EINVAL;
    const int st = lbm_fd_layout(p, &need);
    if (st != LBM_OK) return st;
    if (buf_bytes < need) {
        lbm_set_error("lbm_fd_init: buffer smaller than lbm_fd_layout requires");
        return LBM_EINVAL;
    }
    if (p->var_tau && !(p->rho_l_tau > p->rho_v_tau)) {
        lbm_set_error("lbm_fd_init: Eq. RelaxationTime needs rho_l_tau > rho_v_tau");
        return LBM_EINVAL;
    }
    lbm_fd_ctx* c = new (std::nothrow) lbm_fd_ctx();
    if (!c) return LBM_EINVAL;
    c->P = *p;
    c->eos = dev_eos(p->eos);
    {
        const double q = 2.0 * (lbm_eos_pressure(&p->eos, p->eos.rho_l) - p->eos.rho_l / 3.0) / p->G;
        c->psi_wall = q > 0.0 ? std::sqrt(q) : 0.0;  // psi_l of Eq. B2
    }
    c->n = (size_t)p->nx * p->ny;
    char* b = (char*)buf;
    c->err = (unsigned*)b;
    b += 256;
    const size_t arr = (c->n * sizeof(double) + 255) & ~(size_t)255;
    double** slots[kFdArrays] = {&c->rho, &c->u, &c->v, &c->rs, &c->us, &c->vs};
    for (size_t k = 0; k < kFdArrays; ++k, b += arr) *slots[k] = (double*)b;
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = c->n * sizeof(double);
    bool good = ok(hipMemsetAsync(c->err, 0, 256, s), "fd clear") &&
                ok(hipMemcpyAsync(c->rho, rho0, nb, hipMemcpyDeviceToDevice, s), "fd rho0");
    good = good && (u0 ? ok(hipMemcpyAsync(c->u, u0, nb, hipMemcpyDeviceToDevice, s), "fd u0")
                       : ok(hipMemsetAsync(c->u, 0, nb, s), "fd u0"));
    good = good && (v0 ? ok(hipMemcpyAsync(c->v, v0, nb, hipMemcpyDeviceToDevice, s), "fd v0")
                       : ok(hipMemsetAsync(c->v, 0, nb, s), "fd v0"));
    if (!good) {
        delete c;
        return LBM_EHIP;
    }
    *out = c;
    return LBM_OK;
}

int lbm_fd_step(lbm_fd_ctx* c, int64_t nsteps, void* stream)
{
    if (!c || nsteps < 0) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const dim3 blk(kTx, kTy), grd((c->P.nx + kTx - 1) / kTx, (c->P.ny + kTy - 1) / kTy);
    for (int64_t t = 0; t < nsteps; ++t) {
        FdArgs A = fd_args(c);
        hipLaunchKernelGGL(k_fd_stage<+1>, grd, blk, 0, s, A, (const double*)c->rho, (const double*)c->u,
                           (const double*)c->v, (const double*)nullptr, (const double*)nullptr,
                           (const double*)nullptr, 0.0, 1.0, c->rs, c->us, c->vs);
        hipLaunchKernelGGL(k_fd_stage<-1>, grd, blk, 0, s, A, (const double*)c->rs, (const double*)c->us,
                           (const double*)c->vs, (const double*)c->rho, (const double*)c->u, (const double*)c->v,
                           0.5, 0.5, c->rho, c->u, c->v);
        if (!ok(hipGetLastError(), "fd step launch")) return LBM_EHIP;
        c->step++;
    }
    return LBM_OK;
}

int lbm_fd_fields(lbm_fd_ctx* c, double* rho, double* u, double* v, void* stream)
{
    if (!c) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = c->n * sizeof(double);
    bool good = true;
    if (rho) good = good && ok(hipMemcpyAsync(rho, c->rho, nb, hipMemcpyDeviceToDevice, s), "fd rho out");
    if (u) good = good && ok(hipMemcpyAsync(u, c->u, nb, hipMemcpyDeviceToDevice, s), "fd u out");
    if (v) good = good && ok(hipMemcpyAsync(v, c->v, nb, hipMemcpyDeviceToDevice, s), "fd v out");
    return good ? LBM_OK : LBM_EHIP;
}

int lbm_fd_status(lbm_fd_ctx* c, void* stream)
{
    if (!c) return LBM_EINVAL;
    unsigned h[2];
    hipStream_t s = (hipStream_t)stream;
    if (!ok(hipMemcpyAsync(h, c->err, sizeof(h), hipMemcpyDeviceToHost, s), "fd status") ||
        !ok(hipStreamSynchronize(s), "fd status sync"))
        return LBM_EHIP;
    if (h[0]) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "lbm_fd: psi^2 < 0 or non-positive density at step %u", h[1]);
        lbm_set_error(buf);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

void lbm_fd_destroy(lbm_fd_ctx* c) { delete c; }

}  // extern "C"
