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
// One launch per step: each workgroup evaluates the predictor on its tile grown
// by two nodes in LDS and then the corrector on the tile, writing the new state
// to the second state buffer (the two buffers swap roles every step).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>

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

// One MacCormack step per launch.  A workgroup owns a kTx x kTy output tile.
// LDS holds the state, p_EOS and psi on the tile grown by 4 (region R4; the
// predictor at the tile grown by 2 reaches two more nodes through the
// Laplacian of psi in Eq. FDforce), then the predicted state, p_EOS and psi
// on the tile grown by 2 (region R2).  Ghost rows beyond the walls are
// written into both regions by the wall rules, so every stencil reads LDS
// with the same offsets.  Traffic per node-step: the state read once (plus
// the four-node ring, mostly from L2) and written once.
constexpr int kTx = 32, kTy = 16;
constexpr int kAx = kTx + 8, kAy = kTy + 8;   // R4
constexpr int kBx = kTx + 4, kBy = kTy + 4;   // R2

// right-hand sides of the mass equation and Eq. FDmomentum at LDS node (a, b)
// of arrays with row pitch P: one-sided first derivatives (DIR), central second
// derivatives, and Eq. FDforce from psi with central differences
template <int DIR, int P>
__device__ __forceinline__ void fd_rhs(const FdArgs& A, const double* R, const double* U, const double* V,
                                       const double* Pe, const double* S, int a, int b, double& dr, double& du,
                                       double& dv)
{
    const int c = b * P + a;
    const double cs2 = 1.0 / 3.0;
    const double r = R[c], ux = U[c], uy = V[c];
    // one-sided first derivatives
    const double rx = (DIR > 0 ? R[c + 1] - r : r - R[c - 1]) * A.inv_h;
    const double ry = (DIR > 0 ? R[c + P] - r : r - R[c - P]) * A.inv_h;
    const double u_x = (DIR > 0 ? U[c + 1] - ux : ux - U[c - 1]) * A.inv_h;
    const double u_y = (DIR > 0 ? U[c + P] - ux : ux - U[c - P]) * A.inv_h;
    const double v_x = (DIR > 0 ? V[c + 1] - uy : uy - V[c - 1]) * A.inv_h;
    const double v_y = (DIR > 0 ? V[c + P] - uy : uy - V[c - P]) * A.inv_h;
    const double px = (DIR > 0 ? Pe[c + 1] - Pe[c] : Pe[c] - Pe[c - 1]) * A.inv_h;
    const double py = (DIR > 0 ? Pe[c + P] - Pe[c] : Pe[c] - Pe[c - P]) * A.inv_h;
    const double div = u_x + v_y;
    dr = -(r * div + ux * rx + uy * ry);
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
    const double u_xx = (U[c + 1] - 2.0 * ux + U[c - 1]) * A.inv_h2, u_yy = (U[c + P] - 2.0 * ux + U[c - P]) * A.inv_h2;
    const double v_xx = (V[c + 1] - 2.0 * uy + V[c - 1]) * A.inv_h2, v_yy = (V[c + P] - 2.0 * uy + V[c - P]) * A.inv_h2;
    const double u_xy = (U[c + P + 1] - U[c - P + 1] - U[c + P - 1] + U[c - P - 1]) * A.inv_4h2;
    const double v_xy = (V[c + P + 1] - V[c - P + 1] - V[c + P - 1] + V[c - P - 1]) * A.inv_4h2;
    // divergence of the viscous stress (Eq. FDstressTensor)
    const double Sx = mux * (2.0 * u_x) + muy * (v_x + u_y) + mu * (2.0 * u_xx + u_yy + v_xy) + mBx * div +
                      muB * (u_xx + v_xy);
    const double Sy = mux * (u_y + v_x) + muy * (2.0 * v_y) + mu * (v_xx + 2.0 * v_yy + u_xy) + mBy * div +
                      muB * (u_xy + v_yy);
    // Eq. FDforce, central differences of psi (the Laplacian at x+-1, y+-1 reaches two nodes out)
    const double s0 = S[c], sxp = S[c + 1], sxm = S[c - 1], syp = S[c + P], sym = S[c - P];
    const double spp = S[c + P + 1], spm = S[c - P + 1], smp = S[c + P - 1], smm = S[c - P - 1];
    const double sx = (sxp - sxm) * A.inv_2h, sy = (syp - sym) * A.inv_2h;
    const double sxx = (sxp - 2.0 * s0 + sxm) * A.inv_h2, syy = (syp - 2.0 * s0 + sym) * A.inv_h2;
    const double sxy = (spp - spm - smp + smm) * A.inv_4h2;
    const double L = sxx + syy;
    const double Lxp = (S[c + 2] - 2.0 * sxp + s0) * A.inv_h2 + (spp - 2.0 * sxp + spm) * A.inv_h2;
    const double Lxm = (s0 - 2.0 * sxm + S[c - 2]) * A.inv_h2 + (smp - 2.0 * sxm + smm) * A.inv_h2;
    const double Lyp = (spp - 2.0 * syp + smp) * A.inv_h2 + (S[c + 2 * P] - 2.0 * syp + s0) * A.inv_h2;
    const double Lym = (spm - 2.0 * sym + smm) * A.inv_h2 + (s0 - 2.0 * sym + S[c - 2 * P]) * A.inv_h2;
    const double Lx = (Lxp - Lxm) * A.inv_2h, Ly = (Lyp - Lym) * A.inv_2h;
    const double gx = sx * sxx + sy * sxy, gy = sx * sxy + sy * syy;
    const double G = A.G;
    const double Px = -A.eps * G * 0.25 * gx + G * (1.0 / 12.0) * sx * L + G * (1.0 / 6.0) * gx + G * 0.25 * s0 * Lx;
    const double Py = -A.eps * G * 0.25 * gy + G * (1.0 / 12.0) * sy * L + G * (1.0 / 6.0) * gy + G * 0.25 * s0 * Ly;
    // Eq. FDmomentum
    const double inv_r = 1.0 / r;
    du = -(ux * u_x + uy * u_y) + (Sx - px - Px) * inv_r;
    dv = -(ux * v_x + uy * v_y) + (Sy - py - Py) * inv_r;
}

// Ghost rows of a region (pitch P, rows b with global row gj = j_base + b) from its
// fluid rows: b1 (gj = -1): rho and psi extrapolated, u = v = 0, p = p_EOS(rho_b1);
// b2 (gj = -2): psi of Eq. B2 only; above row ny-1: the mirror of rows ny-2, ny-3
// with u, v reversed.  Periodic lattices have no ghost rows.
template <int P, int NY>
__device__ __forceinline__ void fd_ghost_rows(const FdArgs& A, double* R, double* U, double* V, double* Pe,
                                              double* S, int j_base, int tid, int nthreads)
{
    for (int q = tid; q < P * NY; q += nthreads) {
        const int a = q % P, b = q / P, gj = j_base + b;
        const int c = b * P + a;
        if (gj == -1 || gj == -2) {
            const int c0 = (0 - j_base) * P + a, c1 = c0 + P;  // rows 0 and 1 (inside the region)
            const double b1 = 2.0 * S[c0] - S[c1];
            if (gj == -1) {
                R[c] = 2.0 * R[c0] - R[c1];
                U[c] = 0.0;
                V[c] = 0.0;
                Pe[c] = dev_eos_p(A.eos, R[c]);
                S[c] = b1;
            } else {
                S[c] = b1 + 2.0 * A.h * (A.psi_wall - b1);
            }
        } else if (gj >= A.ny && gj <= A.ny + 1) {
            const int cm = (2 * (A.ny - 1) - gj - j_base) * P + a;
            R[c] = R[cm];
            U[c] = -U[cm];
            V[c] = -V[cm];
            Pe[c] = Pe[cm];
            S[c] = S[cm];
        }
    }
}

template <bool NT>
__global__ __launch_bounds__(kTx * kTy) void k_fd_step(FdArgs A, const double* rho, const double* u, const double* v,
                                                       double* o_r, double* o_u, double* o_v)
{
    __shared__ double aR[kAy * kAx], aU[kAy * kAx], aV[kAy * kAx], aP[kAy * kAx], aS[kAy * kAx];
    __shared__ double bR[kBy * kBx], bU[kBy * kBx], bV[kBy * kBx], bP[kBy * kBx], bS[kBy * kBx];
    const int nt = kTx * kTy, tid = threadIdx.y * kTx + threadIdx.x;
    const int i0 = blockIdx.x * kTx, j0 = blockIdx.y * kTy;
    // 1. the state, p_EOS and psi on R4; the rows beyond the walls are filled afterwards
    for (int q = tid; q < kAx * kAy; q += nt) {
        const int a = q % kAx, b = q / kAx;
        int gi = (i0 - 4 + a) % A.nx;
        gi = gi < 0 ? gi + A.nx : gi;
        int gj = j0 - 4 + b;
        if (A.walls && (gj < 0 || gj >= A.ny)) continue;
        gj %= A.ny;
        gj = gj < 0 ? gj + A.ny : gj;
        const size_t g = (size_t)gj * A.nx + gi;
        const double r = rho[g];
        const double pe = dev_eos_p(A.eos, r);
        const double qq = (pe - r * (1.0 / 3.0)) * A.two_inv_G;
        if (!(r > 0.0) || !(qq >= 0.0)) fd_flag(A);
        aR[q] = r;
        aU[q] = u[g];
        aV[q] = v[g];
        aP[q] = pe;
        aS[q] = qq > 0.0 ? sqrt(qq) : 0.0;
    }
    __syncthreads();
    if (A.walls) {
        fd_ghost_rows<kAx, kAy>(A, aR, aU, aV, aP, aS, j0 - 4, tid, nt);
        __syncthreads();
    }
    // 2. predictor Q* = Q + dt R+(Q) on the fluid nodes of R2
    for (int q = tid; q < kBx * kBy; q += nt) {
        const int a = q % kBx, b = q / kBx, gj = j0 - 2 + b;
        if (A.walls && (gj < 0 || gj >= A.ny)) continue;
        double dr, du, dv;
        fd_rhs<+1, kAx>(A, aR, aU, aV, aP, aS, a + 2, b + 2, dr, du, dv);
        const int c = (b + 2) * kAx + a + 2;
        const double nr = aR[c] + A.dt * dr;
        bR[q] = nr;
        bU[q] = aU[c] + A.dt * du;
        bV[q] = aV[c] + A.dt * dv;
        const double pe = dev_eos_p(A.eos, nr);
        const double qq = (pe - nr * (1.0 / 3.0)) * A.two_inv_G;
        bP[q] = pe;
        bS[q] = qq > 0.0 ? sqrt(qq) : 0.0;
    }
    __syncthreads();
    if (A.walls) {
        fd_ghost_rows<kBx, kBy>(A, bR, bU, bV, bP, bS, j0 - 2, tid, nt);
        __syncthreads();
    }
    // 3. corrector Q^{n+1} = (Q + Q* + dt R-(Q*)) / 2 on the tile
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= A.nx || j >= A.ny) return;
    double dr, du, dv;
    fd_rhs<-1, kBx>(A, bR, bU, bV, bP, bS, threadIdx.x + 2, threadIdx.y + 2, dr, du, dv);
    const int cb = (threadIdx.y + 2) * kBx + threadIdx.x + 2, ca = (threadIdx.y + 4) * kAx + threadIdx.x + 4;
    const size_t g = (size_t)j * A.nx + i;
    const double nr = 0.5 * aR[ca] + 0.5 * (bR[cb] + A.dt * dr);
    const double nu = 0.5 * aU[ca] + 0.5 * (bU[cb] + A.dt * du);
    const double nv = 0.5 * aV[ca] + 0.5 * (bV[cb] + A.dt * dv);
    if constexpr (NT) {
        // streaming stores when both state buffers fit in the MALL (as the LBM kernels do)
        __builtin_nontemporal_store(nr, o_r + g);
        __builtin_nontemporal_store(nu, o_u + g);
        __builtin_nontemporal_store(nv, o_v + g);
    } else {
        o_r[g] = nr;
        o_u[g] = nu;
        o_v[g] = nv;
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
    // streaming stores when both state buffers (2 x 3 fields x 8 B per node) are small
    const bool nt = (size_t)c->P.nx * c->P.ny * 48 <= kStreamBytes;
    for (int64_t t = 0; t < nsteps; ++t) {
        FdArgs A = fd_args(c);
        if (nt)
            hipLaunchKernelGGL(k_fd_step<true>, grd, blk, 0, s, A, (const double*)c->rho, (const double*)c->u,
                               (const double*)c->v, c->rs, c->us, c->vs);
        else
            hipLaunchKernelGGL(k_fd_step<false>, grd, blk, 0, s, A, (const double*)c->rho, (const double*)c->u,
                               (const double*)c->v, c->rs, c->us, c->vs);
        if (!ok(hipGetLastError(), "fd step launch")) return LBM_EHIP;
        // the new state is in (rs, us, vs): swap the roles of the two state buffers
        std::swap(c->rho, c->rs);
        std::swap(c->u, c->us);
        std::swap(c->v, c->vs);
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
