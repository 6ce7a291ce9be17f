// liblbm.so: discrete adjoint of the fused D2Q9 step (gradients of a loss on
// the final density field with respect to the four knots of the shaped EOS
// loop (Sec. III.D), the interaction constant G and the Eq. LiFS sigma).
//
// The forward stores its state every K steps (lbm_set_checkpointing).  The
// adjoint walks the segments backwards: it restores a checkpoint, re-runs the
// segment with a recording step that keeps (rho - rho_ref, j, psi) per node and
// step, and then applies the transpose of each step in reverse.  One adjoint
// step is one kernel (row block of 12 waves, one lattice row per wave, 62 output
// columns per wave plus one halo column each side; the first and last waves are
// halo rows):
//   every lane  lambda^{t+1} pulled from the downstream nodes (bounce-back at
//               walls), transposed moment transform and MRT relaxation, Eq. LiFS
//               and Eq. EquilibriumDistribution derivatives -> dL/dF~ (to LDS)
//               and the local dL/dpsi;
//   interior    dL/dpsi(x) gathered from the neighbours' dL/dF~ (transpose of
//               Eq. ShanChenForce), through psi'(rho) (Eq. InteractionPotential)
//               into lambda^t; dL/dp(rho(x)) accumulates the derivatives with
//               respect to the loop coefficients, and the F~ and psi parts of
//               dL/dG and dL/dsigma are summed.
// Parameter gradients are summed in FP64 per workgroup in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_ctx.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace {

using namespace lbmk;

enum { A_PMAX, A_RMAX, A_PMIN, A_RMIN, A_B1, A_A1, A_B3, A_A3, A_G, A_SIG, kAcc };

struct AdjArgs {
    StepArgs S;          // forward parameters (EOS, rates, G, sigma, walls, shift)
    const void* lam_in;  // lambda^{t+1}: 9 planes [ny][ld]
    void* lam_out;       // lambda^t
    const void* rec;     // step t: drho, j_x, j_y, psi planes [ny][nx]
    const void* rec_lo;  // step t - 1 (two transposed steps per launch)
    double* acc;         // [blocks][kAcc] running sums
    int strips;          // column strips of kAdjW outputs
    int strips2;         // column strips of kAdj2W outputs (two steps per launch)
    size_t lplane, rplane;
    double c_e, c_q;     // 1/(tau_e - 1/2), 1/(tau_eps - 1/2) of Eq. LiFS
    double inv_G;
    // the same constants in the arithmetic type of the path
    struct K { double c_e, c_q, two_sigma, inv_G; } kd;
    struct KF { float c_e, c_q, two_sigma, inv_G; } kf;
};

template <typename T>
struct AdjK;
template <>
struct AdjK<double> {
    __device__ static const AdjArgs::K& get(const AdjArgs& A) { return A.kd; }
};
template <>
struct AdjK<float> {
    __device__ static const AdjArgs::KF& get(const AdjArgs& A) { return A.kf; }
};
template <typename T>
__device__ __forceinline__ auto adj_coef(const AdjArgs& A) -> decltype(AdjK<T>::get(A))
{
    return AdjK<T>::get(A);
}

template <typename T>
struct LocalAdj {
    T df[9];
    T dftx, dfty, dpsi;
    T dsig;
};

template <typename T>
__device__ __forceinline__ T ldT(const void* base, size_t i)
{
    return ((const T*)base)[i];
}

// 1/x for the adjoint's own divisions: the hardware estimate (FP32), or in FP64 the estimate
// refined by two Newton steps (within an ulp or two of the IEEE quotient)
__device__ __forceinline__ float arcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double arcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// node coordinates with periodic wrap in x and y (walls handled by the callers)
__device__ __forceinline__ int wrapx(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// what the transposed step at (x, y) reads of record rec: drho, j and the 3 x 3 psi stencil
// (ghost psi beyond the walls)
template <typename T>
struct RecNode {
    T dr, jx, jy;
    T p[9];  // rows y - 1, y, y + 1; columns x - 1, x, x + 1
};

template <typename T>
__device__ __forceinline__ void rec_load(const AdjArgs& A, const void* rec, int x, int y, RecNode<T>& R)
{
    const StepArgs& S = A.S;
    const size_t o = (size_t)y * S.nx + x;
    R.dr = ((const T*)rec)[o];
    R.jx = ((const T*)rec)[A.rplane + o];
    R.jy = ((const T*)rec)[2 * A.rplane + o];
    const T* ps = (const T*)rec + 3 * A.rplane;
    const int xm = x == 0 ? S.nx - 1 : x - 1, xp = x == S.nx - 1 ? 0 : x + 1;
    // the rows above and below with the periodic wrap (always in the lattice); beyond a wall
    // the loaded values are replaced by the ghost psi, so no load waits on a branch
    const T* rm = ps + (size_t)(y == 0 ? S.ny - 1 : y - 1) * S.nx;
    const T* rc = ps + (size_t)y * S.nx;
    const T* rp = ps + (size_t)(y == S.ny - 1 ? 0 : y + 1) * S.nx;
    const bool lo = S.walls && y == 0, hi = S.walls && y == S.ny - 1;
    const T glo = (T)S.psi_lo, ghi = (T)S.psi_hi;
    R.p[0] = lo ? glo : rm[xm];
    R.p[1] = lo ? glo : rm[x];
    R.p[2] = lo ? glo : rm[xp];
    R.p[3] = rc[xm];
    R.p[4] = rc[x];
    R.p[5] = rc[xp];
    R.p[6] = hi ? ghi : rp[xm];
    R.p[7] = hi ? ghi : rp[x];
    R.p[8] = hi ? ghi : rp[xp];
}

// psi and F~ (Eq. ShanChenForce) of a loaded record
template <typename T>
__device__ __forceinline__ void rec_force(const StepArgs& S, const RecNode<T>& R, T& psi, T& ftx, T& fty)
{
    psi = R.p[4];
    force_tilde<T>(S, R.p[0], R.p[1], R.p[2], R.p[3], R.p[5], R.p[6], R.p[7], R.p[8], ftx, fty);
}

// mu_i = dL/df*_i(x) = lambda^{t+1}_i(x + c_i), or lambda^{t+1}_opp(i)(x) when x + c_i is solid
template <typename T>
__device__ __forceinline__ void pull_adjoint(const AdjArgs& A, int x, int y, T mu[9])
{
    const StepArgs& S = A.S;
    const T* L = (const T*)A.lam_in;
    const size_t P = A.lplane;
    const int ld = S.ld;
    const bool top = S.walls && y == S.ny - 1, bot = S.walls && y == 0;
    const int yp = y == S.ny - 1 ? 0 : y + 1, ym = y == 0 ? S.ny - 1 : y - 1;
    const int xp = wrapx(x + 1, S.nx), xm = wrapx(x - 1, S.nx);
    const size_t r0 = (size_t)y * ld, rp = (size_t)yp * ld, rm = (size_t)ym * ld;
    mu[0] = L[r0 + x];
    mu[1] = L[1 * P + r0 + xp];
    mu[3] = L[3 * P + r0 + xm];
    mu[2] = top ? L[4 * P + r0 + x] : L[2 * P + rp + x];
    mu[5] = top ? L[7 * P + r0 + x] : L[5 * P + rp + xp];
    mu[6] = top ? L[8 * P + r0 + x] : L[6 * P + rp + xm];
    mu[4] = bot ? L[2 * P + r0 + x] : L[4 * P + rm + x];
    mu[7] = bot ? L[5 * P + r0 + x] : L[7 * P + rm + xm];
    mu[8] = bot ? L[6 * P + r0 + x] : L[8 * P + rm + xp];
}

// Transpose of the node update (moments, MRT relaxation, Eq. LiFS source,
// equilibrium, forced velocity) for fixed psi(x) and F~(x).
template <typename T>
__device__ __forceinline__ void local_adjoint(const AdjArgs& A, const T mu[9], T dr, T jx, T jy, T psi, T ftx, T fty,
                                              LocalAdj<T>& o)
{
    const StepArgs& S = A.S;
    const Coef<T>& K = coef<T>(S);
    const T rho = (T)(S.rho_ref + (double)dr);
    const T Fx = psi * ftx, Fy = psi * fty;
    const T inv = arcp(rho);
    const T ux = (jx + (T)0.5 * Fx) * inv, uy = (jy + (T)0.5 * Fy) * inv;
    // nu = D^-1 M mu  (adjoint of f* = M^T D^-1 m*)
    const T m14 = (mu[1] + mu[2]) + (mu[3] + mu[4]);
    const T m58 = (mu[5] + mu[6]) + (mu[7] + mu[8]);
    const T n0 = (mu[0] + m14 + m58) * (T)(1.0 / 9.0);
    const T n1 = (-4 * mu[0] - m14 + 2 * m58) * (T)(1.0 / 36.0);
    const T n2 = (4 * mu[0] - 2 * m14 + m58) * (T)(1.0 / 36.0);
    const T a13 = mu[1] - mu[3], a24 = mu[2] - mu[4];
    const T a5678x = (mu[5] - mu[6]) - (mu[7] - mu[8]);
    const T a5678y = (mu[5] + mu[6]) - (mu[7] + mu[8]);
    const T n3 = (a13 + a5678x) * (T)(1.0 / 6.0);
    const T n4 = (-2 * a13 + a5678x) * (T)(1.0 / 12.0);
    const T n5 = (a24 + a5678y) * (T)(1.0 / 6.0);
    const T n6 = (-2 * a24 + a5678y) * (T)(1.0 / 12.0);
    const T n7 = ((mu[1] - mu[2]) + (mu[3] - mu[4])) * (T)0.25;
    const T n8 = ((mu[5] - mu[6]) + (mu[7] - mu[8])) * (T)0.25;
    // m*_k = m_k - s_k (m_k - m^eq_k) + (1 - s_k/2) S_k: direct, equilibrium and source adjoints
    // (rate 1 for e, eps, q_x, q_y: no direct part, the equilibrium part whole, half the source)
    const bool u1 = S.unit_rates;
    const T d1 = u1 ? (T)0 : n1 * ((T)1 - K.se), E1 = u1 ? n1 : n1 * K.se, Q1 = u1 ? (T)0.5 * n1 : n1 * K.he;
    const T d2 = u1 ? (T)0 : n2 * ((T)1 - K.sq), E2 = u1 ? n2 : n2 * K.sq, Q2 = u1 ? (T)0.5 * n2 : n2 * K.hq;
    const T d4 = u1 ? (T)0 : n4 * ((T)1 - K.sqx), E4 = u1 ? n4 : n4 * K.sqx, Q4 = u1 ? (T)0.5 * n4 : n4 * K.hqx;
    const T d6 = u1 ? (T)0 : n6 * ((T)1 - K.sqy), E6 = u1 ? n6 : n6 * K.sqy, Q6 = u1 ? (T)0.5 * n6 : n6 * K.hqy;
    const T d7 = n7 * ((T)1 - K.snu), E7 = n7 * K.snu, Q7 = n7 * K.hnu;
    const T d8 = n8 * ((T)1 - K.snu), E8 = n8 * K.snu, Q8 = n8 * K.hnu;
    // conserved moments: m*_0 = rho, m*_3 = j_x + F_x, m*_5 = j_y + F_y
    T drho = n0, djx = n3, djy = n5, dFx = n3, dFy = n5;
    // equilibrium moments (Eq. EquilibriumDistribution in the moment basis)
    const T u2 = ux * ux + uy * uy;
    drho += E1 * (3 * u2 - 2) + E2 * (1 - 3 * u2) - E4 * ux - E6 * uy + E7 * (ux * ux - uy * uy) + E8 * ux * uy;
    T dux = 6 * rho * ux * (E1 - E2) - E4 * rho + 2 * rho * ux * E7 + rho * uy * E8;
    T duy = 6 * rho * uy * (E1 - E2) - E6 * rho - 2 * rho * uy * E7 + rho * ux * E8;
    // Eq. LiFS source terms
    const T q12 = 6 * (Q1 - Q2);
    dux += Fx * q12 + 2 * Fx * Q7 + Fy * Q8;
    duy += Fy * q12 - 2 * Fy * Q7 + Fx * Q8;
    dFx += ux * q12 - Q4 + 2 * ux * Q7 + uy * Q8;
    dFy += uy * q12 - Q6 - 2 * uy * Q7 + ux * Q8;
    // sigma |F~|^2 enters S_e and S_eps with 12/(tau - 1/2); z = dL/d(sigma |F~|^2)
    const T z = (T)12 * (adj_coef<T>(A).c_e * Q1 - adj_coef<T>(A).c_q * Q2);
    T dftx = adj_coef<T>(A).two_sigma * z * ftx, dfty = adj_coef<T>(A).two_sigma * z * fty;
    o.dsig = z * (ftx * ftx + fty * fty);
    // u = (j + F/2)/rho (Eq. Momentum)
    djx += dux * inv;
    djy += duy * inv;
    dFx += (T)0.5 * dux * inv;
    dFy += (T)0.5 * duy * inv;
    drho -= (dux * ux + duy * uy) * inv;
    // F = psi F~
    dftx += psi * dFx;
    dfty += psi * dFy;
    o.dpsi = dFx * ftx + dFy * fty;
    o.dftx = dftx;
    o.dfty = dfty;
    // rho = sum f, j = sum f c, m_k = sum M_ki f_i
    if (u1) {
        // d1 = d2 = d4 = d6 = 0
        o.df[0] = drho;
        const T cp = drho + d7, cm = drho - d7, dp = drho + d8, dm = drho - d8, sp = djx + djy, sm = djx - djy;
        o.df[1] = cp + djx;
        o.df[3] = cp - djx;
        o.df[2] = cm + djy;
        o.df[4] = cm - djy;
        o.df[5] = dp + sp;
        o.df[7] = dp - sp;
        o.df[6] = dm - sm;
        o.df[8] = dm + sm;
        return;
    }
    o.df[0] = drho - 4 * d1 + 4 * d2;
    const T b14 = drho - d1 - 2 * d2;
    o.df[1] = b14 + djx - 2 * d4 + d7;
    o.df[2] = b14 + djy - 2 * d6 - d7;
    o.df[3] = b14 - djx + 2 * d4 + d7;
    o.df[4] = b14 - djy + 2 * d6 - d7;
    const T b58 = drho + 2 * d1 + d2;
    o.df[5] = b58 + djx + d4 + djy + d6 + d8;
    o.df[6] = b58 - djx - d4 + djy + d6 - d8;
    o.df[7] = b58 - djx - d4 - djy - d6 + d8;
    o.df[8] = b58 + djx + d4 - djy - d6 - d8;
}

// In the loop of a Smooth / Modified Smooth EOS (Sec. III.D): adds dL/dp(rho) = P times the
// derivatives of p(rho) with respect to the loop coefficients to v.
__device__ __forceinline__ void knot_adjoint(const DevEos& E, double rho, double P, double v[kAcc])
{
    // each branch sets its four terms; the sums below use fixed indices, so that v stays in
    // registers
    double pmax = 0, pmin = 0, rmax = 0, rmin = 0, b1 = 0, a1 = 0, b3 = 0, a3 = 0;
    if (rho <= E.rho_max) {
        const double dd = rho - E.rho_max, sq = sqrt(1.0 - dd * dd * E.inv_a1sq);
        pmax = P;
        b1 = -P * (1.0 - sq);
        a1 = P * E.b1 * dd * dd * E.inv_a1sq * E.inv_a1sq / (2.0 * sq);
        rmax = P * E.b1 * dd * E.inv_a1sq / sq;
    } else if (rho < E.rho_min) {
        const double tt = (rho - E.rho_max) * E.inv_L;
        const double h = tt * tt * (3.0 - 2.0 * tt), hp = 6.0 * tt * (1.0 - tt);
        pmax = P * (1.0 - h);
        pmin = P * h;
        rmax = P * (E.p_min - E.p_max) * hp * (tt - 1.0) * E.inv_L;
        rmin = P * (E.p_min - E.p_max) * hp * (-tt) * E.inv_L;
    } else {
        const double dd = rho - E.rho_min, sq = sqrt(1.0 - dd * dd * E.inv_a3sq);
        pmin = P;
        b3 = P * (1.0 - sq);
        a3 = -P * E.b3 * dd * dd * E.inv_a3sq * E.inv_a3sq / (2.0 * sq);
        rmin = -P * E.b3 * dd * E.inv_a3sq / sq;
    }
    v[A_PMAX] += pmax;
    v[A_PMIN] += pmin;
    v[A_RMAX] += rmax;
    v[A_RMIN] += rmin;
    v[A_B1] += b1;
    v[A_A1] += a1;
    v[A_B3] += b3;
    v[A_A3] += a3;
}

__device__ __forceinline__ bool knot_node(const DevEos& E, double rho)
{
    return (E.shape == LBM_SHAPE_SMOOTH || E.shape == LBM_SHAPE_MODSMOOTH) && rho > E.rho_v && rho < E.rho_l;
}

// the loop-coefficient part of psi_adjoint alone, for a node whose dL/dpsi is known
template <typename T>
__device__ __forceinline__ void knot_adjoint_of(const AdjArgs& A, double rho, T psi, T dpsi, double v[kAcc])
{
    if (psi > (T)0 && knot_node(A.S.eos, rho)) {
        const double inv_gpsi = A.inv_G * arcp((double)psi);
        knot_adjoint(A.S.eos, rho, (double)dpsi * inv_gpsi, v);
    }
}

// dL/drho(x) through psi(rho(x)) (Eq. InteractionPotential: psi' = (p' - 1/3)/(G psi),
// dpsi/dp = 1/(G psi)) for a given dL/dpsi(x); also adds the psi part of dL/dG to vG and,
// with knots set, the loop-coefficient derivatives (knot_adjoint) to v.
template <typename T>
__device__ __forceinline__ T psi_adjoint(const AdjArgs& A, double rho, T psi, T dpsi, double* v, T& vG,
                                         bool knots = true)
{
    const StepArgs& S = A.S;
    const DevEos& E = S.eos;
    const T G = coef<T>(S).G, iG = adj_coef<T>(A).inv_G;
    T drho_eos = 0;
    if (psi > (T)0) {
        vG += dpsi * (-psi * (T)0.5 * iG);
        const bool in_loop = E.shape != LBM_SHAPE_NONE && rho > E.rho_v && rho < E.rho_l;
        if (sizeof(T) == 4 && !in_loop && E.shape != LBM_SHAPE_NONE) {
            // bulk branches in FP32, as in the forward
            const float r = (float)rho, dpb = dev_base_dpf(E, r);
            const float dp = rho <= E.rho_v ? E.fk_vap * dpb : dpb;
            drho_eos = (T)((dp - (1.0f / 3.0f)) * (float)dpsi * rcp((float)G * (float)psi));
        } else {
            const double inv_gpsi = A.inv_G * arcp((double)psi);
            drho_eos = (T)((dev_eos_dp(E, rho) - 1.0 / 3.0) * inv_gpsi * (double)dpsi);
            if (knots && knot_node(E, rho)) knot_adjoint(E, rho, (double)dpsi * inv_gpsi, v);
        }
    }
    return drho_eos;
}

// transpose of Eq. ShanChenForce at (wave k, lane l) of a row block: sum over k of
// (-G w_k c_k) . dL/dF~(x - c_k) from the LDS planes sfx, sfy (rows k-1, k, k+1)
template <typename T, int NW>
__device__ __forceinline__ T force_transpose(const StepArgs& S, const T (&sfx)[NW][64], const T (&sfy)[NW][64], int k,
                                             int lane, int y)
{
    const T G = coef<T>(S).G;
    const T g3 = -G * (T)(1.0 / 3.0), g12 = -G * (T)(1.0 / 12.0);
    const bool lo_ok = !S.walls || y >= 1, hi_ok = !S.walls || y + 1 < S.ny;
    T d = g3 * (sfx[k][lane - 1] - sfx[k][lane + 1]);
    if (lo_ok) d += g3 * sfy[k - 1][lane];
    if (hi_ok) d -= g3 * sfy[k + 1][lane];
    // diagonals: c = (1,1) from (x-1, y-1), (-1,1) from (x+1, y-1), (-1,-1) from (x+1, y+1), (1,-1) from (x-1, y+1)
    if (lo_ok)
        d += g12 * ((sfx[k - 1][lane - 1] + sfy[k - 1][lane - 1]) + (-sfx[k - 1][lane + 1] + sfy[k - 1][lane + 1]));
    if (hi_ok)
        d += g12 * ((-sfx[k + 1][lane + 1] - sfy[k + 1][lane + 1]) + (sfx[k + 1][lane - 1] - sfy[k + 1][lane - 1]));
    return d;
}

// the G dependence of the ghost psi of the solid rows (walls): psi(rho_wall) ~ G^-1/2
template <typename T>
__device__ __forceinline__ void ghost_G(const AdjArgs& A, int y, T dfty, T& vG)
{
    const StepArgs& S = A.S;
    if (S.walls && (y == 0 || y == S.ny - 1)) {
        const T G = coef<T>(S).G, iG = adj_coef<T>(A).inv_G;
        const T half = (T)0.5;  // 1/3 + 2/12
        if (y == 0) vG += (G * dfty * half) * ((T)S.psi_lo * (T)-0.5 * iG);
        if (y == S.ny - 1) vG += (-G * dfty * half) * ((T)S.psi_hi * (T)-0.5 * iG);
    }
}

constexpr int kAdjWaves = 12;            // waves (rows) per workgroup
constexpr int kAdjRows = kAdjWaves - 2;  // output rows per workgroup
constexpr int kAdjW = 62;                // output columns per wave
static_assert(kAcc <= kAdjWaves, "one wave per accumulator in the workgroup sum");

template <typename T, bool NT>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adj_blk(AdjArgs A)
{
    __shared__ T sfx[kAdjWaves][64], sfy[kAdjWaves][64];
    __shared__ double sred[kAcc][kAdjWaves][64];
    const StepArgs& S = A.S;
    const int lane = threadIdx.x & 63;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int strip = blockIdx.x % A.strips, band = blockIdx.x / A.strips;
    const int xs = strip * kAdjW - 1 + lane;  // unwrapped column of this lane
    // xs lies in [-1, nx + 61] and y in [-1, ny + 9]: one wrap each way on lattices at least
    // that wide and tall, remainders otherwise
    const int x = S.nx >= 64 ? wrapx(xs, S.nx) : ((xs % S.nx) + S.nx) % S.nx;
    const int y = band * kAdjRows - 1 + k;    // unwrapped row of this wave
    const bool fluid = S.walls ? (y >= 0 && y < S.ny) : true;
    const int yw = S.walls ? (y < 0 ? 0 : (y >= S.ny ? S.ny - 1 : y))
                           : (S.ny >= 11 ? wrapx(y, S.ny) : ((y % S.ny) + S.ny) % S.ny);
    // running sum of accumulator k of this workgroup, read early (updated at the end by lane kTotalLane of wave k)
    const double acc_prev = (k < kAcc && lane == kTotalLane) ? A.acc[(size_t)blockIdx.x * kAcc + k] : 0.0;

    T mu[9];
    pull_adjoint<T>(A, x, yw, mu);
    RecNode<T> rn;
    rec_load<T>(A, A.rec, x, yw, rn);
    T psi, ftx, fty;
    rec_force<T>(S, rn, psi, ftx, fty);
    const T dr = rn.dr;
    LocalAdj<T> L;
    local_adjoint<T>(A, mu, dr, rn.jx, rn.jy, psi, ftx, fty, L);
    sfx[k][lane] = fluid ? L.dftx : (T)0;
    sfy[k][lane] = fluid ? L.dfty : (T)0;
    __syncthreads();

    double v[kAcc] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool out = k >= 1 && k <= kAdjRows && y < S.ny && lane >= 1 && lane <= kAdjW && xs < S.nx;
    if (out) {
        const T iG = adj_coef<T>(A).inv_G;
        T vG = (ftx * L.dftx + fty * L.dfty) * iG;  // F~ = -G sum(...)
        // transpose of Eq. ShanChenForce: dL/dpsi(x) += sum_k (-G w_k c_k) . dL/dF~(x - c_k)
        const T dpsi = L.dpsi + force_transpose<T, kAdjWaves>(S, sfx, sfy, k, lane, y);
        // ghost solid neighbours x + c_k (walls): psi(rho_wall) depends on G; the x parts cancel
        ghost_G<T>(A, y, L.dfty, vG);
        // psi(rho) (Eq. InteractionPotential)
        const T drho_eos = psi_adjoint<T>(A, S.rho_ref + (double)dr, psi, dpsi, v, vG);
        v[A_G] = (double)vG;
        v[A_SIG] = (double)L.dsig;
        T* Lo = (T*)A.lam_out;
        const size_t li = (size_t)y * S.ld + x;
        for (int i = 0; i < 9; ++i) {
            // streaming stores when both lambda buffers fit in the MALL (as the forward does)
            if constexpr (NT) __builtin_nontemporal_store((T)(L.df[i] + drho_eos), Lo + i * A.lplane + li);
            else Lo[i * A.lplane + li] = L.df[i] + drho_eos;
        }
    }
    // fixed-order workgroup sum: each (accumulator, lane) column over the waves in
    // order, then one wave per accumulator sums its 64 columns
    for (int i = 0; i < kAcc; ++i) sred[i][k][lane] = v[i];
    __syncthreads();
    if (k < kAcc) {
        double s = 0.0;
        for (int w = 0; w < kAdjWaves; ++w) s += sred[k][w][lane];
        s = wave_total(s);
        if (lane == kTotalLane) A.acc[(size_t)blockIdx.x * kAcc + k] = acc_prev + s;
    }
}

// Two transposed steps per launch: lambda^{t+1} -> lambda^t -> lambda^{t-1}, with lambda^t and
// the dL/dF~ of both steps kept in LDS.  lambda^{t-1}(x) depends on lambda^{t+1} within two
// nodes of x (the pull and the transpose of Eq. ShanChenForce each reach one node) and on the
// records of both steps, so a workgroup of NW waves (one lattice row each) computes the first
// step on NW x 64 nodes, its output on the inner (NW - 2) x 62, the second step's local part on
// (NW - 4) x 60 and its output on (NW - 6) x 58: those 58-column, (NW - 6)-row tiles partition
// the lattice.  Each tile adds the parameter derivatives of its own nodes for both steps.
constexpr int kAdj2W = 58;  // output columns per wave

template <int NW>
struct Adj2Lds {
    static constexpr int R = NW - 6;  // output rows per workgroup
    static constexpr size_t lam_bytes(size_t tsz) { return 8 * NW * 64 * tsz; }
    static constexpr size_t red_bytes = (size_t)kAcc * R * 64 * sizeof(double);
    static constexpr size_t union_bytes(size_t tsz) { return lam_bytes(tsz) > red_bytes ? lam_bytes(tsz) : red_bytes; }
};

// The kernel's AdjArgs argument (the first, at offset 0 of the argument segment) through a
// pointer the compiler cannot follow: a phase that reads its constants from it reloads them
// with scalar loads instead of keeping an earlier phase's scalar registers live.
__device__ __forceinline__ const AdjArgs& reloaded_args()
{
    typedef const __attribute__((address_space(4))) AdjArgs KArgs;
    KArgs* p = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const AdjArgs*)p;
}

// the arguments for the first step's output phase: reloaded in FP32, where the kernel's scalar
// registers would otherwise spill; FP64 has room for them and keeps them (measured at 512^2:
// FP32 two-step launch 19.2 -> 17.7 us with the reload, FP64 transposed steps 4% slower)
template <typename T>
__device__ __forceinline__ const AdjArgs& first_output_args(const AdjArgs& A)
{
    if constexpr (sizeof(T) == 4) return reloaded_args();
    else return A;
}

template <typename T, bool NT, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) void k_adj2_blk(AdjArgs A)
{
    constexpr int R = Adj2Lds<NW>::R;
    __shared__ T sfx[NW][64], sfy[NW][64];
    // lambda^t, populations 1..8 ([i - 1][wave][lane]); after the second step the same
    // memory holds the workgroup sum's staging ([accumulator][output row][lane])
    __shared__ __align__(16) char ubuf[Adj2Lds<NW>::union_bytes(sizeof(T))];
    T(*lam)[NW][64] = reinterpret_cast<T(*)[NW][64]>(ubuf);
    double(*red)[R][64] = reinterpret_cast<double(*)[R][64]>(ubuf);
    const StepArgs& S = A.S;
    const int lane = threadIdx.x & 63;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int strip = blockIdx.x % A.strips2, band = blockIdx.x / A.strips2;
    const int xs = strip * kAdj2W - 3 + lane;  // unwrapped column of this lane
    // xs lies in [-3, nx + 60] and y in [-3, ny + NW - 5]: one wrap each way on lattices at
    // least 64 wide and NW tall, remainders otherwise
    const int x = S.nx >= 64 ? wrapx(xs, S.nx) : ((xs % S.nx) + S.nx) % S.nx;
    const int y = band * R - 3 + k;  // unwrapped row of this wave
    const bool fluid = S.walls ? (y >= 0 && y < S.ny) : true;
    const int yw = S.walls ? (y < 0 ? 0 : (y >= S.ny ? S.ny - 1 : y))
                           : (S.ny >= NW ? wrapx(y, S.ny) : ((y % S.ny) + S.ny) % S.ny);
    const bool own = k >= 3 && k < 3 + R && y < S.ny && lane >= 3 && lane < 3 + kAdj2W && xs < S.nx;
    const double acc_prev = (k < kAcc && lane == kTotalLane) ? A.acc[(size_t)blockIdx.x * kAcc + k] : 0.0;
    // what the first step leaves for the parameter sums of this node
    T a_psi = 0, a_dpsi = 0, a_dr = 0, a_vG = 0, a_sig = 0;

    // first step (record t), every node of the block
    T psi, ftx, fty, dr;
    LocalAdj<T> L;
    RecNode<T> rb;  // record t - 1 of this node, loaded before the first barrier
    {
        T mu[9];
        pull_adjoint<T>(A, x, yw, mu);
        RecNode<T> ra;
        rec_load<T>(A, A.rec, x, yw, ra);
        rec_force<T>(S, ra, psi, ftx, fty);
        dr = ra.dr;
        local_adjoint<T>(A, mu, dr, ra.jx, ra.jy, psi, ftx, fty, L);
    }
    if (k >= 2 && k <= NW - 3) rec_load<T>(A, A.rec_lo, x, yw, rb);
    sfx[k][lane] = fluid ? L.dftx : (T)0;
    sfy[k][lane] = fluid ? L.dfty : (T)0;
    __syncthreads();
    T lam0 = 0;  // lambda^t_0 of this node
    if (k >= 1 && k <= NW - 2) {
        if (lane >= 1 && lane <= 62) {
            const AdjArgs& B = first_output_args<T>(A);
            T vG = (ftx * L.dftx + fty * L.dfty) * adj_coef<T>(B).inv_G;
            const T dpsi = L.dpsi + force_transpose<T, NW>(B.S, sfx, sfy, k, lane, y);
            if (own) ghost_G<T>(B, y, L.dfty, vG);
            // the loop-coefficient part waits until the end (knot_adjoint_of), so that no FP64
            // sums are live through the second step
            const T drho_eos = psi_adjoint<T>(B, B.S.rho_ref + (double)dr, psi, dpsi, nullptr, vG, false);
            a_psi = psi;
            a_dpsi = dpsi;
            a_dr = dr;
            a_vG = vG;
            a_sig = L.dsig;
            lam0 = L.df[0] + drho_eos;
#pragma unroll
            for (int i = 1; i < 9; ++i) lam[i - 1][k][lane] = L.df[i] + drho_eos;
        }
    }
    __syncthreads();

    // second step (record t - 1) on waves 2 .. NW - 3: lambda^t pulled from LDS
    if (k >= 2 && k <= NW - 3) {
        T mu[9];
        const int lp = lane < 63 ? lane + 1 : 63, lm = lane > 0 ? lane - 1 : 0;
        const bool top = S.walls && y == S.ny - 1, bot = S.walls && y == 0;
        mu[0] = lam0;
        mu[1] = lam[0][k][lp];
        mu[3] = lam[2][k][lm];
        mu[2] = top ? lam[3][k][lane] : lam[1][k + 1][lane];
        mu[5] = top ? lam[6][k][lane] : lam[4][k + 1][lp];
        mu[6] = top ? lam[7][k][lane] : lam[5][k + 1][lm];
        mu[4] = bot ? lam[1][k][lane] : lam[3][k - 1][lane];
        mu[7] = bot ? lam[4][k][lane] : lam[6][k - 1][lm];
        mu[8] = bot ? lam[5][k][lane] : lam[7][k - 1][lp];
        const AdjArgs& B = reloaded_args();
        rec_force<T>(B.S, rb, psi, ftx, fty);
        dr = rb.dr;
        local_adjoint<T>(B, mu, dr, rb.jx, rb.jy, psi, ftx, fty, L);
        sfx[k][lane] = fluid ? L.dftx : (T)0;
        sfy[k][lane] = fluid ? L.dfty : (T)0;
    }
    __syncthreads();
    double v[kAcc] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (own) {
        const AdjArgs& B = reloaded_args();
        const StepArgs& SB = B.S;
        knot_adjoint_of<T>(B, SB.rho_ref + (double)a_dr, a_psi, a_dpsi, v);
        T vG = (ftx * L.dftx + fty * L.dfty) * adj_coef<T>(B).inv_G;
        const T dpsi = L.dpsi + force_transpose<T, NW>(SB, sfx, sfy, k, lane, y);
        ghost_G<T>(B, y, L.dfty, vG);
        const T drho_eos = psi_adjoint<T>(B, SB.rho_ref + (double)dr, psi, dpsi, v, vG);
        v[A_G] = (double)a_vG + (double)vG;
        v[A_SIG] = (double)a_sig + (double)L.dsig;
        T* Lo = (T*)B.lam_out;
        const size_t li = (size_t)y * SB.ld + x;
        for (int i = 0; i < 9; ++i) {
            if constexpr (NT) __builtin_nontemporal_store((T)(L.df[i] + drho_eos), Lo + i * B.lplane + li);
            else Lo[i * B.lplane + li] = L.df[i] + drho_eos;
        }
    }
    // fixed-order workgroup sum over the output rows, then one wave per accumulator sums its
    // 64 columns (the staging reuses lambda^t's LDS, read before the last barrier)
    if (k >= 3 && k < 3 + R)
        for (int i = 0; i < kAcc; ++i) red[i][k - 3][lane] = v[i];
    __syncthreads();
    if (k < kAcc) {
        double s = 0.0;
        for (int w = 0; w < R; ++w) s += red[k][w][lane];
        s = wave_total(s);
        if (lane == kTotalLane) A.acc[(size_t)blockIdx.x * kAcc + k] = acc_prev + s;
    }
}

// Seed of the adjoint for a loss on the final density and velocity: lambda^T_i(x) = dL/df_i(x, T)
// of the final pulled populations, with u = (j + F/2)/rho (Eq. Momentum), F = psi F~
// (Eq. ShanChenForce) and psi(rho) (Eq. InteractionPotential).  The psi and F~ paths couple
// neighbours (radius 1), so the row block of k_adj_blk is used: dL/dF~ of every node of the
// block (halo included) goes through LDS to the output nodes.  The G and knot derivatives
// of the final psi are added to the workgroup accumulators.
template <typename T>
__global__ __launch_bounds__(64 * kAdjWaves) void k_adj_seed_u(AdjArgs A, const void* fT, const double* dLr,
                                                               const double* dLux, const double* dLuy)
{
    __shared__ T sps[kAdjWaves][64], sfx[kAdjWaves][64], sfy[kAdjWaves][64];
    __shared__ double sred[kAcc][kAdjWaves][64];
    const StepArgs& S = A.S;
    const int lane = threadIdx.x & 63;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int strip = blockIdx.x % A.strips, band = blockIdx.x / A.strips;
    const int xs = strip * kAdjW - 1 + lane;  // unwrapped column of this lane
    // xs lies in [-1, nx + 61] and y in [-1, ny + 9]: one wrap each way on lattices at least
    // that wide and tall, remainders otherwise
    const int x = S.nx >= 64 ? wrapx(xs, S.nx) : ((xs % S.nx) + S.nx) % S.nx;
    const int y = band * kAdjRows - 1 + k;    // unwrapped row of this wave
    const bool fluid = S.walls ? (y >= 0 && y < S.ny) : true;
    const int yw = S.walls ? (y < 0 ? 0 : (y >= S.ny ? S.ny - 1 : y))
                           : (S.ny >= 11 ? wrapx(y, S.ny) : ((y % S.ny) + S.ny) % S.ny);
    const size_t o = (size_t)yw * S.nx + x;
    const double acc_prev = (k < kAcc && lane == kTotalLane) ? A.acc[(size_t)blockIdx.x * kAcc + k] : 0.0;

    // the final state at (x, yw): pulled populations, rho, j, psi; dL/dF~ = psi dL/dF, dL/dF = g / (2 rho)
    const View<T> V = make_view<T>(fT, S.plane);
    const int xm = x == 0 ? S.nx - 1 : x - 1, xp = x == S.nx - 1 ? 0 : x + 1;
    double g0;
    T g[9];
    pull<T>(V, S, x, xm, xp, yw, g0, g);
    const double dr = node_drho<T>(g0, g);
    T psi = node_psi<T>(S, dr, false);
    if (!fluid) psi = (T)(y < 0 ? S.psi_lo : S.psi_hi);
    const T rho = (T)(S.rho_ref + dr);
    const T gx = (fluid && dLux) ? (T)dLux[o] : (T)0, gy = (fluid && dLuy) ? (T)dLuy[o] : (T)0;
    const T inv = arcp(rho);
    const T dFx = (T)0.5 * gx * inv, dFy = (T)0.5 * gy * inv;
    sps[k][lane] = psi;
    sfx[k][lane] = fluid ? psi * dFx : (T)0;
    sfy[k][lane] = fluid ? psi * dFy : (T)0;
    __syncthreads();

    double v[kAcc] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool out = k >= 1 && k <= kAdjRows && y < S.ny && lane >= 1 && lane <= kAdjW && xs < S.nx;
    if (out) {
        T ftx, fty;
        force_tilde<T>(S, sps[k - 1][lane - 1], sps[k - 1][lane], sps[k - 1][lane + 1], sps[k][lane - 1],
                       sps[k][lane + 1], sps[k + 1][lane - 1], sps[k + 1][lane], sps[k + 1][lane + 1], ftx, fty);
        T jx, jy;
        node_j<T>(g, jx, jy);
        const T ux = (jx + (T)0.5 * psi * ftx) * inv, uy = (jy + (T)0.5 * psi * fty) * inv;
        const T iG = adj_coef<T>(A).inv_G;
        const T dftx = psi * dFx, dfty = psi * dFy;
        T vG = (ftx * dftx + fty * dfty) * iG;  // F~ = -G sum(...)
        const T dpsi = (dFx * ftx + dFy * fty) + force_transpose<T, kAdjWaves>(S, sfx, sfy, k, lane, y);
        ghost_G<T>(A, y, dfty, vG);
        const T drho_eos = psi_adjoint<T>(A, S.rho_ref + dr, psi, dpsi, v, vG);
        v[A_G] = (double)vG;
        // direct dependence on rho and j: du/drho = -u/rho, du/dj = 1/rho
        const T d0 = (dLr ? (T)dLr[o] : (T)0) - (gx * ux + gy * uy) * inv + drho_eos;
        const T ax = gx * inv, ay = gy * inv;
        T* Lo = (T*)A.lam_out;
        const size_t li = (size_t)y * S.ld + x;
        const size_t P = A.lplane;
        Lo[li] = d0;
        Lo[P + li] = d0 + ax;
        Lo[2 * P + li] = d0 + ay;
        Lo[3 * P + li] = d0 - ax;
        Lo[4 * P + li] = d0 - ay;
        Lo[5 * P + li] = d0 + ax + ay;
        Lo[6 * P + li] = d0 - ax + ay;
        Lo[7 * P + li] = d0 - ax - ay;
        Lo[8 * P + li] = d0 + ax - ay;
    }
    for (int i = 0; i < kAcc; ++i) sred[i][k][lane] = v[i];
    __syncthreads();
    if (k < kAcc) {
        double s = 0.0;
        for (int w = 0; w < kAdjWaves; ++w) s += sred[k][w][lane];
        s = wave_total(s);
        if (lane == kTotalLane) A.acc[(size_t)blockIdx.x * kAcc + k] = acc_prev + s;
    }
}

template <typename T>
__global__ void k_adj_seed(int nx, int ny, int ld, size_t lplane, const double* dL, void* lam)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    const T v = (T)dL[(size_t)y * nx + x];
    T* L = (T*)lam;
    for (int i = 0; i < 9; ++i) L[i * lplane + (size_t)y * ld + x] = v;
}

// dL/drho0(x) = sum_i w_i lambda^0_i(x)  (initial state f^eq(rho0, u = 0))
template <typename T>
__global__ void k_adj_rho0(int nx, int ny, int ld, size_t lplane, const void* lam, double* out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    const double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    const T* L = (const T*)lam;
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += w[i] * (double)L[i * lplane + (size_t)y * ld + x];
    out[(size_t)y * nx + x] = s;
}

__global__ void k_zero(double* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

void launch_adj_step(bool f32, bool nt, int blocks, hipStream_t s, const AdjArgs& A)
{
    const dim3 g(blocks), b(64 * kAdjWaves);
    if (f32 && nt) hipLaunchKernelGGL((k_adj_blk<float, true>), g, b, 0, s, A);
    else if (f32) hipLaunchKernelGGL((k_adj_blk<float, false>), g, b, 0, s, A);
    else if (nt) hipLaunchKernelGGL((k_adj_blk<double, true>), g, b, 0, s, A);
    else hipLaunchKernelGGL((k_adj_blk<double, false>), g, b, 0, s, A);
}

constexpr int kAdj2Waves = 16;  // waves (rows) per workgroup of the two-step transposed kernel

void launch_adj2_step(bool f32, bool nt, int blocks, hipStream_t s, const AdjArgs& A)
{
    const dim3 g(blocks), b(64 * kAdj2Waves);
    if (f32 && nt) hipLaunchKernelGGL((k_adj2_blk<float, true, kAdj2Waves>), g, b, 0, s, A);
    else if (f32) hipLaunchKernelGGL((k_adj2_blk<float, false, kAdj2Waves>), g, b, 0, s, A);
    else if (nt) hipLaunchKernelGGL((k_adj2_blk<double, true, kAdj2Waves>), g, b, 0, s, A);
    else hipLaunchKernelGGL((k_adj2_blk<double, false, kAdj2Waves>), g, b, 0, s, A);
}

struct AdjLayout {
    size_t tsz, rec_bytes, off_fT, off_lam0, off_lam1, off_acc, total;
    int strips, blocks;    // one transposed step per launch
    int strips2, blocks2;  // two per launch
    size_t nacc;           // accumulators: kAcc per workgroup of the larger grid
};

AdjLayout adj_layout(const lbm_params& p, int ld, size_t pop_bytes, int K)
{
    AdjLayout L;
    L.tsz = p.prec == LBM_FP32_SHIFTED ? sizeof(float) : sizeof(double);
    const size_t nn = (size_t)p.nx * p.ny, lp = (size_t)ld * p.ny;
    L.rec_bytes = (size_t)K * 4 * nn * L.tsz;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    L.strips = (p.nx + kAdjW - 1) / kAdjW;
    L.blocks = L.strips * ((p.ny + kAdjRows - 1) / kAdjRows);
    constexpr int R2 = Adj2Lds<kAdj2Waves>::R;
    L.strips2 = (p.nx + kAdj2W - 1) / kAdj2W;
    L.blocks2 = L.strips2 * ((p.ny + R2 - 1) / R2);
    L.nacc = (size_t)(L.blocks > L.blocks2 ? L.blocks : L.blocks2) * kAcc;
    size_t o = 0;
    L.off_fT = o;
    o += al(pop_bytes);
    L.off_lam0 = o;
    o += al(9 * lp * L.tsz);
    L.off_lam1 = o;
    o += al(9 * lp * L.tsz);
    L.off_acc = o;
    o += al(L.nacc * sizeof(double));
    L.total = o;
    return L;
}

// Transposed steps from record rec (step t) down: two per launch when the record of step t - 1
// is given (rec_lo), else one.  lambda moves from lam[li] to lam[li ^ 1].
bool adj_launch(AdjArgs& A, const void* rec, const void* rec_lo, void* lam[2], int& li, bool f32, bool nt,
                const AdjLayout& L, hipStream_t s)
{
    A.rec = rec;
    A.rec_lo = rec_lo;
    A.lam_in = lam[li];
    A.lam_out = lam[li ^ 1];
    if (rec_lo) launch_adj2_step(f32, nt, L.blocks2, s, A);
    else launch_adj_step(f32, nt, L.blocks, s, A);
    li ^= 1;
    return hip_ok(hipGetLastError(), "adjoint step launch");
}

}  // namespace

namespace lbmk {
// A second stream (default priority) for the checkpointed adjoint's recomputation, and the
// events that order it against the caller's stream: rec_ready[h] once half h of the record
// buffer holds a segment, adj_done[h] once the transposed steps have read it.  open() makes
// the new stream wait for everything already queued on the caller's stream; the destructor
// drains the stream before destroying it.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t rec_ready[2] = {nullptr, nullptr}, adj_done[2] = {nullptr, nullptr};
    hipEvent_t start = nullptr;
    bool used[2] = {false, false};  // adj_done[h] recorded
    bool open(hipStream_t caller)
    {
        if (!hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "adjoint stream")) return false;
        for (int h = 0; h < 2; ++h)
            if (!hip_ok(hipEventCreateWithFlags(&rec_ready[h], hipEventDisableTiming), "adjoint event") ||
                !hip_ok(hipEventCreateWithFlags(&adj_done[h], hipEventDisableTiming), "adjoint event"))
                return false;
        return hip_ok(hipEventCreateWithFlags(&start, hipEventDisableTiming), "adjoint event") &&
               hip_ok(hipEventRecord(start, caller), "adjoint event") &&
               hip_ok(hipStreamWaitEvent(s, start, 0), "adjoint wait");
    }
    ~AuxStream()
    {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        for (hipEvent_t e : {rec_ready[0], rec_ready[1], adj_done[0], adj_done[1], start})
            if (e) (void)hipEventDestroy(e);
    }
};
}  // namespace lbmk

extern "C" {

int lbm_adjoint_layout(const lbm_params* p, int K, size_t* rec_bytes, size_t* adj_bytes)
{
    if (!p || K < 1) {
        lbm_set_error("lbm_adjoint_layout: need parameters and K >= 1");
        return LBM_EINVAL;
    }
    int ld;
    size_t pop, ws;
    const int st = lbm_layout(p, &ld, &pop, &ws);
    if (st != LBM_OK) return st;
    const AdjLayout L = adj_layout(*p, ld, pop, K);
    if (rec_bytes) *rec_bytes = L.rec_bytes;
    if (adj_bytes) *adj_bytes = L.total;
    return LBM_OK;
}

int lbm_set_checkpointing(lbm_ctx* c, void* ckpt_buf, size_t ckpt_bytes, int K)
{
    if (!c || (K > 0 && !ckpt_buf)) return LBM_EINVAL;
    if (c->aa && K > 0) {
        lbm_set_error("lbm_set_checkpointing: the in-place AA variant has no adjoint");
        return LBM_EINVAL;
    }
    if (c->step != 0) {
        lbm_set_error("lbm_set_checkpointing: enable checkpointing before the first step");
        return LBM_ESTATE;
    }
    c->ckpt = ckpt_buf;
    c->ckpt_K = K > 0 ? K : 0;
    c->ckpt_slots = K > 0 ? (int64_t)(ckpt_bytes / c->pop_bytes) : 0;
    if (K > 0 && c->ckpt_slots < 1) {
        lbm_set_error("lbm_set_checkpointing: buffer smaller than one population buffer");
        return LBM_EINVAL;
    }
    return LBM_OK;
}

int lbm_set_recording(lbm_ctx* c, void* rec_buf, size_t rec_bytes, int64_t max_steps)
{
    if (!c || max_steps < 0 || (max_steps > 0 && !rec_buf)) return LBM_EINVAL;
    if (c->aa && max_steps > 0) {
        lbm_set_error("lbm_set_recording: the in-place AA variant has no adjoint");
        return LBM_EINVAL;
    }
    if (c->step != 0) {
        lbm_set_error("lbm_set_recording: enable recording before the first step");
        return LBM_ESTATE;
    }
    const size_t tsz = c->P.prec == LBM_FP32_SHIFTED ? sizeof(float) : sizeof(double);
    const size_t per_step = 4 * (size_t)c->P.nx * c->P.ny * tsz;
    if (max_steps > 0 && rec_bytes / per_step < (size_t)max_steps) {
        lbm_set_error("lbm_set_recording: buffer smaller than max_steps records");
        return LBM_EINVAL;
    }
    c->rec_all = max_steps > 0 ? rec_buf : nullptr;
    c->rec_steps = max_steps;
    return LBM_OK;
}

int lbm_adjoint(lbm_ctx* c, const double* dL_drho_T, void* rec_buf, size_t rec_bytes, void* adj_buf, size_t adj_bytes,
                double* grad_out, double* dL_drho0, void* stream)
{
    if (!dL_drho_T) return LBM_EINVAL;
    return lbm_adjoint_fields(c, dL_drho_T, nullptr, nullptr, rec_buf, rec_bytes, adj_buf, adj_bytes, grad_out,
                              dL_drho0, stream);
}

int lbm_adjoint_fields(lbm_ctx* c, const double* dL_drho_T, const double* dL_dux_T, const double* dL_duy_T,
                       void* rec_buf, size_t rec_bytes, void* adj_buf, size_t adj_bytes, double* grad_out,
                       double* dL_drho0, void* stream)
{
    using lbmk::AuxStream;
    if (!c || !adj_buf || !grad_out || !(dL_drho_T || dL_dux_T || dL_duy_T)) return LBM_EINVAL;
    const lbm_params& P = c->P;
    // a forward recorded from step 0 needs no recomputation
    const bool recorded = c->rec_all != nullptr && c->step >= 1 && c->step <= c->rec_steps;
    if (!recorded && (c->ckpt_K < 1 || c->step < 1 || !rec_buf)) {
        lbm_set_error("lbm_adjoint: run the forward with recording (lbm_set_recording) or checkpointing "
                      "(lbm_set_checkpointing) enabled first; checkpointing needs rec_buf");
        return LBM_ESTATE;
    }
    if (P.var_tau) {
        lbm_set_error("lbm_adjoint: density-dependent relaxation (Eq. RelaxationTime) is not differentiated");
        return LBM_EINVAL;
    }
    const int64_t T_end = c->step;
    const int K = recorded ? 1 : c->ckpt_K;
    const int64_t S = recorded ? 1 : (T_end + K - 1) / K;
    if (!recorded && S > c->ckpt_slots) return LBM_ESTATE;
    const AdjLayout L = adj_layout(P, c->ld, c->pop_bytes, K);
    if ((!recorded && rec_bytes < L.rec_bytes) || adj_bytes < L.total) {
        lbm_set_error("lbm_adjoint: record or adjoint workspace smaller than lbm_adjoint_layout requires");
        return LBM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    char* ab = (char*)adj_buf;
    const bool f32 = P.prec == LBM_FP32_SHIFTED;
    const size_t nn = (size_t)P.nx * P.ny, lp = (size_t)c->ld * P.ny;
    // keep the final forward state; the recomputation overwrites the buffers
    if (!recorded &&
        !hip_ok(hipMemcpyAsync(ab + L.off_fT, c->buf[c->cur], c->pop_bytes, hipMemcpyDeviceToDevice, s), "save f(T)"))
        return LBM_EHIP;
    void* lam[2] = {ab + L.off_lam0, ab + L.off_lam1};
    double* acc = (double*)(ab + L.off_acc);
    const size_t nacc = L.nacc;
    hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, acc, nacc);
    dim3 g1((P.nx + 127) / 128, P.ny);

    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.S = c->args;
    A.acc = acc;
    A.strips = L.strips;
    A.strips2 = L.strips2;
    A.lplane = lp;
    const bool nt = 2 * 9 * lp * L.tsz <= kStreamBytes;  // streaming lambda stores on small lattices
    A.rplane = nn;
    A.c_e = 1.0 / (P.tau[1] - 0.5);
    A.c_q = 1.0 / (P.tau[2] - 0.5);
    A.inv_G = 1.0 / P.G;
    A.kd = {A.c_e, A.c_q, 2.0 * P.sigma, A.inv_G};
    A.kf = {(float)A.c_e, (float)A.c_q, (float)(2.0 * P.sigma), (float)A.inv_G};
    if (dL_dux_T || dL_duy_T) {
        // lambda^T from the final state (still in buf[cur]: the recomputation starts after this launch)
        A.lam_out = lam[0];
        if (f32)
            hipLaunchKernelGGL(k_adj_seed_u<float>, dim3(L.blocks), dim3(64 * kAdjWaves), 0, s, A,
                               (const void*)c->buf[c->cur], dL_drho_T, dL_dux_T, dL_duy_T);
        else
            hipLaunchKernelGGL(k_adj_seed_u<double>, dim3(L.blocks), dim3(64 * kAdjWaves), 0, s, A,
                               (const void*)c->buf[c->cur], dL_drho_T, dL_dux_T, dL_duy_T);
    } else {
        if (f32) hipLaunchKernelGGL(k_adj_seed<float>, g1, dim3(128), 0, s, P.nx, P.ny, c->ld, lp, dL_drho_T, lam[0]);
        else hipLaunchKernelGGL(k_adj_seed<double>, g1, dim3(128), 0, s, P.nx, P.ny, c->ld, lp, dL_drho_T, lam[0]);
    }
    if (!hip_ok(hipGetLastError(), "adjoint seed")) return LBM_EHIP;
    int li = 0;
    if (recorded) {
        // the forward kept every step's record: transposed steps only, T_end - 1 down to 0
        for (int64_t j = T_end - 1; j >= 0; j -= j >= 1 ? 2 : 1) {
            const char* r = (const char*)c->rec_all;
            if (!adj_launch(A, r + (size_t)j * 4 * nn * L.tsz, j >= 1 ? r + (size_t)(j - 1) * 4 * nn * L.tsz : nullptr,
                            lam, li, f32, nt, L, s))
                return LBM_EHIP;
        }
    }
    // A record buffer of two segments lets the recomputation of segment k - 1 run on a
    // second stream beside the transposed steps of segment k (the segments alternate
    // between the halves): both kernels are latency-bound at the sizes the adjoint runs,
    // and each fills the issue slots the other leaves.  The recomputation touches only
    // the lattice's population buffers and its half of the records; the transposed steps
    // only lambda, the accumulators and the other half.  Both precisions: the FP64 two-step
    // transposed kernel holds a CU per workgroup and runs in two rounds at 512^2, and the
    // recomputation fills the CUs its second round leaves (measured at 512^2: 89.7 ms on one
    // stream, 84.9 ms on two; FP32 57.1 ms against 53.1 ms).
    const bool piped = !recorded && S > 1 && rec_bytes >= 2 * L.rec_bytes;
    AuxStream aux;
    if (piped && !aux.open(s)) return LBM_EHIP;
    hipStream_t sr = piped ? aux.s : s;  // the recomputation's stream
    for (int64_t k = recorded ? -1 : S - 1; k >= 0; --k) {
        const int64_t t0 = k * K;
        const int n = (int)((T_end - t0) < K ? (T_end - t0) : K);
        const int half = piped ? (int)(k & 1) : 0;
        char* seg = (char*)rec_buf + (size_t)half * L.rec_bytes;
        // the transposed steps of segment k + 2 read this half last (the first two segments
        // find it unused)
        if (piped && aux.used[half] && !hip_ok(hipStreamWaitEvent(sr, aux.adj_done[half], 0), "adjoint wait"))
            return LBM_EHIP;
        if (!hip_ok(hipMemcpyAsync(c->buf[c->cur], (char*)c->ckpt + k * c->pop_bytes, c->pop_bytes,
                                   hipMemcpyDeviceToDevice, sr),
                    "restore checkpoint"))
            return LBM_EHIP;
        c->step = t0;
        for (int j = 0; j < n;) {
            // recompute the segment's records, two steps per launch where the forward's
            // two-step kernel applies (its two records land in consecutive slots)
            void* rec = seg + (size_t)j * 4 * nn * L.tsz;
            const bool pair = c->blk2 && j + 1 < n;
            if (!(pair ? launch_record_pair(c, rec, sr) : launch_record_step(c, rec, sr))) return LBM_EHIP;
            c->cur ^= 1;
            c->step += pair ? 2 : 1;
            j += pair ? 2 : 1;
        }
        if (piped && !(hip_ok(hipEventRecord(aux.rec_ready[half], sr), "adjoint event") &&
                       hip_ok(hipStreamWaitEvent(s, aux.rec_ready[half], 0), "adjoint wait")))
            return LBM_EHIP;
        for (int j = n - 1; j >= 0; j -= j >= 1 ? 2 : 1) {
            if (!adj_launch(A, seg + (size_t)j * 4 * nn * L.tsz, j >= 1 ? seg + (size_t)(j - 1) * 4 * nn * L.tsz : nullptr,
                            lam, li, f32, nt, L, s))
                return LBM_EHIP;
        }
        if (piped) {
            if (!hip_ok(hipEventRecord(aux.adj_done[half], s), "adjoint event")) return LBM_EHIP;
            aux.used[half] = true;
        }
    }
    // restore the forward state at T
    if (!recorded &&
        !hip_ok(hipMemcpyAsync(c->buf[c->cur], ab + L.off_fT, c->pop_bytes, hipMemcpyDeviceToDevice, s), "restore f(T)"))
        return LBM_EHIP;
    c->step = T_end;
    if (dL_drho0) {
        if (f32) hipLaunchKernelGGL(k_adj_rho0<float>, g1, dim3(128), 0, s, P.nx, P.ny, c->ld, lp, (const void*)lam[li], dL_drho0);
        else hipLaunchKernelGGL(k_adj_rho0<double>, g1, dim3(128), 0, s, P.nx, P.ny, c->ld, lp, (const void*)lam[li], dL_drho0);
    }
    std::vector<double> h(nacc);
    if (!hip_ok(hipMemcpyAsync(h.data(), acc, nacc * sizeof(double), hipMemcpyDeviceToHost, s), "gradient copy") ||
        !hip_ok(hipStreamSynchronize(s), "adjoint sync"))
        return LBM_EHIP;
    // every workgroup slot of both grids (the one-step and the two-step kernel tile the
    // lattice differently; slots a grid does not reach stay zero)
    double a[kAcc] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t b = 0; b < nacc / kAcc; ++b)
        for (int k = 0; k < kAcc; ++k) a[k] += h[b * kAcc + k];
    // chain the loop coefficients (b1, a1^2), (b3, a3^2) back to the four knots
    double gk[4] = {0, 0, 0, 0};
    if (P.eos.shape == LBM_SHAPE_SMOOTH || P.eos.shape == LBM_SHAPE_MODSMOOTH) {
        double J1[2][2], J3[2][2];
        lbm_knot_jacobians(&P.eos, J1, J3);
        gk[0] = a[A_RMAX] + a[A_B1] * J1[0][0] + a[A_A1] * J1[1][0];
        gk[1] = a[A_PMAX] + a[A_B1] * J1[0][1] + a[A_A1] * J1[1][1];
        gk[2] = a[A_RMIN] + a[A_B3] * J3[0][0] + a[A_A3] * J3[1][0];
        gk[3] = a[A_PMIN] + a[A_B3] * J3[0][1] + a[A_A3] * J3[1][1];
    }
    grad_out[0] = gk[0];
    grad_out[1] = gk[1];
    grad_out[2] = gk[2];
    grad_out[3] = gk[3];
    grad_out[4] = a[A_G];
    grad_out[5] = a[A_SIG];
    return lbm_status_check(c, stream);
}

}  // extern "C"
