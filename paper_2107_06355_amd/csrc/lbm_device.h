// Device building blocks of the fused D2Q9 step (included by the .hip sources of
// liblbm.so): shaped-EOS evaluation, the population pull with half-way
// bounce-back, the pseudopotential psi, the Shan-Chen force stencil and the
// MRT node update with the Li et al. source.  See lbm_step.hip for the
// kernels that assemble them.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbmk {

// build-time tuning: occupancy hint for the step kernel (waves per SIMD, 0 = none)
#ifndef LBM_WAVES_PER_EU
#define LBM_WAVES_PER_EU 0
#endif
#if LBM_WAVES_PER_EU > 0 && defined(LBM_WAVES_PER_EU_MAX)
#define LBM_OCCUPANCY_HINT __attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU, LBM_WAVES_PER_EU_MAX)))
#elif LBM_WAVES_PER_EU > 0
#define LBM_OCCUPANCY_HINT __attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU)))
#else
#define LBM_OCCUPANCY_HINT
#endif

// build-time tuning of the FP64 two-step kernel: waves per workgroup and per SIMD
#ifndef LBM_K2_WAVES_F64
#define LBM_K2_WAVES_F64 12
#endif
#ifndef LBM_K2_EU_F64
#define LBM_K2_EU_F64 6
#endif


// Kernels store their new state with the non-temporal hint when both of its buffers
// together take at most this many bytes.  Measured on MI355X: faster at 12-38 MB (512^2
// lattices in both precisions: 4%; 64 batched planar lattices: 20%; the adjoint's lambda:
// 6%; the finite-difference solver: 9%), slower at 168 MB (walled 2048 x 1024 FP32:
// 23.6 -> 27.7 us/step) and beyond.
constexpr size_t kStreamBytes = (size_t)64 << 20;

constexpr int kStripW = 62;   // interior columns per wave (lanes 0 and 63 are the psi halo)

// ----------------------------------------------------------------- device EOS
struct DevEos {
    int base, shape;
    double RT, aal, b, scale, k_vap, dP;
    double rho_v, rho_l, rho_max, rho_min;
    double p0, p_max, p_min, inv_a1sq, b1, inv_a3sq, b3, inv_L, rho_m, theta;
    float fRT, faal, fb, fscale, fk_vap, fdP;  // the bulk-branch constants rounded to FP32 (FP32 path)
};

__device__ __forceinline__ double dev_base_p(const DevEos& E, double r)
{
    if (E.base == LBM_BASE_CS) {
        const double n = 0.25 * E.b * r, m = 1.0 - n;
        return E.scale * (E.RT * r * (1.0 + n * (1.0 + n * (1.0 - n))) / (m * m * m) - E.aal * r * r);
    }
    const double br = E.b * r;
    return E.scale * (E.RT * r / (1.0 - br) - E.aal * r * r / (1.0 + br * (2.0 - br)));
}

__device__ __forceinline__ double dev_eos_p(const DevEos& E, double r)
{
    if (E.shape == LBM_SHAPE_NONE) return dev_base_p(E, r);
    if (r <= E.rho_v) return E.k_vap * dev_base_p(E, r);
    if (r >= E.rho_l) return dev_base_p(E, r) + E.dP;
    if (E.shape == LBM_SHAPE_PENG) return E.p0 + E.theta * (r - E.rho_v) * (r - E.rho_l) * (r - E.rho_m);
    if (r <= E.rho_max) {
        const double d = r - E.rho_max;
        return E.p_max - E.b1 * (1.0 - sqrt(1.0 - d * d * E.inv_a1sq));
    }
    if (r < E.rho_min) {
        const double t = (r - E.rho_max) * E.inv_L;
        return E.p_max + (E.p_min - E.p_max) * t * t * (3.0 - 2.0 * t);
    }
    const double d = r - E.rho_min;
    return E.p_min + E.b3 * (1.0 - sqrt(1.0 - d * d * E.inv_a3sq));
}

__device__ __forceinline__ double dev_base_dp(const DevEos& E, double r)
{
    if (E.base == LBM_BASE_CS) {
        const double n = 0.25 * E.b * r, m = 1.0 - n;
        const double m2 = m * m;
        return E.scale * (E.RT * (1.0 + n * (4.0 + n * (4.0 + n * (-4.0 + n)))) / (m2 * m2) - 2.0 * E.aal * r);
    }
    const double br = E.b * r, m = 1.0 - br, D = 1.0 + br * (2.0 - br);
    return E.scale * (E.RT / (m * m) - 2.0 * E.aal * r * (1.0 + br) / (D * D));
}

// dp/drho of the shaped EOS (FP64)
__device__ __forceinline__ double dev_eos_dp(const DevEos& E, double r)
{
    if (E.shape == LBM_SHAPE_NONE) return dev_base_dp(E, r);
    if (r <= E.rho_v) return E.k_vap * dev_base_dp(E, r);
    if (r >= E.rho_l) return dev_base_dp(E, r);
    if (E.shape == LBM_SHAPE_PENG) {
        const double u = r - E.rho_v, v = r - E.rho_l, w = r - E.rho_m;
        return E.theta * (u * v + v * w + w * u);
    }
    if (r <= E.rho_max) {
        const double d = r - E.rho_max;
        return -E.b1 * d * E.inv_a1sq / sqrt(1.0 - d * d * E.inv_a1sq);
    }
    if (r < E.rho_min) {
        const double t = (r - E.rho_max) * E.inv_L;
        return (E.p_min - E.p_max) * 6.0 * t * (1.0 - t) * E.inv_L;
    }
    const double d = r - E.rho_min;
    return E.b3 * d * E.inv_a3sq / sqrt(1.0 - d * d * E.inv_a3sq);
}

// ----------------------------------------------------------------- kernel arguments
// Per-lattice constants of the node update, precomputed on the host in the
// arithmetic type of the path (no per-node conversions or divisions).
template <typename T>
struct Coef {
    T se, sq, sqx, sqy, snu;   // rates 1/tau of e, eps, q_x, q_y and the shear moments (Eq. RelaxationMatrix)
    T he, hq, hqx, hqy, hnu;   // 1 - s/2 (the (I - Lambda/2) factor of the source)
    T le, lq;                  // Eq. LiFS: 12 sigma (1 - s/2) / (tau - 1/2) for e and eps
    T G, two_inv_G;            // Eq. ShanChenForce and Eq. InteractionPotential
    // node_collide's folded constants: (1 - s_nu)/4, s_nu/4, (1 - s_nu/2)/2, (1 - s_nu/2)/4 of the
    // shear moments (constant rates only), and (1 - s_e/2)/6, le/36 of the e source
    T sh1, sh2, sh3, sh4, he6, le36;
};

struct StepArgs {
    const void* src;
    void* dst;
    size_t plane;            // elements per population plane (ny * ld)
    int nx, ny, ld, walls;
    int strips, seg_h, nseg, nwork;
    int var_tau, blk;        // blk: 1 = row-block (LDS) kernel, 0 = row-march kernel
    // two-step tiles (k_step2_blk): strips and bands of the lattice, patch columns, and
    // whether the tiles run in patch order (host-computed: no integer division per workgroup)
    int strips2, bands2, pcols2, patched;
    int pw_last;             // width in strips of the last patch column (1..8)
    int rows2t;              // output rows of a two-step tile with two rows per wave (<= 2 NW - 6)
    // ceil(2^32 / d) for d = 8 strips2 (tiles per patch row) and d = pw_last > 1 (2^32 does
    // not fit for d = 1, which needs no division): n / d = umulhi(n, magic) for every n the
    // kernel divides
    unsigned prow_magic, pwl_magic;
    double G, sigma;
    double s[9];             // relaxation rates 1/tau
    double tau_v, dtau_drho, tau_lo, tau_hi, rho_v_tau;
    double rho_ref;
    double psi_lo, psi_hi;
    int unit_rates;          // tau = 1 for e, eps, q_x and q_y (node_collide skips those moments)
    Coef<double> cd;
    Coef<float> cf;
    DevEos eos;
    double* partials;        // [nwork][3] FP64 per-wave sums
    unsigned* err;           // [0] flag, [1] first failing step
    long long step;
    // lbm_macros outputs (MODE_MACROS)
    double *o_rho, *o_ux, *o_uy, *o_psi, *o_p, *o_fx, *o_fy;
    // forward record for the adjoint (MODE_RECORD): planes drho, j_x, j_y, psi of [ny][nx]
    void* rec;
    size_t rec_plane;
};

enum { MODE_STEP = 0, MODE_STEP_REDUCE = 1, MODE_MACROS = 2, MODE_RECORD = 3 };

template <typename T>
__device__ __forceinline__ const Coef<T>& coef(const StepArgs& A);
template <>
__device__ __forceinline__ const Coef<double>& coef<double>(const StepArgs& A) { return A.cd; }
template <>
__device__ __forceinline__ const Coef<float>& coef<float>(const StepArgs& A) { return A.cf; }

// reciprocal: hardware v_rcp_f32 (1 ulp) on the FP32 path, IEEE division on the FP64 path
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

__constant__ double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Initial state (Sec. III.A): the shifted population g_k = f^eq_k(rho, u) - w_k rho_ref of
// Eq. EquilibriumDistribution, in FP64.  For the rest population (k = 0) of the FP32-shifted
// storage it returns instead what the eight FP32-rounded moving populations of the same node
// leave of rho - rho_ref, so that the node mass is rho exactly from the first step on (the
// invariant the collision keeps, see node_collide).
template <typename T>
__device__ inline double init_population(int k, double rho, double ux, double uy, double rho_ref)
{
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    auto g = [&](int i) {
        const double cu = cx[i] * ux + cy[i] * uy;
        return kW[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)) - kW[i] * rho_ref;
    };
    if (k != 0 || sizeof(T) == 8) return g(k);
    double moving = 0.0;
    for (int i = 1; i < 9; ++i) moving += (double)(T)g(i);
    return (rho - rho_ref) - moving;
}

template <typename T>
struct Plane;
template <>
struct Plane<double> {
    __device__ static const double* mov(const void* base, size_t plane, int i) { return (const double*)base + i * plane; }
    __device__ static double* movw(void* base, size_t plane, int i) { return (double*)base + i * plane; }
    __device__ static const double* rest(const void* base, size_t plane) { return (const double*)base; }
    __device__ static double* restw(void* base, size_t plane) { return (double*)base; }
};
template <>
struct Plane<float> {
    // planes 1..8: float32 at (i-1)*plane; rest population: float64 after the 8 float planes
    __device__ static const float* mov(const void* base, size_t plane, int i) { return (const float*)base + (i - 1) * plane; }
    __device__ static float* movw(void* base, size_t plane, int i) { return (float*)base + (i - 1) * plane; }
    __device__ static const double* rest(const void* base, size_t plane) { return (const double*)((const float*)base + 8 * plane); }
    __device__ static double* restw(void* base, size_t plane) { return (double*)((float*)base + 8 * plane); }
};

// Read-only and writable views of one population buffer: uniform per-plane base
// pointers (scalar registers) addressed with 32-bit per-lane byte offsets.
template <typename T>
struct View {
    const char* mv[9];   // planes 1..8 of the moving populations (index 0 unused)
    const char* rest;    // rest population (FP64)
};
template <typename T>
struct WView {
    char* mv[9];
    char* rest;
};

template <typename T>
__device__ __forceinline__ View<T> make_view(const void* base, size_t plane)
{
    View<T> V;
    V.mv[0] = nullptr;
    for (int i = 1; i < 9; ++i) V.mv[i] = (const char*)Plane<T>::mov(base, plane, i);
    V.rest = (const char*)Plane<T>::rest(base, plane);
    return V;
}
template <typename T>
__device__ __forceinline__ WView<T> make_wview(void* base, size_t plane)
{
    WView<T> V;
    V.mv[0] = nullptr;
    for (int i = 1; i < 9; ++i) V.mv[i] = (char*)Plane<T>::movw(base, plane, i);
    V.rest = (char*)Plane<T>::restw(base, plane);
    return V;
}

template <typename T>
__device__ __forceinline__ T ld_at(const char* base, uint32_t elem)
{
    return *(const T*)(base + elem * (uint32_t)sizeof(T));
}

// Pull the nine populations of fluid node (x, y): f_i(x) = f*_i(x - c_i), or
// f*_opp(i)(x) when x - c_i is a solid node (half-way bounce-back).  The
// wall test depends on the row only, so the plane choice is a scalar select
// and every load keeps a scalar base with a 32-bit lane offset.
template <typename T>
__device__ __forceinline__ void pull(const View<T>& V, const StepArgs& A, int x, int xm, int xp, int y, double& g0,
                                     T g[9])
{
    const uint32_t ld = (uint32_t)A.ld;
    const uint32_t r0 = (uint32_t)y * ld;
    const bool bot = A.walls && y == 0;
    const bool top = A.walls && y == A.ny - 1;
    const uint32_t rm = (uint32_t)(y == 0 ? A.ny - 1 : y - 1) * ld;
    const uint32_t rp = (uint32_t)(y == A.ny - 1 ? 0 : y + 1) * ld;
    const uint32_t ux = (uint32_t)x, um = (uint32_t)xm, up = (uint32_t)xp;
    g0 = ld_at<double>(V.rest, r0 + ux);
    g[1] = ld_at<T>(V.mv[1], r0 + um);
    g[3] = ld_at<T>(V.mv[3], r0 + up);
    if (!(bot || top)) {
        g[2] = ld_at<T>(V.mv[2], rm + ux);
        g[5] = ld_at<T>(V.mv[5], rm + um);
        g[6] = ld_at<T>(V.mv[6], rm + up);
        g[4] = ld_at<T>(V.mv[4], rp + ux);
        g[7] = ld_at<T>(V.mv[7], rp + up);
        g[8] = ld_at<T>(V.mv[8], rp + um);
    } else {
        g[2] = bot ? ld_at<T>(V.mv[4], r0 + ux) : ld_at<T>(V.mv[2], rm + ux);
        g[5] = bot ? ld_at<T>(V.mv[7], r0 + ux) : ld_at<T>(V.mv[5], rm + um);
        g[6] = bot ? ld_at<T>(V.mv[8], r0 + ux) : ld_at<T>(V.mv[6], rm + up);
        g[4] = top ? ld_at<T>(V.mv[2], r0 + ux) : ld_at<T>(V.mv[4], rp + ux);
        g[7] = top ? ld_at<T>(V.mv[5], r0 + ux) : ld_at<T>(V.mv[7], rp + up);
        g[8] = top ? ld_at<T>(V.mv[6], r0 + ux) : ld_at<T>(V.mv[8], rp + um);
    }
}

// deviation of the node density from rho_ref, exact sum in FP64
template <typename T>
__device__ __forceinline__ double node_drho(double g0, const T g[9])
{
    return g0 + (((double)g[1] + (double)g[2]) + ((double)g[3] + (double)g[4])) +
           (((double)g[5] + (double)g[6]) + ((double)g[7] + (double)g[8]));
}

__device__ __forceinline__ void flag_unstable(const StepArgs& A, int dstep = 0)
{
    atomicOr(A.err, 1u);
    atomicMin(A.err + 1, (unsigned)(A.step + dstep));
}

// base EOS in FP32 (bulk branches of the FP32 path)
__device__ __forceinline__ float dev_base_pf(const DevEos& E, float r)
{
    if (E.base == LBM_BASE_CS) {
        const float n = 0.25f * E.fb * r, m = 1.0f - n;
        return E.fscale *
               (E.fRT * r * (1.0f + n * (1.0f + n * (1.0f - n))) * __builtin_amdgcn_rcpf(m * m * m) - E.faal * r * r);
    }
    const float br = E.fb * r;
    return E.fscale * (E.fRT * r * __builtin_amdgcn_rcpf(1.0f - br) -
                       E.faal * r * r * __builtin_amdgcn_rcpf(1.0f + br * (2.0f - br)));
}

__device__ __forceinline__ float dev_base_dpf(const DevEos& E, float r)
{
    if (E.base == LBM_BASE_CS) {
        const float n = 0.25f * E.fb * r, m = 1.0f - n;
        const float m2 = m * m;
        return E.fscale * (E.fRT * (1.0f + n * (4.0f + n * (4.0f + n * (-4.0f + n)))) * __builtin_amdgcn_rcpf(m2 * m2) -
                           2.0f * E.faal * r);
    }
    const float br = E.fb * r, m = 1.0f - br, D = 1.0f + br * (2.0f - br);
    return E.fscale * (E.fRT * __builtin_amdgcn_rcpf(m * m) - 2.0f * E.faal * r * (1.0f + br) * __builtin_amdgcn_rcpf(D * D));
}

// psi (Eq. InteractionPotential, c = 1) of a node with density rho_ref + drho.
// FP64 path: everything in FP64.  FP32 path: the bulk vapor/liquid branches in
// FP32, the shaped loop between rho_v and rho_l (the branch junctions) in FP64;
// the square root is the hardware one (within 1 ulp, no correction sequence).
template <typename T>
__device__ __forceinline__ T node_psi(const StepArgs& A, const DevEos& E, double drho, bool check, int dstep = 0)
{
    const double rho = A.rho_ref + drho;
    if (sizeof(T) == 4 && E.shape != LBM_SHAPE_NONE && (rho <= E.rho_v || rho >= E.rho_l)) {
        const float r = (float)rho;
        const float pb = dev_base_pf(E, r);
        const float p = rho <= E.rho_v ? E.fk_vap * pb : pb + E.fdP;
        const float q = (p - r * (1.0f / 3.0f)) * A.cf.two_inv_G;
        if (check && !(q >= 0.0f && r > 0.0f)) flag_unstable(A, dstep);
        return (T)(q > 0.0f ? __builtin_amdgcn_sqrtf(q) : 0.0f);
    }
    const double p = dev_eos_p(E, rho);
    const double q = (p - rho * (1.0 / 3.0)) * A.cd.two_inv_G;
    if (check && !(q >= 0.0 && rho > 0.0)) flag_unstable(A, dstep);
    if (sizeof(T) == 4) return (T)(q > 0.0 ? __builtin_amdgcn_sqrtf((float)q) : 0.0f);
    return (T)(q > 0.0 ? sqrt(q) : 0.0);
}
template <typename T>
__device__ __forceinline__ T node_psi(const StepArgs& A, double drho, bool check, int dstep = 0)
{
    return node_psi<T>(A, A.eos, drho, check, dstep);
}

// 32-bit DPP move of each half of a double; lanes without a source (or outside the row mask
// ROWS) read 0
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum of v over the 64 lanes of a wave (all active), valid in lane kTotalLane, in a fixed
// order: a scan within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals
// carried by row_bcast 15 and 31.  Six DPP steps and no LDS round trip.
constexpr int kTotalLane = 63;
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_d<0x111, 0xf>(v);
    v += dpp_d<0x112, 0xf>(v);
    v += dpp_d<0x114, 0xf>(v);
    v += dpp_d<0x118, 0xf>(v);
    v += dpp_d<0x142, 0xa>(v);
    v += dpp_d<0x143, 0xc>(v);
    return v;
}

template <typename T>
struct Row {
    double g0;
    T g[9];
};

struct Lane {
    int lane, x, xm, xp;
    bool valid, interior;
};

struct Acc {
    double m, x, y;
};

// row index that is always safe to load: periodic wrap, or clamped at walls
__device__ __forceinline__ int load_index(const StepArgs& A, int r)
{
    if (A.walls) return r < 0 ? 0 : (r >= A.ny ? A.ny - 1 : r);
    return r < 0 ? r + A.ny : (r >= A.ny ? r % A.ny : r);
}

// Collide row y (populations P, density deviation drp) with psi of rows y-1, y, y+1.
// Node update of an interior lane: moments, forced velocity, MRT relaxation with
// the Eq. LiFS source, inverse transform and store (or the macroscopic outputs).
// psB = psi(x, y); Ftx, Fty = F~ = F/psi(x) from Eq. ShanChenForce.
// pre-collision state the adjoint of a step needs at node o: drho, j (unforced), psi
// (streaming stores: a record is read back only by the adjoint, long after)
template <typename T>
__device__ __forceinline__ void record_node(void* rec, size_t plane, size_t o, T dr, T jx, T jy, T psi)
{
    T* rc = (T*)rec;
    __builtin_nontemporal_store(dr, rc + o);
    __builtin_nontemporal_store(jx, rc + plane + o);
    __builtin_nontemporal_store(jy, rc + 2 * plane + o);
    __builtin_nontemporal_store(psi, rc + 3 * plane + o);
}

// unforced momentum j of pulled populations g (the moment rows of Eq. MatrixMRT)
template <typename T>
__device__ __forceinline__ void node_j(const T* gp, T& jx, T& jy)
{
    jx = (gp[1] - gp[3]) + ((gp[5] - gp[6]) - (gp[7] - gp[8]));
    jy = (gp[2] - gp[4]) + ((gp[5] + gp[6]) - (gp[7] + gp[8]));
}

template <typename T, int MODE>
__device__ __forceinline__ bool node_collide(const StepArgs& A, const Lane& L, int y, const Row<T>& P, double drp,
                                             T psB, T Ftx, T Fty, Acc& acc, T o[9], double& o0)
{
    const T* gp = P.g;
    const int x = L.x;
    const double rho_d = A.rho_ref + drp;
    const T rho = (T)rho_d;
    const T dr = (T)drp;
    const T Fx = psB * Ftx, Fy = psB * Fty;
    const T g0t = (T)P.g0;
    // moments m = M g (Eq. MatrixMRT rows)
    const T s14 = (gp[1] + gp[2]) + (gp[3] + gp[4]);
    const T s58 = (gp[5] + gp[6]) + (gp[7] + gp[8]);
    T jx, jy;
    node_j<T>(gp, jx, jy);
    const T mxx = (gp[1] - gp[2]) + (gp[3] - gp[4]);
    const T mxy = (gp[5] - gp[6]) + (gp[7] - gp[8]);
    // forced velocity (Eq. Momentum)
    const T inv_rho = rcp(rho);
    const T ux = (jx + (T)0.5 * Fx) * inv_rho, uy = (jy + (T)0.5 * Fy) * inv_rho;

    if (MODE == MODE_MACROS) {
        const size_t o = (size_t)y * A.nx + x;
        if (A.o_rho) A.o_rho[o] = rho_d;
        if (A.o_ux) A.o_ux[o] = (double)ux;
        if (A.o_uy) A.o_uy[o] = (double)uy;
        if (A.o_psi) A.o_psi[o] = (double)psB;
        if (A.o_p) A.o_p[o] = dev_eos_p(A.eos, rho_d);
        if (A.o_fx) A.o_fx[o] = (double)Fx;
        if (A.o_fy) A.o_fy[o] = (double)Fy;
    }
    if (MODE == MODE_RECORD) record_node<T>(A.rec, A.rec_plane, (size_t)y * A.nx + x, dr, jx, jy, psB);
    if (MODE == MODE_STEP_REDUCE || MODE == MODE_MACROS) {
        acc.m += rho_d;
        acc.x += (double)rho * (double)ux;
        acc.y += (double)rho * (double)uy;
    }
    if (MODE == MODE_MACROS) return false;
    // rates (Eq. RelaxationMatrix; Eq. RelaxationTime on the shear moments)
    const Coef<T>& K = coef<T>(A);
    T sh1 = K.sh1, sh2 = K.sh2, sh3 = K.sh3, sh4 = K.sh4;
    if (A.var_tau) {
        double tau = A.tau_v + A.dtau_drho * (rho_d - A.rho_v_tau);
        tau = fmin(fmax(tau, A.tau_lo), A.tau_hi);
        const T snu = (T)(1.0 / tau), hnu = (T)1 - (T)0.5 * snu;
        sh1 = ((T)1 - snu) * (T)0.25;
        sh2 = snu * (T)0.25;
        sh3 = hnu * (T)0.5;
        sh4 = hnu * (T)0.25;
    }
    const T u2 = ux * ux + uy * uy;
    const T uF = ux * Fx + uy * Fy;
    const T F2 = Ftx * Ftx + Fty * Fty;  // |F|^2/psi^2
    // equilibrium deviation moments (M f^eq minus the rho_ref rest state)
    const T eqxx = rho * (ux * ux - uy * uy);
    const T eqxy = rho * ux * uy;
    // relaxed moments m* = m - Lambda (m - m^eq) + (I - Lambda/2) S, folded into the parts of
    // f* = M^T D m* that the pairs of populations share: a14 (1-4) and a58 (5-8) isotropic,
    // px, py (axis pairs) and X, Y (diagonal pairs) from j* and q*
    const T n0 = dr * (T)(1.0 / 9.0);
    const T jFx = jx + Fx, jFy = jy + Fy;  // j* = j + F
    T a14, a58, px, py, X, Y;
    if (A.unit_rates) {
        // rate 1 for e, eps, q_x, q_y: m* = m^eq + (I - Lambda/2) S for them, whatever m is,
        // so those four moments of the populations are not formed.  With tau_e = tau_eps the
        // eps source is -S_e (Eq. LiFS), and with e^eq = -2 drho + 3 rho u^2, eps^eq = drho -
        // 3 rho u^2 the isotropic parts reduce to drho/9 + Z and drho/36 + Z, Z = (3 rho u^2 +
        // S_e)/36.  q^eq = -rho u = -(j + F/2) (Eq. Momentum) and (1 - s/2) F = F/2 give q* =
        // -(j + F): the j and q parts of each pair add up to (j + F)/3 on the axes and
        // (j + F)/12 on the diagonals.
        const T Z = (rho * u2) * (T)(1.0 / 12.0) + (uF * K.he6 + F2 * K.le36);
        a14 = n0 + Z;
        a58 = dr * (T)(1.0 / 36.0) + Z;
        px = jFx * (T)(1.0 / 3.0);
        py = jFy * (T)(1.0 / 3.0);
        X = jFx * (T)(1.0 / 12.0);
        Y = jFy * (T)(1.0 / 12.0);
    } else {
        const T njx = jFx * (T)(1.0 / 6.0), njy = jFy * (T)(1.0 / 6.0);
        // Eq. LiFS sources of e and eps, multiplied by (I - Lambda/2)
        const T Se = (T)6 * uF * K.he + K.le * F2;
        const T eqe = -2 * dr + 3 * rho * u2;
        const T eqq = dr - 3 * rho * u2;
        const T Sq = -(T)6 * uF * K.hq - K.lq * F2;
        const T me = -4 * g0t - s14 + 2 * s58;
        const T mq = 4 * g0t - 2 * s14 + s58;
        const T mqx = -2 * (gp[1] - gp[3]) + ((gp[5] - gp[6]) - (gp[7] - gp[8]));
        const T mqy = -2 * (gp[2] - gp[4]) + ((gp[5] + gp[6]) - (gp[7] + gp[8]));
        const T ne = (me - K.se * (me - eqe) + Se) * (T)(1.0 / 36.0);
        const T nq = (mq - K.sq * (mq - eqq) + Sq) * (T)(1.0 / 36.0);
        const T nqx = (mqx - K.sqx * (mqx + rho * ux) - K.hqx * Fx) * (T)(1.0 / 12.0);
        const T nqy = (mqy - K.sqy * (mqy + rho * uy) - K.hqy * Fy) * (T)(1.0 / 12.0);
        a14 = n0 - ne - 2 * nq;
        a58 = n0 + 2 * ne + nq;
        px = njx - 2 * nqx;
        py = njy - 2 * nqy;
        X = njx + nqx;
        Y = njy + nqy;
    }
    // shear moments (Eq. RelaxationTime when var_tau): (m - s (m - m^eq) + (1 - s/2) S) / 4
    const T nxx = mxx * sh1 + (eqxx * sh2 + (ux * Fx - uy * Fy) * sh3);
    const T nxy = mxy * sh1 + (eqxy * sh2 + (ux * Fy + uy * Fx) * sh4);
    // f* = M^-1 m* = M^T diag(1/9,1/36,1/36,1/6,1/12,1/6,1/12,1/4,1/4) m*
    // the rows of M^T pair up as +-: each pair shares its sum and difference terms
    const T c13 = a14 + nxx, c24 = a14 - nxx;
    o[1] = c13 + px;
    o[3] = c13 - px;
    o[2] = c24 + py;
    o[4] = c24 - py;
    const T dp = a58 + nxy, dm = a58 - nxy, sp = X + Y, sm = X - Y;
    o[5] = dp + sp;
    o[7] = dp - sp;
    o[6] = dm - sm;
    o[8] = dm + sm;
    // rest population: exact node mass in FP64 (conserved by the collision)
    o0 = drp - ((((double)o[1] + (double)o[2]) + ((double)o[3] + (double)o[4])) +
                (((double)o[5] + (double)o[6]) + ((double)o[7] + (double)o[8])));
    return true;
}

// node_collide, then the store of f* at (x, y) of the destination buffer
template <typename T, int MODE, bool NT = false>
__device__ __forceinline__ void update_node(const StepArgs& A, const Lane& L, int y, const Row<T>& P, double drp,
                                            T psB, T Ftx, T Fty, Acc& acc)
{
    T o[9];
    double o0;
    if (!node_collide<T, MODE>(A, L, y, P, drp, psB, Ftx, Fty, acc, o, o0)) return;
    const WView<T> D = make_wview<T>(A.dst, A.plane);
    const uint32_t off = (uint32_t)y * (uint32_t)A.ld + (uint32_t)L.x;
    if constexpr (NT) {
        // streaming stores (the callers choose them for small lattices: kStreamBytes)
#pragma unroll
        for (int i = 1; i < 9; ++i) __builtin_nontemporal_store(o[i], (T*)(D.mv[i] + off * (uint32_t)sizeof(T)));
        __builtin_nontemporal_store(o0, (double*)(D.rest + off * 8u));
    } else {
#pragma unroll
        for (int i = 1; i < 9; ++i) *(T*)(D.mv[i] + off * (uint32_t)sizeof(T)) = o[i];
        *(double*)(D.rest + off * 8u) = o0;
    }
}

// Eq. ShanChenForce / psi(x): F~ = -G sum_i w(|c_i|^2) psi(x + c_i) c_i, written as
// differences; arguments are psi at (x-1, x, x+1) of rows y-1 (m), y (c), y+1 (n).
template <typename T>
__device__ __forceinline__ void force_tilde(const StepArgs& A, T lm, T cm, T rm_, T lc, T rc, T ln, T cn, T rn_,
                                            T& Ftx, T& Fty)
{
    const T G = coef<T>(A).G;
    const T third = (T)(1.0 / 3.0), twelfth = (T)(1.0 / 12.0);
    Ftx = -G * ((rc - lc) * third + ((rn_ - ln) + (rm_ - lm)) * twelfth);
    Fty = -G * ((cn - cm) * third + ((rn_ + ln) - (rm_ + lm)) * twelfth);
}

// Collide row y of a marching wave: psi of the x-neighbours comes from the
// adjacent lanes (all lanes take part in the shuffles).
template <typename T, int MODE>
__device__ __forceinline__ void collide_row(const StepArgs& A, const Lane& L, int y, const Row<T>& P, double drp,
                                            T psA, T psB, T ps, Acc& acc)
{
    const T lm = __shfl(psA, L.lane - 1, 64), rm_ = __shfl(psA, L.lane + 1, 64);
    const T lc = __shfl(psB, L.lane - 1, 64), rc = __shfl(psB, L.lane + 1, 64);
    const T ln = __shfl(ps, L.lane - 1, 64), rn_ = __shfl(ps, L.lane + 1, 64);
    T Ftx, Fty;
    force_tilde<T>(A, lm, psA, rm_, lc, rc, ln, ps, rn_, Ftx, Fty);
    if (!L.interior) return;
    update_node<T, MODE>(A, L, y, P, drp, psB, Ftx, Fty, acc);
}


// Two time steps per launch (temporal blocking).  A
// workgroup of NW waves owns an output tile of NW - 6 rows x 58 columns; wave k
// holds row y0-3+k and lane l column x0-3+l in every phase, so the tile grown
// by d nodes is the set of (wave, lane) pairs at distance <= d from it:
//   1. pull step t from the source buffer on the tile grown by 3; rho, psi(t) -> LDS
//   2. collide step t on the tile grown by 2 (psi of the 3x3 stencil from LDS);
//      the post-collision populations go to LDS in their storage format
//   3. pull step t+1 from LDS on the tile grown by 1; rho, psi(t+1) -> LDS
//   4. collide step t+1 on the tile and store to the destination buffer.
// With walls the rows beyond them are solid: they carry the ghost psi of
// Eq. ShanChenForce, and the pulls at the wall rows bounce back half-way.
// Every node runs the arithmetic of the one-step kernels, and LDS holds the
// intermediate state exactly as global memory would (FP32 deviations, FP64
// rest population), so one launch equals two one-step launches.  Memory
// traffic per output node is one population read (plus the 3-node ring) and
// one write per two steps.  MODE_RECORD also stores, for the tile's nodes,
// what the adjoint of each of the two steps needs (rho - rho_ref, j, psi).
// Waves per two-step workgroup (tile rows = waves - 6): FP32 16, two workgroups per CU at
// 8 waves per SIMD; FP64 12, two workgroups per CU at the 77 VGPRs the FP64 path needs
// (measured on MI355X: FP64 8192^2 1468 vs 1553 us/step with 16 waves; FP32 loses with 12).
template <typename T>
constexpr int k2WavesOf = sizeof(T) == 4 ? 16 : LBM_K2_WAVES_F64;
inline int k2waves_of_prec(int prec) { return prec == LBM_FP32_SHIFTED ? k2WavesOf<float> : k2WavesOf<double>; }
constexpr int k2Cols = 64 - 6;
// Two rows per wave (step2_tile_rows, k_step2_rows2): a workgroup of NW waves holds the 2 NW
// rows of its tile grown by 3 (wave k holds rows k and k + NW), so the tile is 2 NW - 6 rows
// tall and the ring rows both steps recompute are a smaller share of its work: per output
// row, 2.4 collisions and 2.8 pulls for 16 waves x 1 row, 2.2 and 2.4 for 12 x 2.  FP32: 12
// waves (18-row tiles, 63 KB of LDS, two workgroups per CU); FP64: 8 waves (10-row tiles
// instead of the 6 rows of 12 x 1, 73 KB, two per CU).  Measured on MI355X (two A/B runs per
// precision): FP64 2048^2 .. 16384^2 8.5 - 17% faster, 512^2 8% faster, the walled 2048 x 1024
// impact 2%; FP32 4096^2 .. 16384^2 13 - 17% faster, 2048^2 2.5%, but the impact lattice (4
// rounds and 4 workgroups of the chip's 512 slots) no faster and 512^2 (261 tiles on 256 CUs)
// 30% slower.  So FP32 takes two-row tiles on lattices of at least kRows2MinTiles of them.
template <typename T>
constexpr int k2rWavesOf = sizeof(T) == 4 ? 12 : 8;
template <typename T>
constexpr int k2rRowsOf = 2 * k2rWavesOf<T> - 6;
constexpr int kRows2MinTiles = 4096;
// Workgroups the chip runs at once with two two-step workgroups per CU (256 CUs).
constexpr int kTwoStepSlots = 512;
// waves per workgroup and output rows of the single-lattice two-step tile, and whether it
// has two rows per wave
struct TwoStepShape {
    int waves, rows;
    bool rows2;
};
// the shape of an explicit tile height h (lbm_params.tile_rows > 0)
inline TwoStepShape shape_of_height(bool f32, int h)
{
    if (f32 && h == k2WavesOf<float> - 6) return {k2WavesOf<float>, h, false};
    return {f32 ? k2rWavesOf<float> : k2rWavesOf<double>, h, true};
}
// Heights lbm_params.tile_rows may name: FP32 10 (one row per wave) .. 18, FP64 5 .. 10.
inline bool tile_rows_valid(const lbm_params& p)
{
    if (p.tile_rows == 0 || p.tile_rows == -1) return true;
    const bool f32 = p.prec == LBM_FP32_SHIFTED;
    const int lo = f32 ? k2WavesOf<float> - 6 : k2rRowsOf<double> / 2, hi = f32 ? k2rRowsOf<float> : k2rRowsOf<double>;
    return p.tile_rows >= lo && p.tile_rows <= hi;
}
// The library's choice (tile_rows 0, and the shape before timing for -1): FP64 two-row tiles
// of 10 rows; FP32 one-row tiles of 10 rows, or two-row tiles of 18 on lattices of at least
// kRows2MinTiles of them (measured: see k2rWavesOf).
inline TwoStepShape two_step_shape(const lbm_params& p)
{
    const bool f32 = p.prec == LBM_FP32_SHIFTED;
    if (p.tile_rows > 0) return shape_of_height(f32, p.tile_rows);
    if (!f32) return {k2rWavesOf<double>, k2rRowsOf<double>, true};
    const long long strips = (p.nx + k2Cols - 1) / k2Cols;
    if (strips * ((p.ny + k2rRowsOf<float> - 1) / k2rRowsOf<float>) >= kRows2MinTiles)
        return {k2rWavesOf<float>, k2rRowsOf<float>, true};
    return {k2WavesOf<float>, k2WavesOf<float> - 6, false};
}
// Candidates lbm_init times for tile_rows = -1, the library's choice first.  How the tiles of a
// launch fill the chip's rounds of workgroups, its XCDs and its L2s makes the best height
// depend on the lattice by up to 9% (measured on MI355X, FP32: the walled 2048 x 1024 impact
// 47.6 us per launch with 16-row tiles against 49.7 with 18 and 51.2 with one-row tiles;
// 4096 x 2048 184.5 us with 17 rows against 201.7 with 18 and 213.7 with 16; 8192^2 best with
// 18).  Lattices the chip runs in one round keep the library's choice.
constexpr int kMaxShapes = 8;
inline int two_step_candidates(const lbm_params& p, TwoStepShape out[kMaxShapes])
{
    const bool f32 = p.prec == LBM_FP32_SHIFTED;
    int n = 0;
    out[n++] = two_step_shape(p);
    if (p.tile_rows != -1) return n;
    const long long strips = (p.nx + k2Cols - 1) / k2Cols;
    const int hmax = f32 ? k2rRowsOf<float> : k2rRowsOf<double>;
    if (strips * ((p.ny + hmax - 1) / hmax) <= kTwoStepSlots) return n;
    const int lo = f32 ? hmax - 4 : hmax - 3;
    auto add = [&](TwoStepShape sh) {
        for (int i = 0; i < n; ++i)
            if (out[i].rows == sh.rows && out[i].rows2 == sh.rows2) return;
        out[n++] = sh;
    };
    if (f32) add({k2WavesOf<float>, k2WavesOf<float> - 6, false});
    for (int h = hmax; h >= lo; --h) add(shape_of_height(f32, h));
    return n;
}

// Order of the two-step tiles within the range of tiles one XCD runs (k_step2_blk maps
// blockIdx to XCD-contiguous ranges): patches of 8 strips x 8 bands, patch rows from the top,
// patches left to right, tiles band-major inside a patch.  The last patch column is as wide
// as the strips left (1 to 8), so a patch row holds 8 x strips slots and only the bands past
// the lattice in the last patch row are empty slots.  The 64 workgroups an XCD runs at once
// (32 CUs x 2) then cover one patch, and the three-node ring each tile re-reads above, below
// and beside it belongs to tiles of the same patch that were just loaded into that XCD's L2.
// Band-major order over whole lattice rows leaves the ring rows above and below to HBM once
// a lattice row of tiles outgrows the L2.  Measured at 8192^2 (MI355X, PMC), band-major ->
// patches: FP64 reads 144 -> 84 B per cell and launch, FP32 63 -> 45 B (the floor is 72 and 40).
constexpr int kPatchW = 8, kPatchH = 8;
// Lattices of at most this many tiles run in one or two rounds of the chip's 512 workgroup
// slots; their tile order does not decide what the L2 holds, and they keep band-major order.
// So do lattices under two patches wide or tall: band-major order already keeps their ring
// in L2, and short lattices would leave most slots of their one patch row empty.
constexpr int kPatchMinTiles = 1024;
inline int patch_grid(int strips, int bands, bool patched)
{
    if (!patched) return (strips * bands + 7) & ~7;
    return (((bands + kPatchH - 1) / kPatchH) * kPatchH * strips + 7) & ~7;
}
// tile of XCD-contiguous slot `logical`; false when the slot has none
__device__ __forceinline__ bool two_step_tile(const StepArgs& A, int logical, int& strip, int& band)
{
    if (A.patched) {
        const unsigned pr = __umulhi((unsigned)logical, A.prow_magic);  // patch row
        const int rem = logical - (int)pr * (kPatchH * A.strips2);
        const int pc = rem / (kPatchW * kPatchH);                         // patch column
        if (pc < A.pcols2 - 1) {
            strip = pc * kPatchW + rem % kPatchW;
            band = (int)pr * kPatchH + (rem % (kPatchW * kPatchH)) / kPatchW;
        } else {
            const int w = rem - (A.pcols2 - 1) * (kPatchW * kPatchH);
            const int q = A.pw_last == 1 ? w : (int)__umulhi((unsigned)w, A.pwl_magic);
            strip = (A.pcols2 - 1) * kPatchW + (w - q * A.pw_last);
            band = (int)pr * kPatchH + q;
        }
        return band < A.bands2;
    }
    band = logical / A.strips2;
    strip = logical - band * A.strips2;
    return logical < A.strips2 * A.bands2;
}

// LDS of one two-step tile
template <typename T>
struct Step2Lds {
    DevEos eos;                          // the lattice's EOS record (read by node_psi)
    T sps[k2WavesOf<T>][64];            // psi of the tile grown by 3 (step t), then by 1 (step t+1)
    T smv[8][k2WavesOf<T> - 2][64];     // post-collision moving populations of step t (tile grown by 2)
    double sg0[k2WavesOf<T> - 2][64];   // and their FP64 rest population
    double sred[k2WavesOf<T>][3];       // a reducing launch's wave totals (mass, momentum)
};

// Advance output tile (strip, band) of lattice A by two steps (see above).
template <typename T, int MODE, bool WALLS, bool NT = false>
__device__ __forceinline__ void step2_tile(const StepArgs& A, int strip, int band, Step2Lds<T>& S)
{
    auto& sps = S.sps;
    auto& smv = S.smv;
    auto& sg0 = S.sg0;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    constexpr int k2Rows = k2WavesOf<T> - 6;
    const int x0 = strip * k2Cols, y0 = band * k2Rows;
    const int W = min(k2Cols, A.nx - x0), H = min(k2Rows, A.ny - y0);
    // distance of this lane's column and this wave's row from the output tile
    const int dl = l < 3 ? 3 - l : (l > W + 2 ? l - (W + 2) : 0);
    const int dk = k < 3 ? 3 - k : (k > H + 2 ? k - (H + 2) : 0);
    const int d = max(dl, dk);
    Lane L;
    L.lane = l;
    L.valid = d <= 3;
    L.interior = d == 0;
    // columns of lanes with dl <= 3 lie in [-3, nx + 2]: one wrap each way unless nx < 3
    // (lattices 1 or 2 wide: x mod 2 = (x + 4) & 1 for x >= -4; no integer division)
    int x = x0 - 3 + l;
    if (A.nx >= 3) x = x < 0 ? x + A.nx : (x >= A.nx ? x - A.nx : x);
    else x = A.nx == 1 ? 0 : ((x + 4) & 1);
    if (dl > 3) x = 0;
    L.x = x;
    L.xm = x == 0 ? A.nx - 1 : x - 1;
    L.xp = x == A.nx - 1 ? 0 : x + 1;
    const int r = y0 - 3 + k;  // unwrapped row; in [0, ny) on the output tile
    // periodic: rows wrap; walls: rows outside [0, ny) are the solid nodes (ghost psi only).
    // WALLS (compile time) says whether walls may occur at all, so that the periodic kernel
    // carries none of this (its scalar registers are the occupancy limit).
    const bool walls = WALLS && A.walls;
    const bool fluid = !walls || (r >= 0 && r < A.ny);
    // r lies in [-3, ny + 2] for every wave: one wrap each way unless ny < 3 (then r >= -3, and
    // r mod 2 = (r + 4) & 1)
    const int rw = walls ? r
                         : (A.ny >= 3 ? (r < 0 ? r + A.ny : (r >= A.ny ? r - A.ny : r))
                                      : (A.ny == 1 ? 0 : ((r + 4) & 1)));
    const T ghost = walls ? (T)(r < 0 ? A.psi_lo : A.psi_hi) : (T)0;
    Acc acc = {0.0, 0.0, 0.0};

    // 1. step t: pull, rho, psi.  The EOS record is copied to LDS while the pull is in
    //    flight: psi reads it there in phases 1 and 3, instead of the launch holding it in
    //    scalar registers (which spills them to vector lanes at this occupancy).
    if (threadIdx.x == 0) S.eos = A.eos;
    Row<T> R;
    double dr = 0.0;
    T ps = (T)0;
    const bool ring3 = dk <= 3 && dl <= 3;
    if (ring3 && fluid) {
        const View<T> V = make_view<T>(A.src, A.plane);
        pull<T>(V, A, L.x, L.xm, L.xp, rw, R.g0, R.g);
    }
    __syncthreads();
    if (ring3) {
        if (fluid) {
            dr = node_drho<T>(R.g0, R.g);
            ps = node_psi<T>(A, S.eos, dr, true);
        } else {
            ps = ghost;
        }
    }
    sps[k][l] = ps;
    __syncthreads();
    // 2. step t: collide on the tile grown by 2, post-collision state to LDS
    if (dk <= 2 && dl <= 2 && fluid) {
        T Ftx, Fty;
        force_tilde<T>(A, sps[k - 1][l - 1], sps[k - 1][l], sps[k - 1][l + 1], sps[k][l - 1], sps[k][l + 1],
                       sps[k + 1][l - 1], sps[k + 1][l], sps[k + 1][l + 1], Ftx, Fty);
        T o[9];
        double o0;
        node_collide<T, MODE_STEP>(A, L, rw, R, dr, ps, Ftx, Fty, acc, o, o0);
#pragma unroll
        for (int i = 1; i < 9; ++i) smv[i - 1][k - 1][l] = o[i];
        sg0[k - 1][l] = o0;
        if (MODE == MODE_RECORD && d == 0) {
            T jx, jy;
            node_j<T>(R.g, jx, jy);
            record_node<T>(A.rec, A.rec_plane, (size_t)r * A.nx + x, (T)dr, jx, jy, ps);
        }
    }
    __syncthreads();
    // 3. step t+1: pull from LDS on the tile grown by 1 (f_i(x) = f*_i(x - c_i), or the node's
    //    own opposite population where x - c_i is solid), psi(t+1)
    if (dk <= 1 && dl <= 1 && fluid) {
        const int q = k - 1;  // LDS row of this wave
        const bool bot = walls && r == 0, top = walls && r == A.ny - 1;
        R.g0 = sg0[q][l];
        R.g[1] = smv[0][q][l - 1];
        R.g[3] = smv[2][q][l + 1];
        if (!bot) {
            R.g[2] = smv[1][q - 1][l];
            R.g[5] = smv[4][q - 1][l - 1];
            R.g[6] = smv[5][q - 1][l + 1];
        } else {
            R.g[2] = smv[3][q][l];
            R.g[5] = smv[6][q][l];
            R.g[6] = smv[7][q][l];
        }
        if (!top) {
            R.g[4] = smv[3][q + 1][l];
            R.g[7] = smv[6][q + 1][l + 1];
            R.g[8] = smv[7][q + 1][l - 1];
        } else {
            R.g[4] = smv[1][q][l];
            R.g[7] = smv[4][q][l];
            R.g[8] = smv[5][q][l];
        }
        dr = node_drho<T>(R.g0, R.g);
        ps = node_psi<T>(A, S.eos, dr, true, 1);
        sps[k][l] = ps;
    } else if (walls && dk <= 1 && dl <= 1) {
        sps[k][l] = ghost;
    }
    __syncthreads();
    // 4. step t+1: collide on the tile and store (tile rows are fluid rows)
    if (d == 0) {
        T Ftx, Fty;
        force_tilde<T>(A, sps[k - 1][l - 1], sps[k - 1][l], sps[k - 1][l + 1], sps[k][l - 1], sps[k][l + 1],
                       sps[k + 1][l - 1], sps[k + 1][l], sps[k + 1][l + 1], Ftx, Fty);
        update_node<T, MODE == MODE_STEP_REDUCE ? MODE_STEP_REDUCE : MODE_STEP, NT>(A, L, r, R, dr, ps, Ftx, Fty, acc);
        if (MODE == MODE_RECORD) {
            T jx, jy;
            node_j<T>(R.g, jx, jy);
            record_node<T>((char*)A.rec + 4 * A.rec_plane * sizeof(T), A.rec_plane, (size_t)r * A.nx + x, (T)dr, jx,
                           jy, ps);
        }
    }
    if (MODE == MODE_STEP_REDUCE) {
        // FP64 mass and momentum of step t+1 (each node once: the tile's own): each wave's
        // total, then the waves in order, one partial per tile in tile order
        const double m = wave_total(acc.m), jx = wave_total(acc.x), jy = wave_total(acc.y);
        if (l == kTotalLane) {
            S.sred[k][0] = m;
            S.sred[k][1] = jx;
            S.sred[k][2] = jy;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double r = 0.0;
            for (int w = 0; w < k2WavesOf<T>; ++w) r += S.sred[w][threadIdx.x];
            A.partials[3 * ((size_t)band * ((A.nx + k2Cols - 1) / k2Cols) + strip) + threadIdx.x] = r;
        }
    }
}

template <typename T, int NW, int RPW>
struct Step2RowsLds {
    static constexpr int NR = NW * RPW;  // rows of the tile grown by 3
    DevEos eos;                          // the lattice's EOS record (read by node_psi)
    T sps[NR][64];                       // psi of the tile grown by 3 (step t), then by 1 (step t+1)
    T smv[8][NR - 2][64];                // post-collision moving populations of step t (tile grown by 2)
    double sg0[NR - 2][64];              // and their FP64 rest population
    double sred[NW][3];                  // a reducing launch's wave totals (mass, momentum)
};

// step2_tile with RPW rows per wave: a workgroup of NW waves holds the NW * RPW rows of the
// tile grown by 3 (wave k holds rows k + j NW, j < RPW), in the same four phases and with the
// same node arithmetic.  The rows of one wave are processed one after the other inside each
// phase; their loads are issued together.
template <typename T, int MODE, bool WALLS, bool NT, int NW, int RPW>
__device__ __forceinline__ void step2_tile_rows(const StepArgs& A, int strip, int band, Step2RowsLds<T, NW, RPW>& S)
{
    constexpr int NR = NW * RPW;
    auto& sps = S.sps;
    auto& smv = S.smv;
    auto& sg0 = S.sg0;
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int k2Rows = A.rows2t;  // at most NR - 6
    const int x0 = strip * k2Cols, y0 = band * k2Rows;
    const int W = min(k2Cols, A.nx - x0), H = min(k2Rows, A.ny - y0);
    // distance of this lane's column from the output tile
    const int dl = l < 3 ? 3 - l : (l > W + 2 ? l - (W + 2) : 0);
    Lane L;
    L.lane = l;
    L.valid = true;
    L.interior = true;
    // columns of lanes with dl <= 3 lie in [-3, nx + 2]: one wrap each way unless nx < 3
    // (lattices 1 or 2 wide: x mod 2 = (x + 4) & 1 for x >= -4; no integer division)
    int x = x0 - 3 + l;
    if (A.nx >= 3) x = x < 0 ? x + A.nx : (x >= A.nx ? x - A.nx : x);
    else x = A.nx == 1 ? 0 : ((x + 4) & 1);
    if (dl > 3) x = 0;
    L.x = x;
    L.xm = x == 0 ? A.nx - 1 : x - 1;
    L.xp = x == A.nx - 1 ? 0 : x + 1;
    const bool walls = WALLS && A.walls;
    // per row kk of this wave (kk = k + j NW): distance from the output tile, unwrapped lattice
    // row (in [0, ny) on the output tile), wrapped row, fluid.  Recomputed where needed (scalar
    // arithmetic) rather than held across the barriers.
    auto dk_of = [&](int kk) { return kk < 3 ? 3 - kk : (kk > H + 2 ? kk - (H + 2) : 0); };
    auto r_of = [&](int kk) { return y0 - 3 + kk; };
    auto fluid_of = [&](int r) { return !walls || (r >= 0 && r < A.ny); };
    // r lies in [-3, ny + 2] for the rows that load: one wrap each way unless ny < 3 (then
    // r >= -3, and r mod 2 = (r + 4) & 1)
    auto rw_of = [&](int r) {
        return walls ? r
                     : (A.ny >= 3 ? (r < 0 ? r + A.ny : (r >= A.ny ? r - A.ny : r))
                                  : (A.ny == 1 ? 0 : ((r + 4) & 1)));
    };
    auto ghost_of = [&](int r) { return walls ? (T)(r < 0 ? A.psi_lo : A.psi_hi) : (T)0; };
    Acc acc = {0.0, 0.0, 0.0};

    // 1. step t: pull, rho, psi.  The EOS record is copied to LDS while the pull is in
    //    flight: psi reads it there in phases 1 and 3, instead of the launch holding it in
    //    scalar registers (which spills them to vector lanes at this occupancy).
    if (threadIdx.x == 0) S.eos = A.eos;
    Row<T> R[RPW];
    double dr[RPW];
    T ps[RPW];
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
        const int kk = k + j * NW, r = r_of(kk);
        dr[j] = 0.0;
        ps[j] = (T)0;
        if (dk_of(kk) <= 3 && dl <= 3 && fluid_of(r)) {
            const View<T> V = make_view<T>(A.src, A.plane);
            pull<T>(V, A, L.x, L.xm, L.xp, rw_of(r), R[j].g0, R[j].g);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
        const int kk = k + j * NW, r = r_of(kk);
        if (dk_of(kk) <= 3 && dl <= 3) {
            if (fluid_of(r)) {
                dr[j] = node_drho<T>(R[j].g0, R[j].g);
                ps[j] = node_psi<T>(A, S.eos, dr[j], true);
            } else {
                ps[j] = ghost_of(r);
            }
        }
        sps[kk][l] = ps[j];
    }
    __syncthreads();
    // 2. step t: collide on the tile grown by 2, post-collision state to LDS
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
        const int kk = k + j * NW, r = r_of(kk), dk = dk_of(kk);
        if (dk <= 2 && dl <= 2 && fluid_of(r)) {
            T Ftx, Fty;
            force_tilde<T>(A, sps[kk - 1][l - 1], sps[kk - 1][l], sps[kk - 1][l + 1], sps[kk][l - 1], sps[kk][l + 1],
                           sps[kk + 1][l - 1], sps[kk + 1][l], sps[kk + 1][l + 1], Ftx, Fty);
            T o[9];
            double o0;
            node_collide<T, MODE_STEP>(A, L, rw_of(r), R[j], dr[j], ps[j], Ftx, Fty, acc, o, o0);
#pragma unroll
            for (int i = 1; i < 9; ++i) smv[i - 1][kk - 1][l] = o[i];
            sg0[kk - 1][l] = o0;
            if (MODE == MODE_RECORD && dk == 0 && dl == 0) {
                T jx, jy;
                node_j<T>(R[j].g, jx, jy);
                record_node<T>(A.rec, A.rec_plane, (size_t)r * A.nx + x, (T)dr[j], jx, jy, ps[j]);
            }
        }
    }
    __syncthreads();
    // 3. step t+1: pull from LDS on the tile grown by 1 (f_i(x) = f*_i(x - c_i), or the node's
    //    own opposite population where x - c_i is solid), psi(t+1)
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
        const int kk = k + j * NW, r = r_of(kk), dk = dk_of(kk);
        if (dk <= 1 && dl <= 1 && fluid_of(r)) {
            const int q = kk - 1;  // LDS row of this row
            const bool bot = walls && r == 0, top = walls && r == A.ny - 1;
            R[j].g0 = sg0[q][l];
            R[j].g[1] = smv[0][q][l - 1];
            R[j].g[3] = smv[2][q][l + 1];
            if (!bot) {
                R[j].g[2] = smv[1][q - 1][l];
                R[j].g[5] = smv[4][q - 1][l - 1];
                R[j].g[6] = smv[5][q - 1][l + 1];
            } else {
                R[j].g[2] = smv[3][q][l];
                R[j].g[5] = smv[6][q][l];
                R[j].g[6] = smv[7][q][l];
            }
            if (!top) {
                R[j].g[4] = smv[3][q + 1][l];
                R[j].g[7] = smv[6][q + 1][l + 1];
                R[j].g[8] = smv[7][q + 1][l - 1];
            } else {
                R[j].g[4] = smv[1][q][l];
                R[j].g[7] = smv[4][q][l];
                R[j].g[8] = smv[5][q][l];
            }
            dr[j] = node_drho<T>(R[j].g0, R[j].g);
            ps[j] = node_psi<T>(A, S.eos, dr[j], true, 1);
            sps[kk][l] = ps[j];
        } else if (walls && dk <= 1 && dl <= 1) {
            sps[kk][l] = ghost_of(r);
        }
    }
    __syncthreads();
    // 4. step t+1: collide on the tile and store (tile rows are fluid rows)
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
        const int kk = k + j * NW, r = r_of(kk);
        if (dk_of(kk) == 0 && dl == 0) {
            T Ftx, Fty;
            force_tilde<T>(A, sps[kk - 1][l - 1], sps[kk - 1][l], sps[kk - 1][l + 1], sps[kk][l - 1], sps[kk][l + 1],
                           sps[kk + 1][l - 1], sps[kk + 1][l], sps[kk + 1][l + 1], Ftx, Fty);
            update_node<T, MODE == MODE_STEP_REDUCE ? MODE_STEP_REDUCE : MODE_STEP, NT>(A, L, r, R[j], dr[j], ps[j],
                                                                                          Ftx, Fty, acc);
            if (MODE == MODE_RECORD) {
                T jx, jy;
                node_j<T>(R[j].g, jx, jy);
                record_node<T>((char*)A.rec + 4 * A.rec_plane * sizeof(T), A.rec_plane, (size_t)r * A.nx + x,
                               (T)dr[j], jx, jy, ps[j]);
            }
        }
    }
    if (MODE == MODE_STEP_REDUCE) {
        // FP64 mass and momentum of step t+1 (each node once: the tile's own): each wave's
        // total, then the waves in order, one partial per tile in tile order
        const double m = wave_total(acc.m), jx = wave_total(acc.x), jy = wave_total(acc.y);
        if (l == kTotalLane) {
            S.sred[k][0] = m;
            S.sred[k][1] = jx;
            S.sred[k][2] = jy;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double r = 0.0;
            for (int w = 0; w < NW; ++w) r += S.sred[w][threadIdx.x];
            A.partials[3 * ((size_t)band * ((A.nx + k2Cols - 1) / k2Cols) + strip) + threadIdx.x] = r;
        }
    }
}

// ----------------------------------------------------------------- host helpers
inline DevEos dev_eos(const lbm_eos& e)
{
    DevEos E{};
    E.base = e.base;
    E.shape = e.shape;
    E.RT = e.R * e.T;
    if (e.base == LBM_BASE_PR) {
        const double kap = 0.37464 + 1.54226 * e.omega - 0.26992 * e.omega * e.omega;
        const double t = 1.0 + kap * (1.0 - std::sqrt(e.T / e.Tc));
        E.aal = e.a * t * t;
    } else {
        E.aal = e.a;
    }
    E.b = e.b;
    E.scale = e.scale;
    E.k_vap = e.k_vap;
    E.dP = e.dP_liq;
    E.rho_v = e.rho_v;
    E.rho_l = e.rho_l;
    E.rho_max = e.rho_max;
    E.rho_min = e.rho_min;
    E.p0 = e.p_sat;
    E.p_max = e.p_max;
    E.p_min = e.p_min;
    E.inv_a1sq = e.a1sq > 0 ? 1.0 / e.a1sq : 0.0;
    E.b1 = e.b1;
    E.inv_a3sq = e.a3sq > 0 ? 1.0 / e.a3sq : 0.0;
    E.b3 = e.b3;
    E.inv_L = e.rho_min > e.rho_max ? 1.0 / (e.rho_min - e.rho_max) : 0.0;
    E.rho_m = e.rho_m;
    E.theta = e.theta;
    E.fRT = (float)E.RT;
    E.faal = (float)E.aal;
    E.fb = (float)E.b;
    E.fscale = (float)E.scale;
    E.fk_vap = (float)E.k_vap;
    E.fdP = (float)E.dP;
    return E;
}

// Node-update constants of a lattice from its relaxation times (Eq. RelaxationMatrix),
// G and the Eq. LiFS sigma, in both arithmetic types.
inline void fill_coef(StepArgs& A, const double tau[9], double G, double sigma)
{
    Coef<double> c;
    const double s[9] = {1 / tau[0], 1 / tau[1], 1 / tau[2], 1 / tau[3], 1 / tau[4],
                         1 / tau[5], 1 / tau[6], 1 / tau[7], 1 / tau[8]};
    c.se = s[1];
    c.sq = s[2];
    c.sqx = s[4];
    c.sqy = s[6];
    c.snu = s[7];
    c.he = 1 - 0.5 * s[1];
    c.hq = 1 - 0.5 * s[2];
    c.hqx = 1 - 0.5 * s[4];
    c.hqy = 1 - 0.5 * s[6];
    c.hnu = 1 - 0.5 * s[7];
    c.le = 12.0 * sigma * c.he / (tau[1] - 0.5);
    c.lq = 12.0 * sigma * c.hq / (tau[2] - 0.5);
    c.G = G;
    c.two_inv_G = 2.0 / G;
    c.sh1 = (1.0 - s[7]) * 0.25;
    c.sh2 = s[7] * 0.25;
    c.sh3 = c.hnu * 0.5;
    c.sh4 = c.hnu * 0.25;
    c.he6 = c.he / 6.0;
    c.le36 = c.le / 36.0;
    A.cd = c;
    A.unit_rates = tau[1] == 1.0 && tau[2] == 1.0 && tau[4] == 1.0 && tau[6] == 1.0;
    A.cf = Coef<float>{(float)c.se, (float)c.sq, (float)c.sqx, (float)c.sqy, (float)c.snu,
                       (float)c.he, (float)c.hq, (float)c.hqx, (float)c.hqy, (float)c.hnu,
                       (float)c.le, (float)c.lq, (float)c.G, (float)c.two_inv_G, (float)c.sh1, (float)c.sh2,
                       (float)c.sh3, (float)c.sh4, (float)c.he6, (float)c.le36};
}

inline int validate(const lbm_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1 || (p->prec != LBM_FP64 && p->prec != LBM_FP32_SHIFTED)) {
        lbm_set_error("lbm: invalid lattice size or precision");
        return LBM_EINVAL;
    }
    if ((long long)((p->nx + 63) & ~63) * p->ny * 8 >= (1LL << 32)) {
        lbm_set_error("lbm: one population plane must stay below 4 GiB (lattice too large)");
        return LBM_EINVAL;
    }
    if (!(p->G < 0.0)) {
        lbm_set_error("lbm: G must be negative (Eq. InteractionPotential with p_EOS < rho c_s^2)");
        return LBM_EINVAL;
    }
    for (int k = 0; k < 9; ++k)
        if (!(p->tau[k] > 0.5)) {
            lbm_set_error("lbm: every relaxation time must exceed 1/2");
            return LBM_EINVAL;
        }
    if (!tile_rows_valid(*p)) {
        lbm_set_error("lbm: tile_rows must be 0 (automatic), -1 (timed at lbm_init), 10..18 (FP32) or 5..10 (FP64)");
        return LBM_EINVAL;
    }
    if (p->kernel_variant < 0 || p->kernel_variant > LBM_VARIANT_AA) {
        lbm_set_error("lbm: kernel_variant must be 0 (automatic), 1 (row march), 2 (row block), 3 (two-step block) "
                      "or 4 (in-place AA)");
        return LBM_EINVAL;
    }
    if (p->band_rows < 0 || p->band_rows > 4096) {
        lbm_set_error("lbm: band_rows must be in [0, 4096] (0 = automatic)");
        return LBM_EINVAL;
    }
    if (p->tau[7] != p->tau[8]) {
        lbm_set_error("lbm: Eq. RelaxationMatrix relaxes both shear moments with tau_nu (tau[7] == tau[8])");
        return LBM_EINVAL;
    }
    if (p->var_tau && !(p->tau_l > 0.5 && p->tau_v > 0.5 && p->rho_l_tau != p->rho_v_tau)) {
        lbm_set_error("lbm: Eq. RelaxationTime needs tau_l, tau_v > 1/2 and rho_l != rho_v");
        return LBM_EINVAL;
    }
    if (p->prec == LBM_FP32_SHIFTED && !(p->rho_ref > 0.0)) {
        lbm_set_error("lbm: FP32-shifted storage needs rho_ref > 0");
        return LBM_EINVAL;
    }
    if (!(p->eos.T > 0.0)) {
        lbm_set_error("lbm: EOS not built (call lbm_eos_build first)");
        return LBM_EINVAL;
    }
    return LBM_OK;
}

}  // namespace lbmk
