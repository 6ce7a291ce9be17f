// In-place streaming with the AA access pattern (LBM_VARIANT_AA): one population buffer
// instead of two.
//
// Storage A_i[x] holds population i of node x.  Steps alternate between two access
// patterns, so that in every step each location is read and written by one node only:
//   even step t (natural layout): node x reads f_i(x, t) = A_i[x] and writes its
//     post-collision f*_i(x, t) to A_opp(i)[x] (its own node, opposite slot);
//   odd step t (swapped layout):  node x reads f_i(x, t) = f*_i(x - c_i, t - 1) =
//     A_opp(i)[x - c_i] and writes f*_i(x, t) to A_i[x + c_i], which is where the next
//     even step's node x + c_i reads f_i.
// Half-way bounce-back (walls) keeps that: in an odd step a population that would come from
// a solid node is f*_opp(i)(x, t - 1), which the even step left at A_i[x], and one that
// would go into a solid node is stored at A_opp(i)[x], where the even step's node x reads
// f_opp(i).  The rest population stays at its node.  After an even number of steps node x
// holds its own f_i(x, t) (the two-buffer variants hold the post-collision f*_i(x, t - 1)
// there and pull), after an odd number the swapped layout above.
//
// What the fused pull kernels cannot do here is form psi of the neighbours while updating
// a node (Eq. ShanChenForce): the densities of x + c_i live in locations those nodes
// overwrite during the same pass.  So each step is two launches: k_aa_psi writes psi of
// every node to a plane of the workspace, then k_aa_step reads psi of the 3 x 3 stencil
// from it, collides (node_collide, the same node arithmetic as every other variant) and
// writes in place.  Per FP32-shifted node update that is 80 B of populations plus 40 B
// read again and 8 B of psi: the variant halves the population memory, not the traffic.
#include "lbm_ctx.h"

namespace {

using namespace lbmk;

constexpr int kAaRows = 4;  // rows (one wavefront each) per 256-thread workgroup
constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

struct AaNode {
    int x, y;
    bool live;
};

__device__ __forceinline__ AaNode aa_node(const StepArgs& A)
{
    AaNode n;
    n.x = blockIdx.x * 64 + (threadIdx.x & 63);
    n.y = blockIdx.y * kAaRows + (threadIdx.x >> 6);
    n.live = n.x < A.nx && n.y < A.ny;
    return n;
}

// node (x + dx, y + dy): periodic wrap in x always, in y without walls; with walls a row
// outside [0, ny) is solid (returns false)
__device__ __forceinline__ bool aa_neighbour(const StepArgs& A, int x, int y, int dx, int dy, uint32_t& off)
{
    int xn = x + dx, yn = y + dy;
    xn = xn < 0 ? xn + A.nx : (xn >= A.nx ? xn - A.nx : xn);
    if (yn < 0 || yn >= A.ny) {
        if (A.walls) return false;
        yn = yn < 0 ? yn + A.ny : yn - A.ny;
    }
    off = (uint32_t)yn * (uint32_t)A.ld + (uint32_t)xn;
    return true;
}

// f_i(x, t) of the step with parity ODD, i = 0..8 (rest population in g0)
template <typename T, bool ODD>
__device__ __forceinline__ void aa_gather(const View<T>& V, const StepArgs& A, int x, int y, double& g0, T g[9])
{
    const uint32_t own = (uint32_t)y * (uint32_t)A.ld + (uint32_t)x;
    g0 = ld_at<double>(V.rest, own);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!ODD) {
            g[i] = ld_at<T>(V.mv[i], own);
        } else {
            uint32_t src;
            // from x - c_i; bounce-back from a solid node: the slot the even step left at x
            g[i] = aa_neighbour(A, x, y, -kCx[i], -kCy[i], src) ? ld_at<T>(V.mv[kOpp[i]], src) : ld_at<T>(V.mv[i], own);
        }
    }
}

// store f*_i(x, t) of the step with parity ODD
template <typename T, bool ODD>
__device__ __forceinline__ void aa_scatter(const WView<T>& D, const StepArgs& A, int x, int y, const T o[9], double o0)
{
    const uint32_t own = (uint32_t)y * (uint32_t)A.ld + (uint32_t)x;
    *(double*)(D.rest + own * 8u) = o0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        if (!ODD) {
            *(T*)(D.mv[kOpp[i]] + own * (uint32_t)sizeof(T)) = o[i];
        } else {
            uint32_t dst;
            if (aa_neighbour(A, x, y, kCx[i], kCy[i], dst)) *(T*)(D.mv[i] + dst * (uint32_t)sizeof(T)) = o[i];
            else *(T*)(D.mv[kOpp[i]] + own * (uint32_t)sizeof(T)) = o[i];  // into a wall: bounce back
        }
    }
}

// Initial state in the natural layout: f_i(x, 0) = f^eq_i(rho0, u0) of the node itself (the
// two-buffer variants store the same populations one node upstream, for their first pull).
// In FP32-shifted storage the FP64 rest population takes what the node's eight FP32-rounded
// moving populations leave of rho0, as there.
template <typename T>
__global__ __launch_bounds__(256) void k_aa_init(StepArgs A, const double* rho0, const double* ux0, const double* uy0)
{
    const AaNode n = aa_node(A);
    if (!n.live) return;
    const size_t c = (size_t)n.y * A.nx + n.x, off = (size_t)n.y * A.ld + n.x;
    const double r = rho0[c], u = ux0 ? ux0[c] : 0.0, v = uy0 ? uy0[c] : 0.0;
    Plane<T>::restw(A.dst, A.plane)[off] = init_population<T>(0, r, u, v, A.rho_ref);
    for (int i = 1; i < 9; ++i) Plane<T>::movw(A.dst, A.plane, i)[off] = (T)init_population<T>(i, r, u, v, A.rho_ref);
}

// psi of the density the populations hold before a step of parity ODD, into plane psi
template <typename T, bool ODD>
__global__ __launch_bounds__(256) void k_aa_psi(StepArgs A, T* psi, int check)
{
    const AaNode n = aa_node(A);
    if (!n.live) return;
    const View<T> V = make_view<T>(A.src, A.plane);
    double g0;
    T g[9];
    aa_gather<T, ODD>(V, A, n.x, n.y, g0, g);
    psi[(size_t)n.y * A.ld + n.x] = node_psi<T>(A, node_drho<T>(g0, g), check != 0);
}

// psi at (x + dx, y + dy) from the plane; the ghost psi of Eq. ShanChenForce beyond a wall
template <typename T>
__device__ __forceinline__ T aa_psi_at(const StepArgs& A, const T* psi, int x, int y, int dx, int dy)
{
    uint32_t off;
    if (aa_neighbour(A, x, y, dx, dy, off)) return psi[off];
    return (T)(y + dy < 0 ? A.psi_lo : A.psi_hi);
}

// One step of parity ODD in place: gather, Eq. ShanChenForce from the psi plane,
// node_collide, scatter.  MODE_STEP_REDUCE leaves one FP64 (mass, j_x, j_y) triple per
// workgroup in A.partials (blocks in row-major grid order); MODE_MACROS writes the
// macroscopic fields and stores nothing.
template <typename T, bool ODD, int MODE>
__global__ __launch_bounds__(256) void k_aa_step(StepArgs A, const T* psi)
{
    const AaNode n = aa_node(A);
    Acc acc = {0.0, 0.0, 0.0};
    if (n.live) {
        const View<T> V = make_view<T>(A.src, A.plane);
        Row<T> R;
        aa_gather<T, ODD>(V, A, n.x, n.y, R.g0, R.g);
        const double dr = node_drho<T>(R.g0, R.g);
        const T pc = psi[(size_t)n.y * A.ld + n.x];
        T Ftx, Fty;
        force_tilde<T>(A, aa_psi_at(A, psi, n.x, n.y, -1, -1), aa_psi_at(A, psi, n.x, n.y, 0, -1),
                       aa_psi_at(A, psi, n.x, n.y, 1, -1), aa_psi_at(A, psi, n.x, n.y, -1, 0),
                       aa_psi_at(A, psi, n.x, n.y, 1, 0), aa_psi_at(A, psi, n.x, n.y, -1, 1),
                       aa_psi_at(A, psi, n.x, n.y, 0, 1), aa_psi_at(A, psi, n.x, n.y, 1, 1), Ftx, Fty);
        Lane L;
        L.lane = threadIdx.x & 63;
        L.x = n.x;
        L.xm = L.xp = 0;
        L.valid = L.interior = true;
        T o[9];
        double o0;
        if (node_collide<T, MODE>(A, L, n.y, R, dr, pc, Ftx, Fty, acc, o, o0))
            aa_scatter<T, ODD>(make_wview<T>(A.dst, A.plane), A, n.x, n.y, o, o0);
    }
    if (MODE == MODE_STEP_REDUCE || MODE == MODE_MACROS) {
        // fixed-order sums: lanes by wave_total, then the four waves in order
        __shared__ double sm[kAaRows][3];
        const double m = wave_total(acc.m), jx = wave_total(acc.x), jy = wave_total(acc.y);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == kTotalLane) {
            sm[w][0] = m;
            sm[w][1] = jx;
            sm[w][2] = jy;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int k = 0; k < kAaRows; ++k) s += sm[k][threadIdx.x];
            A.partials[3 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x) + threadIdx.x] = s;
        }
    }
}

// FP64 populations f_i = g_i + w_i rho_ref at their nodes, from either layout
template <typename T, bool ODD>
__global__ __launch_bounds__(256) void k_aa_populations(StepArgs A, double* out)
{
    const AaNode n = aa_node(A);
    if (!n.live) return;
    const View<T> V = make_view<T>(A.src, A.plane);
    double g0;
    T g[9];
    aa_gather<T, ODD>(V, A, n.x, n.y, g0, g);
    const size_t np = (size_t)A.nx * A.ny, o = (size_t)n.y * A.nx + n.x;
    out[o] = g0 + kW[0] * A.rho_ref;
    for (int i = 1; i < 9; ++i) out[i * np + o] = (double)g[i] + kW[i] * A.rho_ref;
}

dim3 aa_grid(const lbm_params& p) { return dim3((p.nx + 63) / 64, (p.ny + kAaRows - 1) / kAaRows); }

template <typename T>
bool aa_launch(lbm_ctx* c, int mode, hipStream_t s, double* const* macros)
{
    StepArgs A = c->args;
    A.src = c->buf[0];
    A.dst = c->buf[0];
    A.step = c->step;
    if (macros) {
        A.o_rho = macros[0];
        A.o_ux = macros[1];
        A.o_uy = macros[2];
        A.o_psi = macros[3];
        A.o_p = macros[4];
        A.o_fx = macros[5];
        A.o_fy = macros[6];
    }
    T* psi = (T*)c->aa_psi;
    const dim3 g = aa_grid(c->P), b(256);
    const bool odd = c->step & 1;
    const int check = mode != MODE_MACROS;
    if (odd) hipLaunchKernelGGL((k_aa_psi<T, true>), g, b, 0, s, A, psi, check);
    else hipLaunchKernelGGL((k_aa_psi<T, false>), g, b, 0, s, A, psi, check);
    const T* cpsi = psi;
    if (mode == MODE_STEP) {
        if (odd) hipLaunchKernelGGL((k_aa_step<T, true, MODE_STEP>), g, b, 0, s, A, cpsi);
        else hipLaunchKernelGGL((k_aa_step<T, false, MODE_STEP>), g, b, 0, s, A, cpsi);
    } else if (mode == MODE_STEP_REDUCE) {
        if (odd) hipLaunchKernelGGL((k_aa_step<T, true, MODE_STEP_REDUCE>), g, b, 0, s, A, cpsi);
        else hipLaunchKernelGGL((k_aa_step<T, false, MODE_STEP_REDUCE>), g, b, 0, s, A, cpsi);
    } else {
        if (odd) hipLaunchKernelGGL((k_aa_step<T, true, MODE_MACROS>), g, b, 0, s, A, cpsi);
        else hipLaunchKernelGGL((k_aa_step<T, false, MODE_MACROS>), g, b, 0, s, A, cpsi);
    }
    return hip_ok(hipGetLastError(), "k_aa_step launch");
}

}  // namespace

namespace lbmk {

int aa_slots(const lbm_params& p)
{
    const dim3 g = aa_grid(p);
    return (int)(g.x * g.y);
}

size_t aa_psi_bytes(const lbm_params& p, int ld)
{
    const size_t t = p.prec == LBM_FP32_SHIFTED ? sizeof(float) : sizeof(double);
    return ((size_t)ld * p.ny * t + 255) & ~(size_t)255;
}

bool aa_step(lbm_ctx* c, int mode, hipStream_t s)
{
    return c->P.prec == LBM_FP32_SHIFTED ? aa_launch<float>(c, mode, s, nullptr)
                                         : aa_launch<double>(c, mode, s, nullptr);
}

bool aa_macros(lbm_ctx* c, double* const out[7], hipStream_t s)
{
    return c->P.prec == LBM_FP32_SHIFTED ? aa_launch<float>(c, MODE_MACROS, s, out)
                                         : aa_launch<double>(c, MODE_MACROS, s, out);
}

bool aa_init(lbm_ctx* c, const double* rho0, const double* ux0, const double* uy0, hipStream_t s)
{
    StepArgs A = c->args;
    A.dst = c->buf[0];
    const dim3 g = aa_grid(c->P), b(256);
    if (c->P.prec == LBM_FP32_SHIFTED) hipLaunchKernelGGL(k_aa_init<float>, g, b, 0, s, A, rho0, ux0, uy0);
    else hipLaunchKernelGGL(k_aa_init<double>, g, b, 0, s, A, rho0, ux0, uy0);
    return hip_ok(hipGetLastError(), "k_aa_init launch");
}

bool aa_populations(lbm_ctx* c, double* f_out, hipStream_t s)
{
    StepArgs A = c->args;
    A.src = c->buf[0];
    const dim3 g = aa_grid(c->P), b(256);
    const bool odd = c->step & 1, f32 = c->P.prec == LBM_FP32_SHIFTED;
    if (f32 && odd) hipLaunchKernelGGL((k_aa_populations<float, true>), g, b, 0, s, A, f_out);
    else if (f32) hipLaunchKernelGGL((k_aa_populations<float, false>), g, b, 0, s, A, f_out);
    else if (odd) hipLaunchKernelGGL((k_aa_populations<double, true>), g, b, 0, s, A, f_out);
    else hipLaunchKernelGGL((k_aa_populations<double, false>), g, b, 0, s, A, f_out);
    return hip_ok(hipGetLastError(), "k_aa_populations launch");
}

}  // namespace lbmk
