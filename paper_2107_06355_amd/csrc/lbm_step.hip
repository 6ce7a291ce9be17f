// liblbm.so device code and C-ABI entry points (gfx950 / CDNA4).
//
// One time step of the pseudopotential LBM (Eq. LBE) as ONE fused kernel:
//   pull-stream (half-way bounce-back at walls)  ->  rho, j (Eq. Density,
//   Eq. Momentum)  ->  shaped p_EOS(rho) (Sec. III.D, Eq. PengEOS)  ->
//   psi (Eq. InteractionPotential)  ->  Shan-Chen force (Eq. ShanChenForce)
//   ->  forced velocity  ->  MRT relaxation in moment space (Eq. OperatorMRT,
//   Eq. MatrixMRT, Eq. RelaxationMatrix, Eq. RelaxationTime) with the source
//   of Eq. LiFS (Eq. GFS at sigma = 0)  ->  store of the post-collision
//   populations.
//
// Work decomposition.  A wavefront owns a strip of 62 columns and a band of
// H rows.  Its 64 lanes hold columns x0-1 .. x0+62, so the two edge lanes
// are the psi halo in x; the wave marches up the band keeping three rows of
// psi in registers (rows y-1, y, y+1), so every population is pulled once
// (plus the 2/62 column halo and the 2/H row halo, which hit L2), psi never
// goes to memory, and the x-neighbours of psi come from lane shuffles.
// Memory traffic per cell update is the algorithmic minimum: 9 loads and 9
// stores of the populations.  Workgroups are remapped so that consecutive
// bands land on the same XCD (shared L2 for the row halo).
//
// Storage (chosen per lbm_prec): FP64 populations, or FP32 deviations
// g_i = f_i - w_i rho_ref with the rest population g_0 kept in FP64 and set
// after collision to (pre-collision node mass) - sum of the stored moving
// populations, so that every node's mass is exact to FP64 rounding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "lbm.h"
#include "lbm_ctx.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace {

using namespace lbmk;

constexpr int kWaves = 4;     // waves per workgroup of the row-march kernel
constexpr int kHistCap = 4096;

// One row of the march.  Rp holds row r-1 (collision), Rc row r (psi now), Rn
// row r+1 (loads in flight since the previous row) and the loads of row r+2 are
// issued into Rf before anything waits on memory: two rows stay in flight.
template <typename T, int MODE>
__device__ __forceinline__ void march_row(const StepArgs& A, const View<T>& V, const Lane& L, int r, int y0, int y1,
                                          Row<T>& Rp, Row<T>& Rc, Row<T>& Rf, double& drp, double& drc, T& psA,
                                          T& psB, Acc& acc)
{
    if (r > y1) return;
    if (r + 2 <= y1) pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, r + 2), Rf.g0, Rf.g);
    drc = node_drho<T>(Rc.g0, Rc.g);
    T ps;
    if (A.walls && r < 0) ps = (T)A.psi_lo;
    else if (A.walls && r >= A.ny) ps = (T)A.psi_hi;
    else ps = node_psi<T>(A, drc, L.valid);
    if (r - 1 >= y0) collide_row<T, MODE>(A, L, r - 1, Rp, drp, psA, psB, ps, acc);
    psA = psB;
    psB = ps;
}

// FP64: at most 2 waves per SIMD leaves the register budget for the prefetched rows
// (measured on MI355X: 2.0 ms vs 2.16 ms per 8192^2 step with the compiler's choice of 3)
template <typename T, int MODE>
__global__ __launch_bounds__(256) LBM_OCCUPANCY_HINT
    __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 8 ? 2 : 8))) void k_step(StepArgs A)
{
    const int nb = gridDim.x;
    const int logical = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);  // XCD-contiguous bands
    // the wave index is uniform across the wave: keep it (and everything derived
    // from it: band, rows, wall tests, plane selects) in scalar registers
    const int w = logical * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= A.nwork) return;
    Lane L;
    L.lane = threadIdx.x & 63;
    const int strip = w % A.strips, seg = w / A.strips;
    const int x0 = strip * kStripW;
    const int W = min(kStripW, A.nx - x0);
    const int xr = x0 - 1 + L.lane;
    L.valid = L.lane <= W + 1;
    L.interior = L.lane >= 1 && L.lane <= W;
    int x = xr < 0 ? xr + A.nx : (xr >= A.nx ? xr - A.nx : xr);
    if (!L.valid) x = 0;
    L.x = x;
    L.xm = x == 0 ? A.nx - 1 : x - 1;
    L.xp = x == A.nx - 1 ? 0 : x + 1;
    const int y0 = seg * A.seg_h;
    const int y1 = min(A.ny, y0 + A.seg_h);
    const View<T> V = make_view<T>(A.src, A.plane);
    Acc acc = {0.0, 0.0, 0.0};

    if (A.seg_h == 1) {
        // One-row bands (small lattices): all three rows are loaded at once and
        // their psi evaluated as independent chains, so each wave waits on memory
        // only once.
        Row<T> Rm, Rc, Rp;
        pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y0 - 1), Rm.g0, Rm.g);
        pull<T>(V, A, L.x, L.xm, L.xp, y0, Rc.g0, Rc.g);
        pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y0 + 1), Rp.g0, Rp.g);
        const double dm = node_drho<T>(Rm.g0, Rm.g), dc = node_drho<T>(Rc.g0, Rc.g), dp = node_drho<T>(Rp.g0, Rp.g);
        const T psm = (A.walls && y0 == 0) ? (T)A.psi_lo : node_psi<T>(A, dm, L.valid);
        const T psc = node_psi<T>(A, dc, L.valid);
        const T psp = (A.walls && y0 == A.ny - 1) ? (T)A.psi_hi : node_psi<T>(A, dp, L.valid);
        collide_row<T, MODE>(A, L, y0, Rc, dc, psm, psc, psp, acc);
    } else {
    // March over rows r = y0-1 .. y1 (row r-1 is collided once psi(r) is known),
    // unrolled four times so that the four row registers change roles without copies.
    Row<T> R0, R1, R2, R3;
    R3.g0 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) R3.g[i] = (T)0;
    pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y0 - 1), R0.g0, R0.g);
    pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y0), R1.g0, R1.g);
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;  // density deviations of the rows in R0..R3
    T psA = (T)0, psB = (T)0;
    for (int r = y0 - 1; r <= y1; r += 4) {
        march_row<T, MODE>(A, V, L, r, y0, y1, R3, R0, R2, d3, d0, psA, psB, acc);
        march_row<T, MODE>(A, V, L, r + 1, y0, y1, R0, R1, R3, d0, d1, psA, psB, acc);
        march_row<T, MODE>(A, V, L, r + 2, y0, y1, R1, R2, R0, d1, d2, psA, psB, acc);
        march_row<T, MODE>(A, V, L, r + 3, y0, y1, R2, R3, R1, d2, d3, psA, psB, acc);
    }
    }
    if (MODE == MODE_STEP_REDUCE || MODE == MODE_MACROS) {
        acc.m = wave_total(acc.m);
        acc.x = wave_total(acc.x);
        acc.y = wave_total(acc.y);
        if (L.lane == kTotalLane) {
            A.partials[3 * w + 0] = acc.m;
            A.partials[3 * w + 1] = acc.x;
            A.partials[3 * w + 2] = acc.y;
        }
    }
}

// Row-block variant: a workgroup of 12 waves owns 12 consecutive rows of one
// strip (10 output rows and the two psi halo rows).  Every wave pulls ONE row,
// evaluates psi once per node into LDS, and after one barrier the 10 inner
// waves read the 3x3 psi stencil from LDS and update their nodes.  psi is thus
// evaluated 12/10 times per output node, with one row of loads per wave; two
// workgroups fit on a CU at the kernel's scalar-register occupancy.
#ifndef LBM_BLK_WAVES
#define LBM_BLK_WAVES 12
#endif
constexpr int kBlkWaves = LBM_BLK_WAVES;
constexpr int kBlkRows = kBlkWaves - 2;

template <typename T, int MODE>
__global__ __launch_bounds__(64 * LBM_BLK_WAVES) void k_step_blk(StepArgs A)
{
    __shared__ T sps[kBlkWaves][64];
    const int nb = gridDim.x;
    const int logical = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);  // XCD-contiguous blocks
    if (logical * kBlkWaves >= A.nwork) return;  // whole workgroup leaves together
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Lane L;
    L.lane = threadIdx.x & 63;
    const int strip = logical % A.strips, band = logical / A.strips;
    const int x0 = strip * kStripW;
    const int W = min(kStripW, A.nx - x0);
    const int xr = x0 - 1 + L.lane;
    L.valid = L.lane <= W + 1;
    L.interior = L.lane >= 1 && L.lane <= W;
    int x = xr < 0 ? xr + A.nx : (xr >= A.nx ? xr - A.nx : xr);
    if (!L.valid) x = 0;
    L.x = x;
    L.xm = x == 0 ? A.nx - 1 : x - 1;
    L.xp = x == A.nx - 1 ? 0 : x + 1;
    const int y0 = band * kBlkRows;
    const int y1 = min(A.ny, y0 + kBlkRows);
    const int r = y0 - 1 + k;  // this wave's row; rows y0-1 .. y1 are needed
    const View<T> V = make_view<T>(A.src, A.plane);
    Acc acc = {0.0, 0.0, 0.0};

    Row<T> R;
    double dr = 0.0;
    T ps = (T)0;
    if (r <= y1) {
        if (A.walls && r < 0) ps = (T)A.psi_lo;
        else if (A.walls && r >= A.ny) ps = (T)A.psi_hi;
        else {
            pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, r), R.g0, R.g);
            dr = node_drho<T>(R.g0, R.g);
            ps = node_psi<T>(A, dr, L.valid);
        }
    }
    sps[k][L.lane] = ps;
    __syncthreads();
    if (r >= y0 && r < y1 && L.interior) {
        T Ftx, Fty;
        force_tilde<T>(A, sps[k - 1][L.lane - 1], sps[k - 1][L.lane], sps[k - 1][L.lane + 1], sps[k][L.lane - 1],
                       sps[k][L.lane + 1], sps[k + 1][L.lane - 1], sps[k + 1][L.lane], sps[k + 1][L.lane + 1], Ftx, Fty);
        update_node<T, MODE>(A, L, r, R, dr, ps, Ftx, Fty, acc);
    }
    if (MODE == MODE_STEP_REDUCE || MODE == MODE_MACROS) {
        acc.m = wave_total(acc.m);
        acc.x = wave_total(acc.x);
        acc.y = wave_total(acc.y);
        if (L.lane == kTotalLane) {
            const int wv = logical * kBlkWaves + k;
            A.partials[3 * wv + 0] = acc.m;
            A.partials[3 * wv + 1] = acc.x;
            A.partials[3 * wv + 2] = acc.y;
        }
    }
}

// FP32: 16 waves, 8 waves per SIMD, two workgroups per CU (the EOS record in LDS keeps the
// scalar registers within the 8-wave budget).  FP64: 12 waves, 6 per SIMD (76 VGPRs), two
// workgroups per CU; 16-wave FP64 workgroups fit only one per CU, and forcing two of
// them spilled vector registers to scratch (25% slower on MI355X at 4096^2).
// MODE_STEP_REDUCE: the second step also leaves the FP64 mass/momentum partials.
template <typename T, int MODE, bool WALLS, bool NT = false>
__global__ __launch_bounds__(64 * k2WavesOf<T>) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : LBM_K2_EU_F64)))
void k_step2_blk(StepArgs A)
{
    __shared__ Step2Lds<T> S;
    const int nb = gridDim.x;
    const int logical = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);  // XCD-contiguous blocks
    int strip, band;
    if (!two_step_tile(A, logical, strip, band)) return;  // whole workgroup leaves together
    step2_tile<T, MODE, WALLS, NT>(A, strip, band, S);
}

// The same with two rows per wave (step2_tile_rows; the shape two_step_shape picks): FP32 12
// waves at two workgroups per CU (6 waves per SIMD), FP64 8 waves (4 per SIMD).
template <typename T, int MODE, bool WALLS, bool NT = false>
__global__ __launch_bounds__(64 * k2rWavesOf<T>) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 4)))
void k_step2_rows2(StepArgs A)
{
    __shared__ Step2RowsLds<T, k2rWavesOf<T>, 2> S;
    const int nb = gridDim.x;
    const int logical = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);  // XCD-contiguous blocks
    int strip, band;
    if (!two_step_tile(A, logical, strip, band)) return;  // whole workgroup leaves together
    step2_tile_rows<T, MODE, WALLS, NT, k2rWavesOf<T>, 2>(A, strip, band, S);
}

// Fixed-order FP64 reduction of the per-wave partials, two passes: block b sums
// the contiguous chunk b of the partials (thread-strided, then a tree), and one
// block sums the block results.  The order depends only on the sizes, so the
// result is bitwise reproducible.
constexpr int kRedBlocks = 256;

__device__ __forceinline__ void block_sum3(double a0, double a1, double a2, double* out)
{
    __shared__ double sh[3][256];
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] = sh[k][0];
}

__global__ __launch_bounds__(256) void k_reduce_chunks(const double* partials, int n, int chunk, double* blocks)
{
    const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
        a0 += partials[3 * i + 0];
        a1 += partials[3 * i + 1];
        a2 += partials[3 * i + 2];
    }
    block_sum3(a0, a1, a2, blocks + 3 * blockIdx.x);
}

// Up to kRedOneMax partials (a reducing two-step launch leaves one per tile: 468 at 512^2,
// 2,304 on the 2048 x 1024 impact) in one workgroup and one launch: each thread sums its
// strided share in order, each wave its 64 lanes (wave_total),
// and the first three threads the 16 wave totals in order.  The order depends only on n.
// One launch instead of two saves the second launch's latency, which is most of what a small
// reduction costs; one CU's loads set the limit (measured on MI355X: 7,488 partials 4.2 us
// against 7.3 us for the two-pass pair, but 27,648 partials 10.8 us against 9.5 us).
constexpr int kRedOneMax = 16384;
__global__ __launch_bounds__(1024) void k_reduce_one(const double* partials, int n, double* out, long long step,
                                                     int with_step)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int i = (int)threadIdx.x;
    // eight of the thread's partials loaded before any is added, so that their loads overlap;
    // the additions keep the order of i
    for (; i + 7 * 1024 < n; i += 8 * 1024) {
        double v[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[u][c] = partials[3 * (i + u * 1024) + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a0 += v[u][0];
            a1 += v[u][1];
            a2 += v[u][2];
        }
    }
    for (; i < n; i += 1024) {
        a0 += partials[3 * i + 0];
        a1 += partials[3 * i + 1];
        a2 += partials[3 * i + 2];
    }
    a0 = wave_total(a0);
    a1 = wave_total(a1);
    a2 = wave_total(a2);
    __shared__ double sh[3][16];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == kTotalLane) {
        sh[0][w] = a0;
        sh[1][w] = a1;
        sh[2][w] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double r = 0.0;
        for (int k = 0; k < 16; ++k) r += sh[threadIdx.x][k];
        const int o = with_step ? 1 : 0;
        if (threadIdx.x == 0 && with_step) out[0] = (double)step;
        out[o + threadIdx.x] = r;
    }
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* blocks, int nblocks, double* out, long long step,
                                                       int with_step)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if ((int)threadIdx.x < nblocks) {
        a0 = blocks[3 * threadIdx.x + 0];
        a1 = blocks[3 * threadIdx.x + 1];
        a2 = blocks[3 * threadIdx.x + 2];
    }
    double r[3];
    block_sum3(a0, a1, a2, r);
    if (threadIdx.x == 0) {
        int o = 0;
        if (with_step) out[o++] = (double)step;
        for (int k = 0; k < 3; ++k) out[o + k] = r[k];
    }
}

// initial state: store A_j(z) such that the pull of the first step yields f^eq(rho0, u0)
template <typename T>
__global__ void k_init(StepArgs A, const double* rho0, const double* ux0, const double* uy0)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= A.nx || y >= A.ny) return;
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const size_t off = (size_t)y * A.ld + x;
    for (int j = 0; j < 9; ++j) {
        int sx = x + cx[j], sy = y + cy[j], k = j;
        if (A.walls && (sy < 0 || sy >= A.ny)) {
            sx = x;
            sy = y;
            k = op[j];
        }
        sx = sx < 0 ? sx + A.nx : (sx >= A.nx ? sx - A.nx : sx);
        sy = sy < 0 ? sy + A.ny : (sy >= A.ny ? sy - A.ny : sy);
        const size_t c = (size_t)sy * A.nx + sx;
        const double g = init_population<T>(k, rho0[c], ux0 ? ux0[c] : 0.0, uy0 ? uy0[c] : 0.0, A.rho_ref);
        if (j == 0) Plane<T>::restw(A.dst, A.plane)[off] = g;
        else Plane<T>::movw(A.dst, A.plane, j)[off] = (T)g;
    }
}

// f_i(t, x) of Eq. LBE as FP64 [9][ny][nx]
template <typename T>
__global__ void k_populations(StepArgs A, double* out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= A.nx || y >= A.ny) return;
    const int xm = x == 0 ? A.nx - 1 : x - 1;
    const int xp = x == A.nx - 1 ? 0 : x + 1;
    double g0;
    T g[9];
    const View<T> V = make_view<T>(A.src, A.plane);
    pull<T>(V, A, x, xm, xp, y, g0, g);
    const size_t n = (size_t)A.nx * A.ny, o = (size_t)y * A.nx + x;
    out[o] = g0 + kW[0] * A.rho_ref;
    for (int i = 1; i < 9; ++i) out[i * n + o] = (double)g[i] + kW[i] * A.rho_ref;
}

}  // namespace

// ===================================================================== host side
namespace lbmk {

bool hip_ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    lbm_set_error(buf);
    return false;
}

// Work decomposition.  Returns the number of waves (partial-sum slots).
// Row-march kernel: one wave per (strip, band of seg_h rows).  Row-block
// kernel: one 16-wave workgroup per (strip, band of 14 rows).
int resolve_variant(const lbm_params& p)
{
    // measured on MI355X: two steps per launch beat both one-step decompositions on every
    // lattice timed, periodic (512^2 .. 16384^2) and walled (2048 x 1024 drop impact:
    // 25.0 vs 30.0 us FP32, 46.9 vs 60.8 us FP64; 8192 x 2048 FP32: 202 vs 300 us)
    return p.kernel_variant == 0 ? LBM_VARIANT_BLOCK2 : p.kernel_variant;
}

int decompose(const lbm_params& p, int* strips, int* seg_h, int* nseg, int* blk)
{
    *strips = (p.nx + kStripW - 1) / kStripW;
    const int v = resolve_variant(p);
    // BLOCK2 runs its single steps (reductions, checkpoints, odd counts) on the row block
    *blk = v == LBM_VARIANT_BLOCK || v == LBM_VARIANT_BLOCK2;
    if (*blk) {
        *seg_h = kBlkRows;
        *nseg = (p.ny + kBlkRows - 1) / kBlkRows;
        return *strips * *nseg * kBlkWaves;
    }
    int h = p.band_rows;
    if (h <= 0) h = p.prec == LBM_FP32_SHIFTED ? 4 : 8;  // best band heights measured on MI355X
    *seg_h = h;
    *nseg = (p.ny + h - 1) / h;
    return *strips * *nseg;
}

// FP64 partial slots the workspace holds: the one-step layout's one per wave, or, when the
// two-step kernel may reduce, one per (tile, wave) of its launch (its reducing launch writes
// one per tile, its waves summed in order; the slots keep room for a partial per wave)
int two_step_waves(const lbm_params& p, const TwoStepShape& sh)
{
    return ((p.nx + k2Cols - 1) / k2Cols) * ((p.ny + sh.rows - 1) / sh.rows) * sh.waves;
}

// partials of a reducing two-step launch: one per tile (its waves summed in order)
int two_step_tiles(const lbm_params& p, const TwoStepShape& sh)
{
    return ((p.nx + k2Cols - 1) / k2Cols) * ((p.ny + sh.rows - 1) / sh.rows);
}

// the most any candidate shape of p needs (the workspace holds them)
int two_step_waves_max(const lbm_params& p)
{
    TwoStepShape cand[kMaxShapes];
    const int n = two_step_candidates(p, cand);
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const int w = two_step_waves(p, cand[i]);
        m = w > m ? w : m;
    }
    return m;
}

int partial_slots(const lbm_params& p)
{
    int strips, seg_h, nseg, blk;
    int n = decompose(p, &strips, &seg_h, &nseg, &blk);
    if (resolve_variant(p) == LBM_VARIANT_BLOCK2) {
        const int n2 = two_step_waves_max(p);
        n = n2 > n ? n2 : n;
    }
    if (resolve_variant(p) == LBM_VARIANT_AA) {
        const int na = aa_slots(p);
        n = na > n ? na : n;
    }
    return n;
}

size_t ws_layout(int nwork, size_t* off_part, size_t* off_hist, size_t* off_red)
{
    size_t o = 256;  // error word
    *off_part = o;
    o += ((size_t)nwork * 3 * sizeof(double) + 255) & ~(size_t)255;
    o += (size_t)kRedBlocks * 3 * sizeof(double);  // per-block sums of the two-pass reduction
    *off_hist = o;
    o += (size_t)kHistCap * 4 * sizeof(double);
    *off_red = o;
    o += 256;
    return o;
}

void fill_args(lbm_ctx* c)
{
    const lbm_params& p = c->P;
    StepArgs& A = c->args;
    std::memset(&A, 0, sizeof(A));
    A.plane = c->plane;
    A.nx = p.nx;
    A.ny = p.ny;
    A.ld = c->ld;
    A.walls = p.walls;
    A.nwork = decompose(p, &A.strips, &A.seg_h, &A.nseg, &A.blk);
    A.var_tau = p.var_tau;
    A.G = p.G;
    A.sigma = p.sigma;
    for (int k = 0; k < 9; ++k) A.s[k] = 1.0 / p.tau[k];
    fill_coef(A, p.tau, p.G, p.sigma);
    A.tau_v = p.tau_v;
    A.rho_v_tau = p.rho_v_tau;
    A.dtau_drho = p.var_tau ? (p.tau_l - p.tau_v) / (p.rho_l_tau - p.rho_v_tau) : 0.0;
    A.tau_lo = std::fmin(p.tau_l, p.tau_v);
    A.tau_hi = std::fmax(p.tau_l, p.tau_v);
    A.rho_ref = p.prec == LBM_FP32_SHIFTED ? p.rho_ref : 0.0;
    A.eos = dev_eos(p.eos);
    auto psi_host = [&](double r) {
        const double q = 2.0 * (lbm_eos_pressure(&p.eos, r) - r / 3.0) / p.G;
        return q > 0 ? std::sqrt(q) : 0.0;
    };
    A.psi_lo = p.walls ? psi_host(p.rho_wall_lo) : 0.0;
    A.psi_hi = p.walls ? psi_host(p.rho_wall_hi) : 0.0;
    A.partials = c->partials;
    A.err = c->err;
    const TwoStepShape sh = c->shape;
    c->rows2 = sh.rows2;
    A.rows2t = sh.rows;
    A.strips2 = (p.nx + k2Cols - 1) / k2Cols;
    A.bands2 = (p.ny + sh.rows - 1) / sh.rows;
    A.pcols2 = (A.strips2 + kPatchW - 1) / kPatchW;
    A.pw_last = A.strips2 - (A.pcols2 - 1) * kPatchW;
    // umulhi(n, ceil(2^32/d)) = n / d exactly while n * d < 2^32: the multiplier exceeds
    // 2^32/d by less than 1, which moves n/d by less than n/2^32 < 1/d.  The kernel divides
    // slots (below the grid size) by 8 x strips and offsets within a patch row (below 64) by
    // pw_last.
    const long long prow = (long long)kPatchH * A.strips2;
    const long long slots = ((A.bands2 + kPatchH - 1) / kPatchH) * prow;
    A.patched = A.strips2 * A.bands2 > kPatchMinTiles && A.strips2 >= 2 * kPatchW && A.bands2 >= 2 * kPatchH &&
                (slots + 8) * prow < (1LL << 32);
    A.prow_magic = (unsigned)((((unsigned long long)1 << 32) + prow - 1) / prow);
    A.pwl_magic = A.pw_last > 1 ? (unsigned)((((unsigned long long)1 << 32) + A.pw_last - 1) / A.pw_last) : 0u;
    const int blocks = A.blk ? A.nwork / kBlkWaves : (A.nwork + kWaves - 1) / kWaves;
    c->grid = (blocks + 7) & ~7;
    c->blk2 = resolve_variant(p) == LBM_VARIANT_BLOCK2;
    c->grid2 = patch_grid(c->args.strips2, c->args.bands2, c->args.patched);
}

bool launch_reduce(lbm_ctx* c, double* out, long long step, int with_step, hipStream_t s)
{
    return launch_reduce_n(c, c->args.nwork, out, step, with_step, s);
}

// the same over the first n partial slots
bool launch_reduce_n(lbm_ctx* c, int n, double* out, long long step, int with_step, hipStream_t s)
{
    if (n <= kRedOneMax) {
        hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(1024), 0, s, (const double*)c->partials, n, out, step, with_step);
        return hip_ok(hipGetLastError(), "reduction launch");
    }
    int nb = (n + 1023) / 1024;
    nb = nb < 1 ? 1 : (nb > kRedBlocks ? kRedBlocks : nb);
    const int chunk = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nb), dim3(256), 0, s, (const double*)c->partials, n, chunk, c->redblk);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const double*)c->redblk, nb, out, step, with_step);
    return hip_ok(hipGetLastError(), "reduction launch");
}

// one forward step of the row-block kernel that also records (drho, j, psi) per node
bool launch_record_step(lbm_ctx* c, void* rec, hipStream_t s)
{
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    A.dst = c->buf[c->cur ^ 1];
    A.step = c->step;
    A.rec = rec;
    A.rec_plane = (size_t)c->P.nx * c->P.ny;
    if (!A.blk) {
        // recording always uses the row-block decomposition (same node arithmetic)
        int strips, seg_h, nseg, blk;
        lbm_params q = c->P;
        q.kernel_variant = LBM_VARIANT_BLOCK;
        A.nwork = decompose(q, &strips, &seg_h, &nseg, &blk);
        A.strips = strips;
        A.seg_h = seg_h;
        A.nseg = nseg;
        A.blk = 1;
    }
    const int grid = ((A.nwork / kBlkWaves) + 7) & ~7;
    if (c->P.prec == LBM_FP32_SHIFTED)
        hipLaunchKernelGGL((k_step_blk<float, MODE_RECORD>), dim3(grid), dim3(64 * kBlkWaves), 0, s, A);
    else
        hipLaunchKernelGGL((k_step_blk<double, MODE_RECORD>), dim3(grid), dim3(64 * kBlkWaves), 0, s, A);
    return hip_ok(hipGetLastError(), "k_step_blk(record) launch");
}

// two steps in one launch (LBM_VARIANT_BLOCK2): source buf[cur], result in buf[cur ^ 1];
// rec non-NULL: also record both steps (rec, then rec + one step's record)
template <typename T>
bool launch_step2(lbm_ctx* c, void* rec, hipStream_t s, bool reduce = false)
{
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    A.dst = c->buf[c->cur ^ 1];
    A.step = c->step;
    A.rec = rec;
    A.rec_plane = (size_t)c->P.nx * c->P.ny;
    const dim3 g(c->grid2), b(64 * (c->rows2 ? k2rWavesOf<T> : k2WavesOf<T>));
    // streaming stores for small lattices (kStreamBytes)
    const bool nt = 2 * c->pop_bytes <= kStreamBytes;
    if (c->rows2) {
        if (c->P.walls) {
            if (rec && nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_RECORD, true, true>), g, b, 0, s, A);
            else if (rec) hipLaunchKernelGGL((k_step2_rows2<T, MODE_RECORD, true>), g, b, 0, s, A);
            else if (reduce && nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP_REDUCE, true, true>), g, b, 0, s, A);
            else if (reduce) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP_REDUCE, true>), g, b, 0, s, A);
            else if (nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP, true, true>), g, b, 0, s, A);
            else hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP, true>), g, b, 0, s, A);
        } else {
            if (rec && nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_RECORD, false, true>), g, b, 0, s, A);
            else if (rec) hipLaunchKernelGGL((k_step2_rows2<T, MODE_RECORD, false>), g, b, 0, s, A);
            else if (reduce && nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP_REDUCE, false, true>), g, b, 0, s, A);
            else if (reduce) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP_REDUCE, false>), g, b, 0, s, A);
            else if (nt) hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP, false, true>), g, b, 0, s, A);
            else hipLaunchKernelGGL((k_step2_rows2<T, MODE_STEP, false>), g, b, 0, s, A);
        }
        return hip_ok(hipGetLastError(), "k_step2_rows2 launch");
    }
    if (c->P.walls) {
        if (rec && nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_RECORD, true, true>), g, b, 0, s, A);
        else if (rec) hipLaunchKernelGGL((k_step2_blk<T, MODE_RECORD, true>), g, b, 0, s, A);
        else if (reduce && nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP_REDUCE, true, true>), g, b, 0, s, A);
        else if (reduce) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP_REDUCE, true>), g, b, 0, s, A);
        else if (nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP, true, true>), g, b, 0, s, A);
        else hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP, true>), g, b, 0, s, A);
    } else {
        if (rec && nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_RECORD, false, true>), g, b, 0, s, A);
        else if (rec) hipLaunchKernelGGL((k_step2_blk<T, MODE_RECORD, false>), g, b, 0, s, A);
        else if (reduce && nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP_REDUCE, false, true>), g, b, 0, s, A);
        else if (reduce) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP_REDUCE, false>), g, b, 0, s, A);
        else if (nt) hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP, false, true>), g, b, 0, s, A);
        else hipLaunchKernelGGL((k_step2_blk<T, MODE_STEP, false>), g, b, 0, s, A);
    }
    return hip_ok(hipGetLastError(), "k_step2_blk launch");
}

bool launch_record_pair(lbm_ctx* c, void* rec, hipStream_t s)
{
    return c->P.prec == LBM_FP32_SHIFTED ? launch_step2<float>(c, rec, s) : launch_step2<double>(c, rec, s);
}

// FP64 mass/momentum partials of the current state (no step), then the reduction
bool launch_partials(lbm_ctx* c, double* out, long long step, hipStream_t s)
{
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    A.dst = nullptr;
    A.step = c->step;
    const bool f32 = c->P.prec == LBM_FP32_SHIFTED;
    if (A.blk) {
        if (f32) hipLaunchKernelGGL((k_step_blk<float, MODE_MACROS>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
        else hipLaunchKernelGGL((k_step_blk<double, MODE_MACROS>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
    } else {
        if (f32) hipLaunchKernelGGL((k_step<float, MODE_MACROS>), dim3(c->grid), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_step<double, MODE_MACROS>), dim3(c->grid), dim3(256), 0, s, A);
    }
    if (!hip_ok(hipGetLastError(), "k_step(partials) launch")) return false;
    return launch_reduce(c, out, step, 1, s);
}

// record of step t in the forward record buffer (lbm_set_recording)
void* record_slot(lbm_ctx* c, int64_t t)
{
    const size_t tsz = c->P.prec == LBM_FP32_SHIFTED ? sizeof(float) : sizeof(double);
    return (char*)c->rec_all + (size_t)t * 4 * (size_t)c->P.nx * c->P.ny * tsz;
}

template <typename T>
bool launch_step(lbm_ctx* c, int mode, hipStream_t s)
{
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    A.dst = c->buf[c->cur ^ 1];
    A.step = c->step;
    if (A.blk) {
        if (mode == MODE_STEP) hipLaunchKernelGGL((k_step_blk<T, MODE_STEP>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
        else hipLaunchKernelGGL((k_step_blk<T, MODE_STEP_REDUCE>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
    } else {
        if (mode == MODE_STEP) hipLaunchKernelGGL((k_step<T, MODE_STEP>), dim3(c->grid), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_step<T, MODE_STEP_REDUCE>), dim3(c->grid), dim3(256), 0, s, A);
    }
    return hip_ok(hipGetLastError(), "k_step launch");
}

}  // namespace lbmk

extern "C" {

const char* lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EUNSTABLE: return "unstable (psi^2 < 0 or non-finite density)";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ESTATE: return "call out of order";
    case LBM_ENOROOT: return "no root in the admissible bracket";
    default: return "unknown error";
    }
}

int lbm_layout(const lbm_params* p, int* ld_out, size_t* pop_bytes_out, size_t* ws_bytes_out)
{
    if (!p || p->nx < 1 || p->ny < 1) {
        lbm_set_error("lbm_layout: invalid lattice size");
        return LBM_EINVAL;
    }
    const int ld = (p->nx + 63) & ~63;
    if ((long long)ld * p->ny * 8 >= (1LL << 32)) {
        lbm_set_error("lbm_layout: one population plane must stay below 4 GiB (lattice too large)");
        return LBM_EINVAL;
    }
    const size_t plane = (size_t)ld * p->ny;
    const size_t bytes = p->prec == LBM_FP32_SHIFTED ? plane * (8 * sizeof(float) + sizeof(double)) : plane * 9 * sizeof(double);
    int strips, seg_h, nseg, blk;
    decompose(*p, &strips, &seg_h, &nseg, &blk);
    size_t a, b, d;
    size_t ws = ws_layout(partial_slots(*p), &a, &b, &d);
    if (resolve_variant(*p) == LBM_VARIANT_AA) ws += aa_psi_bytes(*p, ld);  // the psi plane
    if (ld_out) *ld_out = ld;
    if (pop_bytes_out) *pop_bytes_out = bytes;
    if (ws_bytes_out) *ws_bytes_out = ws;
    return LBM_OK;
}

int lbm_describe(const lbm_params* p, int* variant_out, int* band_rows_out, int* waves_out)
{
    if (!p || p->nx < 1 || p->ny < 1) {
        lbm_set_error("lbm_describe: invalid lattice size");
        return LBM_EINVAL;
    }
    int strips, seg_h, nseg, blk;
    const int nw = decompose(*p, &strips, &seg_h, &nseg, &blk);
    const int v = resolve_variant(*p);
    if (variant_out) *variant_out = v;
    if (v == LBM_VARIANT_BLOCK2) {
        const TwoStepShape sh = two_step_shape(*p);
        if (band_rows_out) *band_rows_out = sh.rows;
        if (waves_out) *waves_out = sh.waves;
    } else if (v == LBM_VARIANT_AA) {
        // 256-thread workgroups of 4 rows x 64 columns, one wavefront per row
        if (band_rows_out) *band_rows_out = 4;
        if (waves_out) *waves_out = 4;
    } else {
        if (band_rows_out) *band_rows_out = seg_h;
        if (waves_out) *waves_out = nw;
    }
    return LBM_OK;
}

int lbm_tile_shape(const lbm_ctx* c, int* rows_out, int* waves_out)
{
    if (!c || !c->blk2) {
        lbm_set_error("lbm_tile_shape: a context of the two-step variant is required");
        return LBM_EINVAL;
    }
    if (rows_out) *rows_out = c->shape.rows;
    if (waves_out) *waves_out = c->shape.waves;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Checks of lbm_init's arguments; the workspace size a lattice needs goes to *need.
int check_init(const lbm_params* p, void* f_a, void* f_b, const double* rho0, size_t* need)
{
    int st = validate(p);
    if (st != LBM_OK) return st;
    if (resolve_variant(*p) == LBM_VARIANT_AA) {
        if (!f_a || f_b || !rho0) {
            lbm_set_error("lbm_init: the in-place AA variant takes one population buffer (f_b NULL); rho0 non-NULL");
            return LBM_EINVAL;
        }
    } else if (!f_a || !f_b || f_a == f_b || !rho0) {
        lbm_set_error("lbm_init: population buffers must be non-NULL and distinct; rho0 non-NULL");
        return LBM_EINVAL;
    }
    int ld;
    size_t pop_bytes;
    lbm_layout(p, &ld, &pop_bytes, need);
    return LBM_OK;
}

// tile_rows = -1: time each candidate two-step tile shape and keep the fastest.  The timed
// launches advance the lattice from its initial state, alternating the two population
// buffers as a run does (so that each launch reads what the one before it wrote, as in the
// L2 and the MALL of a real run); the caller writes the initial state again afterwards.
// Three rounds over the candidates, each candidate one launch to warm up and then 4 timed,
// and a candidate's time is its best round, so that a stall in one round does not decide.
int time_tile_shapes(lbm_ctx* c, hipStream_t s)
{
    TwoStepShape cand[kMaxShapes];
    const int n = two_step_candidates(c->P, cand);
    if (n <= 1) return LBM_OK;
    hipEvent_t e0, e1;
    if (!hip_ok(hipEventCreate(&e0), "tile timing event")) return LBM_EHIP;
    if (!hip_ok(hipEventCreate(&e1), "tile timing event")) {
        (void)hipEventDestroy(e0);
        return LBM_EHIP;
    }
    const bool f32 = c->P.prec == LBM_FP32_SHIFTED;
    float best_ms[kMaxShapes];
    bool ok = true;
    for (int round = 0; round < 3 && ok; ++round) {
        for (int i = 0; i < n && ok; ++i) {
            c->shape = cand[i];
            fill_args(c);
            for (int r = 0; r < 5 && ok; ++r) {
                if (r == 1) ok = hip_ok(hipEventRecord(e0, s), "tile timing");
                if (ok) ok = f32 ? launch_step2<float>(c, nullptr, s) : launch_step2<double>(c, nullptr, s);
                c->cur ^= 1;
                c->step += 2;
            }
            float ms = 0.0f;
            ok = ok && hip_ok(hipEventRecord(e1, s), "tile timing") && hip_ok(hipEventSynchronize(e1), "tile timing") &&
                 hip_ok(hipEventElapsedTime(&ms, e0, e1), "tile timing");
            if (ok && (round == 0 || ms < best_ms[i])) best_ms[i] = ms;
        }
    }
    int best = 0;
    for (int i = 1; i < n && ok; ++i)
        if (best_ms[i] < best_ms[best]) best = i;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->cur = 0;
    c->step = 0;
    if (!ok) return LBM_EHIP;
    c->shape = cand[best];
    fill_args(c);
    return LBM_OK;
}

// Fill context c over the caller's population buffers and the workspace ws, and write the
// initial state (lbm_init and lbm_init_static)
int init_ctx(lbm_ctx* c, const lbm_params* p, void* f_a, void* f_b, void* ws, size_t ws_bytes, const double* rho0,
             const double* ux0, const double* uy0, void* stream)
{
    int ld;
    size_t pop_bytes, need;
    lbm_layout(p, &ld, &pop_bytes, &need);
    c->P = *p;
    c->ld = ld;
    c->plane = (size_t)ld * p->ny;
    c->pop_bytes = pop_bytes;
    c->aa = resolve_variant(*p) == LBM_VARIANT_AA;
    c->buf[0] = f_a;
    c->buf[1] = c->aa ? f_a : f_b;
    c->cur = 0;
    c->step = 0;
    c->ws = (char*)ws;
    c->ws_bytes = ws_bytes;
    size_t op, oh, orr;
    const size_t ws_base = ws_layout(partial_slots(*p), &op, &oh, &orr);
    c->aa_psi = c->aa ? c->ws + ws_base : nullptr;
    c->err = (unsigned*)c->ws;
    c->partials = (double*)(c->ws + op);
    c->redblk = (double*)(c->ws + oh - (size_t)kRedBlocks * 3 * sizeof(double));
    c->hist = (double*)(c->ws + oh);
    c->red = (double*)(c->ws + orr);
    c->hist_count = 0;
    c->shape = two_step_shape(*p);
    fill_args(c);
    hipStream_t s = (hipStream_t)stream;
    const unsigned init_err[2] = {0u, 0xffffffffu};
    if (!hip_ok(hipMemcpyAsync(c->err, init_err, sizeof(init_err), hipMemcpyHostToDevice, s), "lbm_init error word") ||
        !hip_ok(hipStreamSynchronize(s), "lbm_init sync"))
        return LBM_EHIP;
    if (c->aa) return aa_init(c, rho0, ux0, uy0, s) ? LBM_OK : LBM_EHIP;
    // tile_rows = -1: the candidate shapes are timed on the lattice's own run from the initial
    // state, which is then written again (and the error word cleared) for the real run
    const bool timed = c->blk2 && p->tile_rows == -1;
    for (int pass = 0; pass < (timed ? 2 : 1); ++pass) {
        StepArgs A = c->args;
        A.dst = c->buf[0];
        dim3 g((p->nx + 127) / 128, p->ny);
        if (p->prec == LBM_FP32_SHIFTED) hipLaunchKernelGGL(k_init<float>, g, dim3(128), 0, s, A, rho0, ux0, uy0);
        else hipLaunchKernelGGL(k_init<double>, g, dim3(128), 0, s, A, rho0, ux0, uy0);
        if (!hip_ok(hipGetLastError(), "k_init launch")) return LBM_EHIP;
        if (timed && pass == 0) {
            const int st = time_tile_shapes(c, s);
            if (st != LBM_OK) return st;
            if (!hip_ok(hipMemcpyAsync(c->err, init_err, sizeof(init_err), hipMemcpyHostToDevice, s),
                        "lbm_init error word"))
                return LBM_EHIP;
        }
    }
    return timed ? (hip_ok(hipStreamSynchronize(s), "lbm_init sync") ? LBM_OK : LBM_EHIP) : LBM_OK;
}

// Workspace of lbm_init_static: one file-scope array per GPU (each device the library runs
// on holds its own copy until the process ends).  Host code never names the array except to
// look its address up: the name is a host stand-in, and a kernel given it would fault.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
char* g_scratch[kMaxDevices];        // device address of `scratch` on each device, once looked up
lbm_ctx g_static_ctx[kMaxDevices];   // the one context per device that lbm_init_static hands out
std::mutex g_scratch_mu;

// Device address of the current device's scratch array (looked up once per device).
char* scratch_of_current_device(int* dev_out)
{
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "lbm_init_static hipGetDevice")) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        lbm_set_error("lbm_init_static: device index beyond the library's table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "lbm_init_static hipGetSymbolAddress") || !ptr)
            return nullptr;
        g_scratch[dev] = (char*)ptr;
    }
    *dev_out = dev;
    return g_scratch[dev];
}

}  // namespace

extern "C" {

int lbm_init(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b, void* ws, size_t ws_bytes,
             const double* rho0, const double* ux0, const double* uy0, void* stream)
{
    if (!out) {
        lbm_set_error("lbm_init: null context pointer");
        return LBM_EINVAL;
    }
    *out = nullptr;
    size_t need;
    int st = check_init(p, f_a, f_b, rho0, &need);
    if (st != LBM_OK) return st;
    if (!ws) {
        lbm_set_error("lbm_init: ws must be non-NULL");
        return LBM_EINVAL;
    }
    if (ws_bytes < need) {
        lbm_set_error("lbm_init: workspace smaller than lbm_layout requires");
        return LBM_EINVAL;
    }
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_EINVAL;
    st = init_ctx(c, p, f_a, f_b, ws, ws_bytes, rho0, ux0, uy0, stream);
    if (st != LBM_OK) {
        delete c;
        return st;
    }
    *out = c;
    return LBM_OK;
}

int lbm_init_static(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b, const double* rho0, const double* ux0,
                    const double* uy0, void* stream)
{
    if (!out) {
        lbm_set_error("lbm_init_static: null context pointer");
        return LBM_EINVAL;
    }
    *out = nullptr;
    size_t need;
    int st = check_init(p, f_a, f_b, rho0, &need);
    if (st != LBM_OK) return st;
    if (p->tile_rows == -1) {
        // the timing creates HIP events: not for callers that cannot allocate
        lbm_set_error("lbm_init_static: tile_rows = -1 (timed tile shapes) is not available here; use 0 or a height");
        return LBM_EINVAL;
    }
    if (need > kScratchBytes) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "lbm_init_static: the lattice needs %zu bytes of workspace, more than the "
                                        "library's static %zu", need, kScratchBytes);
        lbm_set_error(buf);
        return LBM_EINVAL;
    }
    int dev = -1;
    char* ws = scratch_of_current_device(&dev);
    if (!ws) return LBM_EHIP;
    lbm_ctx* c = &g_static_ctx[dev];
    *c = lbm_ctx();
    c->is_static = true;
    st = init_ctx(c, p, f_a, f_b, ws, kScratchBytes, rho0, ux0, uy0, stream);
    if (st != LBM_OK) return st;
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t nsteps, void* stream)
{
    if (!c || nsteps < 0) {
        lbm_set_error("lbm_step: invalid arguments");
        return LBM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = c->P.prec == LBM_FP32_SHIFTED;
    const int re = c->P.reduce_every;
    if (c->rec_all && c->step + nsteps > c->rec_steps) {
        lbm_set_error("lbm_step: the forward record (lbm_set_recording) holds fewer steps");
        return LBM_ESTATE;
    }
    // the last checkpoint these steps take (at step t with t % K == 0) must have a slot
    if (c->ckpt_K > 0 && nsteps > 0) {
        const int64_t last = c->step + nsteps - 1;
        const int64_t first_ck = (c->step + c->ckpt_K - 1) / c->ckpt_K * c->ckpt_K;
        if (first_ck <= last && last / c->ckpt_K >= c->ckpt_slots) {
            lbm_set_error("lbm_step: checkpoint buffer full (more steps than slots * K)");
            return LBM_ESTATE;
        }
    }
    if (c->aa) {
        // in place, two launches per step (psi plane, then the update); no records or checkpoints
        for (int64_t k = 0; k < nsteps; ++k) {
            const bool red = re > 0 && (c->step % re) == 0;
            if (!aa_step(c, red ? MODE_STEP_REDUCE : MODE_STEP, s)) return LBM_EHIP;
            if (red) {
                double* row = c->hist + 4 * (c->hist_count % kHistCap);
                if (!launch_reduce_n(c, aa_slots(c->P), row, (long long)c->step, 1, s)) return LBM_EHIP;
                c->hist_count++;
            }
            c->step++;
        }
        return LBM_OK;
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        if (c->ckpt_K > 0 && c->step % c->ckpt_K == 0) {
            const int64_t slot = c->step / c->ckpt_K;
            if (slot >= c->ckpt_slots) {
                lbm_set_error("lbm_step: checkpoint buffer full (more steps than slots * K)");
                return LBM_ESTATE;
            }
            if (!hip_ok(hipMemcpyAsync((char*)c->ckpt + slot * c->pop_bytes, c->buf[c->cur], c->pop_bytes,
                                       hipMemcpyDeviceToDevice, s),
                        "checkpoint copy"))
                return LBM_EHIP;
        }
        const bool red = re > 0 && (c->step % re) == 0;
        void* rec = c->rec_all ? record_slot(c, c->step) : nullptr;
        // two steps in one launch when this step does not reduce and no checkpoint falls
        // between them; if the second step reduces, the launch leaves its partials (a
        // recording forward reduces in a pass of its own instead)
        const bool red2 = re > 0 && (c->step + 1) % re == 0;
        if (c->blk2 && !red && k + 1 < nsteps && !(red2 && rec) &&
            !(c->ckpt_K > 0 && (c->step + 1) % c->ckpt_K == 0)) {
            if (!(f32 ? launch_step2<float>(c, rec, s, red2) : launch_step2<double>(c, rec, s, red2)))
                return LBM_EHIP;
            if (red2) {
                double* row = c->hist + 4 * (c->hist_count % kHistCap);
                if (!launch_reduce_n(c, two_step_tiles(c->P, c->shape), row, (long long)c->step + 1, 1, s))
                    return LBM_EHIP;
                c->hist_count++;
            }
            c->cur ^= 1;
            c->step += 2;
            ++k;
            continue;
        }
        if (rec) {
            // recording forward: the reduction reads the state first, then the step records
            if (red) {
                double* row = c->hist + 4 * (c->hist_count % kHistCap);
                if (!launch_partials(c, row, (long long)c->step, s)) return LBM_EHIP;
                c->hist_count++;
            }
            if (!launch_record_step(c, rec, s)) return LBM_EHIP;
            c->cur ^= 1;
            c->step++;
            continue;
        }
        const int mode = red ? MODE_STEP_REDUCE : MODE_STEP;
        if (!(f32 ? launch_step<float>(c, mode, s) : launch_step<double>(c, mode, s))) return LBM_EHIP;
        if (red) {
            double* row = c->hist + 4 * (c->hist_count % kHistCap);
            if (!launch_reduce(c, row, (long long)c->step, 1, s)) return LBM_EHIP;
            c->hist_count++;
        }
        c->cur ^= 1;
        c->step++;
    }
    return LBM_OK;
}

int lbm_status_check(lbm_ctx* c, void* stream)
{
    if (!c) return LBM_EINVAL;
    unsigned h[2];
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMemcpyAsync(h, c->err, sizeof(h), hipMemcpyDeviceToHost, s), "status copy") ||
        !hip_ok(hipStreamSynchronize(s), "status sync"))
        return LBM_EHIP;
    if (h[0]) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "lbm: psi^2 < 0 or non-positive density first met at step %u", h[1]);
        lbm_set_error(buf);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

int lbm_macros(lbm_ctx* c, double* rho, double* ux, double* uy, double* psi, double* p, double* Fx, double* Fy,
               double* host_mass_mom, void* stream)
{
    if (!c) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    A.dst = nullptr;
    A.step = c->step;
    A.o_rho = rho;
    A.o_ux = ux;
    A.o_uy = uy;
    A.o_psi = psi;
    A.o_p = p;
    A.o_fx = Fx;
    A.o_fy = Fy;
    const bool f32 = c->P.prec == LBM_FP32_SHIFTED;
    if (c->aa) {
        double* const out[7] = {rho, ux, uy, psi, p, Fx, Fy};
        if (!aa_macros(c, out, s) || !launch_reduce_n(c, aa_slots(c->P), c->red, 0LL, 0, s)) return LBM_EHIP;
    } else if (A.blk) {
        if (f32) hipLaunchKernelGGL((k_step_blk<float, MODE_MACROS>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
        else hipLaunchKernelGGL((k_step_blk<double, MODE_MACROS>), dim3(c->grid), dim3(64 * kBlkWaves), 0, s, A);
    } else {
        if (f32) hipLaunchKernelGGL((k_step<float, MODE_MACROS>), dim3(c->grid), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_step<double, MODE_MACROS>), dim3(c->grid), dim3(256), 0, s, A);
    }
    if (!hip_ok(hipGetLastError(), "k_step(macros) launch")) return LBM_EHIP;
    if (!c->aa && !launch_reduce(c, c->red, 0LL, 0, s)) return LBM_EHIP;
    double h[3];
    if (!hip_ok(hipMemcpyAsync(h, c->red, sizeof(h), hipMemcpyDeviceToHost, s), "macros copy") ||
        !hip_ok(hipStreamSynchronize(s), "macros sync"))
        return LBM_EHIP;
    if (host_mass_mom) std::memcpy(host_mass_mom, h, sizeof(h));
    return lbm_status_check(c, stream);
}

int lbm_populations(lbm_ctx* c, double* f_out, void* stream)
{
    if (!c || !f_out) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (c->aa) return aa_populations(c, f_out, s) ? LBM_OK : LBM_EHIP;
    StepArgs A = c->args;
    A.src = c->buf[c->cur];
    dim3 g((c->P.nx + 127) / 128, c->P.ny);
    if (c->P.prec == LBM_FP32_SHIFTED) hipLaunchKernelGGL(k_populations<float>, g, dim3(128), 0, s, A, f_out);
    else hipLaunchKernelGGL(k_populations<double>, g, dim3(128), 0, s, A, f_out);
    return hip_ok(hipGetLastError(), "k_populations launch") ? LBM_OK : LBM_EHIP;
}

int lbm_history(lbm_ctx* c, double* host_rows, int max_rows, int* n_out, void* stream)
{
    if (!c || !host_rows || max_rows < 0) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t avail = c->hist_count < kHistCap ? c->hist_count : kHistCap;
    const int n = (int)(avail < max_rows ? avail : max_rows);
    // newest n rows, oldest first
    for (int k = 0; k < n; ++k) {
        const int64_t idx = (c->hist_count - n + k) % kHistCap;
        if (!hip_ok(hipMemcpyAsync(host_rows + 4 * k, c->hist + 4 * idx, 4 * sizeof(double), hipMemcpyDeviceToHost, s),
                    "history copy"))
            return LBM_EHIP;
    }
    if (!hip_ok(hipStreamSynchronize(s), "history sync")) return LBM_EHIP;
    if (n_out) *n_out = n;
    return LBM_OK;
}

int lbm_state(lbm_ctx* c, int64_t* step_out, int* cur_out)
{
    if (!c) return LBM_EINVAL;
    if (step_out) *step_out = c->step;
    if (cur_out) *cur_out = c->cur;
    return LBM_OK;
}

int lbm_save(lbm_ctx* c, void* dst, void* stream)
{
    if (!c || !dst) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMemcpyAsync(dst, c->buf[c->cur], c->pop_bytes, hipMemcpyDefault, s), "lbm_save copy") ||
        !hip_ok(hipStreamSynchronize(s), "lbm_save sync"))
        return LBM_EHIP;
    return LBM_OK;
}

int lbm_load(lbm_ctx* c, const void* src, int64_t step, void* stream)
{
    if (!c || !src || step < 0) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMemcpyAsync(c->buf[c->cur], src, c->pop_bytes, hipMemcpyDefault, s), "lbm_load copy") ||
        !hip_ok(hipStreamSynchronize(s), "lbm_load sync"))
        return LBM_EHIP;
    c->step = step;
    if (step != 0) {
        // the records and checkpoints belong to another trajectory: an adjoint over them would mix
        // the two, so the loaded state carries none (lbm_adjoint then reports LBM_ESTATE)
        c->rec_all = nullptr;
        c->rec_steps = 0;
        c->ckpt = nullptr;
        c->ckpt_K = 0;
        c->ckpt_slots = 0;
    }
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c)
{
    if (c && !c->is_static) delete c;  // the context of lbm_init_static belongs to the library
}

}  // extern "C"
