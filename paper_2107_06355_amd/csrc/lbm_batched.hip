// liblbm.so: many independent lattices advanced together, in one of two ways.
//
// Persistent: each lattice (its own size, EOS, relaxation times and FP32
// shift) is owned by one workgroup of 16 wavefronts that loops over the time
// steps with a workgroup barrier between steps: neighbouring nodes of a
// lattice are only ever touched by that workgroup, so no grid-wide
// synchronisation is needed.  Best for many small lattices (no launch per step).
// Grouped: one launch per time step over all lattices, one wavefront per
// (lattice, 62-column strip, row); the launches of a chunk of steps are
// replayed as a HIP graph.  Best when a large lattice would keep one
// workgroup busy for many items per step while most CUs idle.
// Populations of all lattices are packed back to back in one pair of buffers;
// scalar fields are packed in the same lattice order ([ny_b][nx_b] each).
// The per-node arithmetic is the fused step of lbm_device.h: pull with
// half-way bounce-back, shaped EOS, psi (Eq. InteractionPotential), the
// Shan-Chen stencil (Eq. ShanChenForce) and the MRT update with Eq. LiFS.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace {

using namespace lbmk;

constexpr int kBatchWaves = 16;

struct BatchItem {
    StepArgs A;           // per-lattice arguments (src/dst filled in the kernel)
    size_t off_bytes;     // byte offset of the lattice in each population buffer
    long long cell_off;   // offset of the lattice in the packed scalar fields
};

template <typename T, int MODE>
__global__ __launch_bounds__(64 * kBatchWaves) void k_batch(const BatchItem* items, char* buf0, char* buf1, int cur0,
                                                            long long nsteps, long long step0, double* o_rho,
                                                            double* o_ux, double* o_uy)
{
    StepArgs A = items[blockIdx.x].A;
    const size_t off = items[blockIdx.x].off_bytes;
    const long long coff = items[blockIdx.x].cell_off;
    if (MODE == MODE_MACROS) {
        A.o_rho = o_rho ? o_rho + coff : nullptr;
        A.o_ux = o_ux ? o_ux + coff : nullptr;
        A.o_uy = o_uy ? o_uy + coff : nullptr;
        A.o_psi = A.o_p = A.o_fx = A.o_fy = nullptr;
    }
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int work = A.strips * A.ny;  // one item = one row of one 62-column strip
    int cur = cur0;
    Acc acc = {0.0, 0.0, 0.0};
    for (long long t = 0; t < nsteps; ++t) {
        A.src = (cur ? buf1 : buf0) + off;
        A.dst = (cur ? buf0 : buf1) + off;
        A.step = step0 + t;
        const View<T> V = make_view<T>(A.src, A.plane);
        for (int w = wv; w < work; w += kBatchWaves) {
            const int strip = w % A.strips, y = w / A.strips;
            Lane L;
            L.lane = threadIdx.x & 63;
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
            Row<T> Rm, Rc, Rp;
            pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y - 1), Rm.g0, Rm.g);
            pull<T>(V, A, L.x, L.xm, L.xp, y, Rc.g0, Rc.g);
            pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y + 1), Rp.g0, Rp.g);
            const double dm = node_drho<T>(Rm.g0, Rm.g), dc = node_drho<T>(Rc.g0, Rc.g), dp = node_drho<T>(Rp.g0, Rp.g);
            const T psm = (A.walls && y == 0) ? (T)A.psi_lo : node_psi<T>(A, dm, L.valid);
            const T psc = node_psi<T>(A, dc, L.valid);
            const T psp = (A.walls && y == A.ny - 1) ? (T)A.psi_hi : node_psi<T>(A, dp, L.valid);
            collide_row<T, MODE>(A, L, y, Rc, dc, psm, psc, psp, acc);
        }
        if (MODE == MODE_MACROS) break;
        __syncthreads();  // this lattice's step t is complete before any wave pulls for t+1
        cur ^= 1;
    }
}

// One step of every lattice: wave w takes item w of the concatenated item lists
// (lattice b owns items [item_off[b], item_off[b+1]), item = strip + strips * row).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_step(const BatchItem* items, const int* item_off, int B, char* buf0,
                                                    char* buf1, int cur, long long step)
{
    const int w = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= item_off[B]) return;
    int lo = 0, hi = B;  // item_off[lo] <= w < item_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_off[mid] <= w) lo = mid;
        else hi = mid;
    }
    StepArgs A = items[lo].A;
    const size_t off = items[lo].off_bytes;
    A.src = (cur ? buf1 : buf0) + off;
    A.dst = (cur ? buf0 : buf1) + off;
    A.step = step;
    const int item = w - item_off[lo];
    const int strip = item % A.strips, y = item / A.strips;
    Lane L;
    L.lane = threadIdx.x & 63;
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
    const View<T> V = make_view<T>(A.src, A.plane);
    Row<T> Rm, Rc, Rp;
    pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y - 1), Rm.g0, Rm.g);
    pull<T>(V, A, L.x, L.xm, L.xp, y, Rc.g0, Rc.g);
    pull<T>(V, A, L.x, L.xm, L.xp, load_index(A, y + 1), Rp.g0, Rp.g);
    const double dm = node_drho<T>(Rm.g0, Rm.g), dc = node_drho<T>(Rc.g0, Rc.g), dp = node_drho<T>(Rp.g0, Rp.g);
    const T psm = (A.walls && y == 0) ? (T)A.psi_lo : node_psi<T>(A, dm, L.valid);
    const T psc = node_psi<T>(A, dc, L.valid);
    const T psp = (A.walls && y == A.ny - 1) ? (T)A.psi_hi : node_psi<T>(A, dp, L.valid);
    Acc acc = {0.0, 0.0, 0.0};
    collide_row<T, MODE_STEP>(A, L, y, Rc, dc, psm, psc, psp, acc);
}

// Two steps of every lattice: workgroup w takes two-step tile w of the concatenated tile
// lists (lattice b owns tiles [tile_off[b], tile_off[b+1]), tile = strip + strips * band);
// the tile arithmetic is step2_tile of the single-lattice two-step kernel.
template <typename T, bool WALLS>
__global__ __launch_bounds__(64 * k2WavesOf<T>) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : LBM_K2_EU_F64)))
void k_batch_step2(const BatchItem* items, const int* tile_off, int B, char* buf0, char* buf1, int cur, long long step)
{
    __shared__ Step2Lds<T> S;
    const int w = blockIdx.x;
    if (w >= tile_off[B]) return;
    int lo = 0, hi = B;  // tile_off[lo] <= w < tile_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= w) lo = mid;
        else hi = mid;
    }
    StepArgs A = items[lo].A;
    const size_t off = items[lo].off_bytes;
    A.src = (cur ? buf1 : buf0) + off;
    A.dst = (cur ? buf0 : buf1) + off;
    A.step = step;
    const int tile = w - tile_off[lo];
    const int strips = (A.nx + k2Cols - 1) / k2Cols;
    step2_tile<T, MODE_STEP, WALLS>(A, tile % strips, tile / strips, S);
}

// Two steps of short periodic lattices (ny <= kFullRows, periodic in y): a workgroup of
// 64 * max(ny) threads owns a 58-column strip over ALL rows of its lattice, wave k row k.
// The rows wrap inside the workgroup, so unlike step2_tile there is no ring of rows; only
// the three-column ring in x is recomputed.  Same phases and node arithmetic as step2_tile.
constexpr int kFullRows = 16;

// The lattice's EOS record in LDS (read by node_psi), except for 16-row FP64 workgroups:
// their 80 KB of LDS leave no room for it beside a second workgroup per CU.
template <bool IN_LDS>
struct FullEos {
    DevEos eos;
    __device__ const DevEos& get(const StepArgs&) const { return eos; }
    __device__ void put(const StepArgs& A) { eos = A.eos; }
};
template <>
struct FullEos<false> {
    __device__ const DevEos& get(const StepArgs& A) const { return A.eos; }
    __device__ void put(const StepArgs&) {}
};

// LDS sized for ROWS rows (4, 8 or kFullRows, the smallest that holds max(ny)): shorter
// lattices fit more workgroups per CU (a 16-row FP32 workgroup takes 45 KB whatever its
// height, i.e. three per CU)
template <typename T, int ROWS>
struct FullLds : FullEos<sizeof(T) == 4 || ROWS < kFullRows> {
    T sps[ROWS][64];
    T smv[8][ROWS][64];
    double sg0[ROWS][64];
};

template <typename T, int ROWS, bool NT>
__global__ __launch_bounds__(64 * ROWS) void k_batch_full2(const BatchItem* items, const int* tile_off, int B,
                                                            char* buf0, char* buf1, int cur, long long step)
{
    __shared__ FullLds<T, ROWS> S;
    const int w = blockIdx.x;
    if (w >= tile_off[B]) return;
    int lo = 0, hi = B;  // tile_off[lo] <= w < tile_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= w) lo = mid;
        else hi = mid;
    }
    StepArgs A = items[lo].A;
    const size_t off = items[lo].off_bytes;
    A.src = (cur ? buf1 : buf0) + off;
    A.dst = (cur ? buf0 : buf1) + off;
    A.step = step;
    const int strip = w - tile_off[lo];
    const int k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const bool row = k < A.ny;  // waves beyond this lattice's rows only keep the barriers
    const int km = k == 0 ? A.ny - 1 : k - 1, kp = k + 1 == A.ny ? 0 : k + 1;
    const int x0 = strip * k2Cols, W = min(k2Cols, A.nx - x0);
    const int dl = l < 3 ? 3 - l : (l > W + 2 ? l - (W + 2) : 0);
    Lane L;
    L.lane = l;
    L.valid = dl <= 3;
    L.interior = dl == 0;
    // columns of lanes with dl <= 3 lie in [-3, nx + 2]: one wrap each way unless nx < 3
    int x = x0 - 3 + l;
    if (A.nx >= 3) x = x < 0 ? x + A.nx : (x >= A.nx ? x - A.nx : x);
    else x = (x % A.nx + A.nx) % A.nx;
    if (dl > 3) x = 0;
    L.x = x;
    L.xm = x == 0 ? A.nx - 1 : x - 1;
    L.xp = x == A.nx - 1 ? 0 : x + 1;
    Acc acc = {0.0, 0.0, 0.0};
    // 1. step t: pull, rho, psi (the EOS record goes to LDS while the pull is in flight,
    //    as in step2_tile)
    if (threadIdx.x == 0) S.put(A);
    Row<T> R;
    double dr = 0.0;
    T ps = (T)0;
    if (row && dl <= 3) {
        const View<T> V = make_view<T>(A.src, A.plane);
        pull<T>(V, A, L.x, L.xm, L.xp, k, R.g0, R.g);
    }
    __syncthreads();
    if (row && dl <= 3) {
        dr = node_drho<T>(R.g0, R.g);
        ps = node_psi<T>(A, S.get(A), dr, true);
    }
    S.sps[k][l] = ps;
    __syncthreads();
    // 2. step t: collide the strip grown by 2 columns into LDS
    if (row && dl <= 2) {
        T Ftx, Fty;
        force_tilde<T>(A, S.sps[km][l - 1], S.sps[km][l], S.sps[km][l + 1], S.sps[k][l - 1], S.sps[k][l + 1],
                       S.sps[kp][l - 1], S.sps[kp][l], S.sps[kp][l + 1], Ftx, Fty);
        T o[9];
        double o0;
        node_collide<T, MODE_STEP>(A, L, k, R, dr, ps, Ftx, Fty, acc, o, o0);
#pragma unroll
        for (int i = 1; i < 9; ++i) S.smv[i - 1][k][l] = o[i];
        S.sg0[k][l] = o0;
    }
    __syncthreads();
    // 3. step t+1: pull from LDS (rows wrap), psi(t+1)
    if (row && dl <= 1) {
        R.g0 = S.sg0[k][l];
        R.g[1] = S.smv[0][k][l - 1];
        R.g[3] = S.smv[2][k][l + 1];
        R.g[2] = S.smv[1][km][l];
        R.g[5] = S.smv[4][km][l - 1];
        R.g[6] = S.smv[5][km][l + 1];
        R.g[4] = S.smv[3][kp][l];
        R.g[7] = S.smv[6][kp][l + 1];
        R.g[8] = S.smv[7][kp][l - 1];
        dr = node_drho<T>(R.g0, R.g);
        ps = node_psi<T>(A, S.get(A), dr, true, 1);
        S.sps[k][l] = ps;
    }
    __syncthreads();
    // 4. step t+1: collide the strip and store
    if (row && dl == 0) {
        T Ftx, Fty;
        force_tilde<T>(A, S.sps[km][l - 1], S.sps[km][l], S.sps[km][l + 1], S.sps[k][l - 1], S.sps[k][l + 1],
                       S.sps[kp][l - 1], S.sps[kp][l], S.sps[kp][l + 1], Ftx, Fty);
        update_node<T, MODE_STEP, NT>(A, L, k, R, dr, ps, Ftx, Fty, acc);
    }
}

template <typename T, bool NT>
void launch_full2_t(int max_ny, dim3 g, dim3 b, hipStream_t s, const BatchItem* it, const int* off, int B, char* b0,
                    char* b1, int cur, long long st)
{
    if (max_ny <= 4) hipLaunchKernelGGL((k_batch_full2<T, 4, NT>), g, b, 0, s, it, off, B, b0, b1, cur, st);
    else if (max_ny <= 8) hipLaunchKernelGGL((k_batch_full2<T, 8, NT>), g, b, 0, s, it, off, B, b0, b1, cur, st);
    else hipLaunchKernelGGL((k_batch_full2<T, kFullRows, NT>), g, b, 0, s, it, off, B, b0, b1, cur, st);
}

// nt: streaming stores, when both population buffers of the batch are small (kStreamBytes)
// (as for a single lattice)
void launch_full2(bool f32, bool nt, int max_ny, dim3 g, dim3 b, hipStream_t s, const BatchItem* it, const int* off,
                  int B, char* b0, char* b1, int cur, long long st)
{
    if (f32 && nt) launch_full2_t<float, true>(max_ny, g, b, s, it, off, B, b0, b1, cur, st);
    else if (f32) launch_full2_t<float, false>(max_ny, g, b, s, it, off, B, b0, b1, cur, st);
    else if (nt) launch_full2_t<double, true>(max_ny, g, b, s, it, off, B, b0, b1, cur, st);
    else launch_full2_t<double, false>(max_ny, g, b, s, it, off, B, b0, b1, cur, st);
}

template <typename T>
__global__ void k_batch_init(const BatchItem* items, char* buf0, const double* rho0, const double* ux0,
                             const double* uy0)
{
    const StepArgs& A = items[blockIdx.y].A;
    const size_t off = items[blockIdx.y].off_bytes;
    const long long coff = items[blockIdx.y].cell_off;
    const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    void* dst = buf0 + off;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < A.nx * A.ny; c += gridDim.x * blockDim.x) {
        const int x = c % A.nx, y = c / A.nx;
        const size_t o = (size_t)y * A.ld + x;
        for (int j = 0; j < 9; ++j) {
            // A_j(z) such that the first pull yields f^eq(rho0, u0)
            int sx = x + cx[j], sy = y + cy[j], k = j;
            if (A.walls && (sy < 0 || sy >= A.ny)) {
                sx = x;
                sy = y;
                k = op[j];
            }
            sx = sx < 0 ? sx + A.nx : (sx >= A.nx ? sx - A.nx : sx);
            sy = sy < 0 ? sy + A.ny : (sy >= A.ny ? sy - A.ny : sy);
            const long long s = coff + (long long)sy * A.nx + sx;
            const double g = init_population<T>(k, rho0[s], ux0 ? ux0[s] : 0.0, uy0 ? uy0[s] : 0.0, A.rho_ref);
            if (j == 0) Plane<T>::restw(dst, A.plane)[o] = g;
            else Plane<T>::movw(dst, A.plane, j)[o] = (T)g;
        }
    }
}

bool hip_ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    lbm_set_error(buf);
    return false;
}

struct Layout {
    std::vector<size_t> off;        // [B+1] byte offsets in a population buffer
    std::vector<long long> cells;   // [B+1] cell offsets in the packed fields
    std::vector<int> ld;
    std::vector<int> item_off;      // [B+1] one-step grouped items (strips x rows) before each lattice
    std::vector<int> tile_off;      // [B+1] two-step grouped tiles before each lattice
    std::vector<int> strip_off;     // [B+1] two-step full-height strips before each lattice
    int any_walls, max_ny;
    size_t off_items, off_item_off, off_tile_off, off_strip_off, ws_bytes;
};

int batch_layout(int B, const lbm_params* p, Layout& L)
{
    if (B < 1 || !p) {
        lbm_set_error("lbm batched: need at least one lattice");
        return LBM_EINVAL;
    }
    L.off.assign(B + 1, 0);
    L.cells.assign(B + 1, 0);
    L.ld.assign(B, 0);
    L.item_off.assign(B + 1, 0);
    L.tile_off.assign(B + 1, 0);
    L.strip_off.assign(B + 1, 0);
    L.any_walls = 0;
    L.max_ny = 0;
    for (int b = 0; b < B; ++b) {
        if (p[b].prec != p[0].prec) {
            lbm_set_error("lbm batched: every lattice must use the same storage precision");
            return LBM_EINVAL;
        }
        const int st = validate(&p[b]);
        if (st != LBM_OK) return st;
        if (p[b].kernel_variant == LBM_VARIANT_AA) {
            lbm_set_error("lbm batched: the in-place AA variant runs single lattices only");
            return LBM_EINVAL;
        }
        const int ld = (p[b].nx + 63) & ~63;
        const size_t plane = (size_t)ld * p[b].ny;
        const size_t bytes = p[b].prec == LBM_FP32_SHIFTED ? plane * (8 * sizeof(float) + sizeof(double))
                                                           : plane * 9 * sizeof(double);
        L.ld[b] = ld;
        L.off[b + 1] = L.off[b] + ((bytes + 255) & ~(size_t)255);
        L.cells[b + 1] = L.cells[b] + (long long)p[b].nx * p[b].ny;
        const long long items = (long long)((p[b].nx + kStripW - 1) / kStripW) * p[b].ny;
        if (L.item_off[b] + items >= (1LL << 31)) {
            lbm_set_error("lbm batched: too many rows x strips in one batch");
            return LBM_EINVAL;
        }
        L.item_off[b + 1] = L.item_off[b] + (int)items;
        const int rows2 = k2waves_of_prec(p[0].prec) - 6;
        L.tile_off[b + 1] = L.tile_off[b] + ((p[b].nx + k2Cols - 1) / k2Cols) * ((p[b].ny + rows2 - 1) / rows2);
        L.strip_off[b + 1] = L.strip_off[b] + (p[b].nx + k2Cols - 1) / k2Cols;
        L.any_walls |= p[b].walls != 0;
        L.max_ny = p[b].ny > L.max_ny ? p[b].ny : L.max_ny;
    }
    // workspace: per-lattice error words, the item records, the grouped-step item offsets
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    L.off_items = al((size_t)B * 2 * sizeof(unsigned));
    L.off_item_off = L.off_items + al((size_t)B * sizeof(BatchItem));
    L.off_tile_off = L.off_item_off + al((size_t)(B + 1) * sizeof(int));
    L.off_strip_off = L.off_tile_off + al((size_t)(B + 1) * sizeof(int));
    L.ws_bytes = L.off_strip_off + al((size_t)(B + 1) * sizeof(int));
    return LBM_OK;
}

}  // namespace

struct lbm_batch {
    int B;
    int prec;
    Layout L;
    char* buf[2];
    int cur;
    int64_t step;
    unsigned* err;
    BatchItem* items;
    int* item_off;          // device copies of Layout::item_off and Layout::tile_off
    int* tile_off;
    int* strip_off;         // device copy of Layout::strip_off (full-height strips)
    int full;               // 1: every lattice is periodic with ny <= kFullRows (full-height two-step)
    int grouped;            // 1: one grouped launch per step; 0: persistent workgroups
    hipStream_t cap;        // capture stream (default priority)
    hipGraphExec_t exec[2]; // per starting buffer: the persistent launch of `graph_steps` steps, or
                            // kGroupChunk two-step grouped launches
    int64_t graph_steps;
};

namespace {
constexpr int kGroupChunk = 64;  // two-step grouped launches per replayed graph (128 steps)

// persistent unless some lattice gives one workgroup more than two items per wave and step
int auto_grouped(const Layout& L, int B)
{
    for (int b = 0; b < B; ++b)
        if (L.item_off[b + 1] - L.item_off[b] > 2 * kBatchWaves) return 1;
    return 0;
}
}  // namespace

extern "C" {

int lbm_batch_layout(int B, const lbm_params* p, size_t* pop_bytes_out, size_t* ws_bytes_out, int64_t* cell_offsets)
{
    Layout L;
    const int st = batch_layout(B, p, L);
    if (st != LBM_OK) return st;
    if (pop_bytes_out) *pop_bytes_out = L.off[B];
    if (ws_bytes_out) *ws_bytes_out = L.ws_bytes;
    if (cell_offsets)
        for (int b = 0; b <= B; ++b) cell_offsets[b] = L.cells[b];
    return LBM_OK;
}

int lbm_init_batched(lbm_batch** out, int B, const lbm_params* p, void* f_a, void* f_b, void* ws, size_t ws_bytes,
                     const double* rho0, const double* ux0, const double* uy0, void* stream)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    Layout L;
    int st = batch_layout(B, p, L);
    if (st != LBM_OK) return st;
    if (!f_a || !f_b || f_a == f_b || !ws || !rho0 || ws_bytes < L.ws_bytes) {
        lbm_set_error("lbm_init_batched: buffers must be non-NULL and distinct, workspace as lbm_batch_layout says");
        return LBM_EINVAL;
    }
    lbm_batch* c = new (std::nothrow) lbm_batch();
    if (!c) return LBM_EINVAL;
    c->B = B;
    c->prec = p[0].prec;
    c->L = L;
    c->buf[0] = (char*)f_a;
    c->buf[1] = (char*)f_b;
    c->err = (unsigned*)ws;
    c->items = (BatchItem*)((char*)ws + L.off_items);
    c->item_off = (int*)((char*)ws + L.off_item_off);
    c->tile_off = (int*)((char*)ws + L.off_tile_off);
    c->strip_off = (int*)((char*)ws + L.off_strip_off);
    c->full = !L.any_walls && L.max_ny <= kFullRows;
    c->grouped = auto_grouped(L, B);
    std::vector<BatchItem> host(B);
    std::vector<unsigned> err0(2 * (size_t)B);
    for (int b = 0; b < B; ++b) {
        const lbm_params& P = p[b];
        StepArgs& A = host[b].A;
        std::memset(&A, 0, sizeof(A));
        A.plane = (size_t)L.ld[b] * P.ny;
        A.nx = P.nx;
        A.ny = P.ny;
        A.ld = L.ld[b];
        A.walls = P.walls;
        A.strips = (P.nx + kStripW - 1) / kStripW;
        A.seg_h = 1;
        A.nseg = P.ny;
        A.nwork = A.strips * P.ny;
        A.var_tau = P.var_tau;
        A.G = P.G;
        A.sigma = P.sigma;
        for (int k = 0; k < 9; ++k) A.s[k] = 1.0 / P.tau[k];
        fill_coef(A, P.tau, P.G, P.sigma);
        A.tau_v = P.tau_v;
        A.rho_v_tau = P.rho_v_tau;
        A.dtau_drho = P.var_tau ? (P.tau_l - P.tau_v) / (P.rho_l_tau - P.rho_v_tau) : 0.0;
        A.tau_lo = P.tau_l < P.tau_v ? P.tau_l : P.tau_v;
        A.tau_hi = P.tau_l < P.tau_v ? P.tau_v : P.tau_l;
        A.rho_ref = P.prec == LBM_FP32_SHIFTED ? P.rho_ref : 0.0;
        A.eos = dev_eos(P.eos);
        auto psi_host = [&](double r) {
            const double q = 2.0 * (lbm_eos_pressure(&P.eos, r) - r / 3.0) / P.G;
            return q > 0 ? std::sqrt(q) : 0.0;
        };
        A.psi_lo = P.walls ? psi_host(P.rho_wall_lo) : 0.0;
        A.psi_hi = P.walls ? psi_host(P.rho_wall_hi) : 0.0;
        A.err = c->err + 2 * b;
        host[b].off_bytes = L.off[b];
        host[b].cell_off = L.cells[b];
        err0[2 * b] = 0u;
        err0[2 * b + 1] = 0xffffffffu;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMemcpyAsync(c->items, host.data(), sizeof(BatchItem) * B, hipMemcpyHostToDevice, s), "batch items") ||
        !hip_ok(hipMemcpyAsync(c->item_off, L.item_off.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, s),
                "batch item offsets") ||
        !hip_ok(hipMemcpyAsync(c->tile_off, L.tile_off.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, s),
                "batch tile offsets") ||
        !hip_ok(hipMemcpyAsync(c->strip_off, L.strip_off.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, s),
                "batch strip offsets") ||
        !hip_ok(hipMemcpyAsync(c->err, err0.data(), sizeof(unsigned) * 2 * B, hipMemcpyHostToDevice, s), "batch errors") ||
        !hip_ok(hipStreamSynchronize(s), "batch init sync")) {
        delete c;
        return LBM_EHIP;
    }
    if (c->prec == LBM_FP32_SHIFTED)
        hipLaunchKernelGGL(k_batch_init<float>, dim3(64, B), dim3(256), 0, s, (const BatchItem*)c->items, c->buf[0], rho0,
                           ux0, uy0);
    else
        hipLaunchKernelGGL(k_batch_init<double>, dim3(64, B), dim3(256), 0, s, (const BatchItem*)c->items, c->buf[0], rho0,
                           ux0, uy0);
    if (!hip_ok(hipGetLastError(), "k_batch_init launch") ||
        !hip_ok(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "capture stream")) {
        delete c;
        return LBM_EHIP;
    }
    *out = c;
    return LBM_OK;
}

// n grouped steps starting from buffer cur at step step0: n / 2 two-step launches, then
// one one-step launch if n is odd
static bool launch_grouped(lbm_batch* c, int n, int cur, int64_t step0, hipStream_t s)
{
    const BatchItem* it = c->items;
    const bool f32 = c->prec == LBM_FP32_SHIFTED, w = c->L.any_walls != 0;
    const dim3 g2(c->L.tile_off[c->B]), b2(64 * k2waves_of_prec(c->prec));
    int k = 0;
    const dim3 gf(c->L.strip_off[c->B]), bf(64 * c->L.max_ny);
    for (; k + 1 < n; k += 2) {
        const long long st = (long long)(step0 + k);
        if (c->full)
            launch_full2(f32, 2 * c->L.off[c->B] <= kStreamBytes, c->L.max_ny, gf, bf, s, it, c->strip_off, c->B,
                         c->buf[0], c->buf[1], cur, st);
        else if (f32 && !w) hipLaunchKernelGGL((k_batch_step2<float, false>), g2, b2, 0, s, it, c->tile_off, c->B, c->buf[0], c->buf[1], cur, st);
        else if (f32) hipLaunchKernelGGL((k_batch_step2<float, true>), g2, b2, 0, s, it, c->tile_off, c->B, c->buf[0], c->buf[1], cur, st);
        else if (!w) hipLaunchKernelGGL((k_batch_step2<double, false>), g2, b2, 0, s, it, c->tile_off, c->B, c->buf[0], c->buf[1], cur, st);
        else hipLaunchKernelGGL((k_batch_step2<double, true>), g2, b2, 0, s, it, c->tile_off, c->B, c->buf[0], c->buf[1], cur, st);
        cur ^= 1;  // two steps land in the other buffer
    }
    if (k < n) {
        const dim3 g((c->L.item_off[c->B] + 3) / 4), b(256);
        if (f32)
            hipLaunchKernelGGL(k_batch_step<float>, g, b, 0, s, it, (const int*)c->item_off, c->B, c->buf[0], c->buf[1],
                               cur, (long long)(step0 + k));
        else
            hipLaunchKernelGGL(k_batch_step<double>, g, b, 0, s, it, (const int*)c->item_off, c->B, c->buf[0], c->buf[1],
                               cur, (long long)(step0 + k));
    }
    return hip_ok(hipGetLastError(), "grouped batch launch");
}

static bool launch_batch(lbm_batch* c, int64_t nsteps, hipStream_t s)
{
    if (c->prec == LBM_FP32_SHIFTED)
        hipLaunchKernelGGL((k_batch<float, MODE_STEP>), dim3(c->B), dim3(64 * kBatchWaves), 0, s,
                           (const BatchItem*)c->items, c->buf[0], c->buf[1], c->cur, (long long)nsteps, (long long)c->step,
                           (double*)nullptr, (double*)nullptr, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_batch<double, MODE_STEP>), dim3(c->B), dim3(64 * kBatchWaves), 0, s,
                           (const BatchItem*)c->items, c->buf[0], c->buf[1], c->cur, (long long)nsteps, (long long)c->step,
                           (double*)nullptr, (double*)nullptr, (double*)nullptr);
    return hip_ok(hipGetLastError(), "k_batch launch");
}

int lbm_set_batch_mode(lbm_batch* c, int mode)
{
    if (!c || mode < LBM_BATCH_AUTO || mode > LBM_BATCH_GROUPED) return LBM_EINVAL;
    const int g = mode == LBM_BATCH_AUTO ? auto_grouped(c->L, c->B) : (mode == LBM_BATCH_GROUPED);
    if (g != c->grouped) {
        for (int k = 0; k < 2; ++k)
            if (c->exec[k]) {
                (void)hipGraphExecDestroy(c->exec[k]);
                c->exec[k] = nullptr;
            }
        c->graph_steps = 0;
        c->grouped = g;
    }
    return LBM_OK;
}

// grouped mode: graphs of kGroupChunk launches (one per starting buffer), the rest launched directly.
// A graph bakes in the step numbers of its capture; they only label the error word's first
// failing step, which is therefore exact for the first chunk of each parity and approximate after.
static int step_grouped(lbm_batch* c, int64_t nsteps, hipStream_t s)
{
    const int chunk = 2 * kGroupChunk;  // steps per replayed graph; a two-step launch flips the buffer,
                                        // so an even number of launches keeps the parity
    int64_t done = 0;
    while (nsteps - done >= chunk) {
        if (!c->exec[c->cur]) {
            hipGraph_t g = nullptr;
            if (!hip_ok(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "batch capture begin"))
                return LBM_EHIP;
            const bool ok = launch_grouped(c, chunk, c->cur, c->step, c->cap);
            if (!hip_ok(hipStreamEndCapture(c->cap, &g), "batch capture end") || !ok) return LBM_EHIP;
            const bool inst =
                hip_ok(hipGraphInstantiate(&c->exec[c->cur], g, nullptr, nullptr, 0), "batch graph instantiate");
            (void)hipGraphDestroy(g);
            if (!inst) return LBM_EHIP;
        }
        if (!hip_ok(hipGraphLaunch(c->exec[c->cur], s), "batch graph launch")) return LBM_EHIP;
        c->step += chunk;
        done += chunk;
    }
    const int rest = (int)(nsteps - done);
    if (rest > 0) {
        if (!launch_grouped(c, rest, c->cur, c->step, s)) return LBM_EHIP;
        c->step += rest;
        // each two-step launch and the one-step launch flip the buffer once
        if (((rest / 2) + (rest & 1)) & 1) c->cur ^= 1;
    }
    return LBM_OK;
}

int lbm_step_batched(lbm_batch* c, int64_t nsteps, void* stream)
{
    if (!c || nsteps < 0) return LBM_EINVAL;
    if (nsteps == 0) return LBM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (c->grouped) return step_grouped(c, nsteps, s);
    // the persistent launch is captured once per (step count, starting buffer) and replayed
    if (c->graph_steps != nsteps) {
        for (int k = 0; k < 2; ++k)
            if (c->exec[k]) {
                (void)hipGraphExecDestroy(c->exec[k]);
                c->exec[k] = nullptr;
            }
        c->graph_steps = nsteps;
    }
    if (!c->exec[c->cur]) {
        hipGraph_t g = nullptr;
        if (!hip_ok(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "batch capture begin")) return LBM_EHIP;
        const bool ok = launch_batch(c, nsteps, c->cap);
        if (!hip_ok(hipStreamEndCapture(c->cap, &g), "batch capture end") || !ok) return LBM_EHIP;
        const bool inst = hip_ok(hipGraphInstantiate(&c->exec[c->cur], g, nullptr, nullptr, 0), "batch graph instantiate");
        (void)hipGraphDestroy(g);
        if (!inst) return LBM_EHIP;
    }
    if (!hip_ok(hipGraphLaunch(c->exec[c->cur], s), "batch graph launch")) return LBM_EHIP;
    c->step += nsteps;
    if (nsteps & 1) c->cur ^= 1;
    return LBM_OK;
}

int lbm_macros_batched(lbm_batch* c, double* rho, double* ux, double* uy, void* stream)
{
    if (!c) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (c->prec == LBM_FP32_SHIFTED)
        hipLaunchKernelGGL((k_batch<float, MODE_MACROS>), dim3(c->B), dim3(64 * kBatchWaves), 0, s,
                           (const BatchItem*)c->items, c->buf[0], c->buf[1], c->cur, 1LL, (long long)c->step, rho, ux, uy);
    else
        hipLaunchKernelGGL((k_batch<double, MODE_MACROS>), dim3(c->B), dim3(64 * kBatchWaves), 0, s,
                           (const BatchItem*)c->items, c->buf[0], c->buf[1], c->cur, 1LL, (long long)c->step, rho, ux, uy);
    if (!hip_ok(hipGetLastError(), "k_batch(macros) launch") || !hip_ok(hipStreamSynchronize(s), "batch macros sync"))
        return LBM_EHIP;
    return LBM_OK;
}

int lbm_status_batched(lbm_batch* c, int* first_bad_out, void* stream)
{
    if (!c) return LBM_EINVAL;
    std::vector<unsigned> h(2 * (size_t)c->B);
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMemcpyAsync(h.data(), c->err, sizeof(unsigned) * h.size(), hipMemcpyDeviceToHost, s), "batch status") ||
        !hip_ok(hipStreamSynchronize(s), "batch status sync"))
        return LBM_EHIP;
    if (first_bad_out) *first_bad_out = -1;
    for (int b = 0; b < c->B; ++b)
        if (h[2 * b]) {
            if (first_bad_out) *first_bad_out = b;
            char buf[160];
            std::snprintf(buf, sizeof(buf), "lbm batched: lattice %d unstable from step %u", b, h[2 * b + 1]);
            lbm_set_error(buf);
            return LBM_EUNSTABLE;
        }
    return LBM_OK;
}

void lbm_destroy_batched(lbm_batch* c)
{
    if (!c) return;
    for (int k = 0; k < 2; ++k)
        if (c->exec[k]) (void)hipGraphExecDestroy(c->exec[k]);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

}  // extern "C"
