// Host context of liblbm.so (internal).
#pragma once

#include "lbm_device.h"

struct lbm_ctx {
    lbm_params P;
    lbmk::StepArgs args;
    int ld;
    size_t plane, pop_bytes;
    void* buf[2];
    int cur;
    int64_t step;
    char* ws;
    size_t ws_bytes;
    unsigned* err;
    double* partials;
    double* redblk;
    double* hist;
    double* red;
    int64_t hist_count;
    int grid;
    int blk2, grid2;  // LBM_VARIANT_BLOCK2: two-step launches and their grid
    bool rows2;       // two-step tiles with two rows per wave (k_step2_rows2)
    lbmk::TwoStepShape shape;  // the two-step tile it runs (lbm_params.tile_rows; timed for -1)
    // checkpoints for the adjoint: the state f*(t) at every t = K*slot
    void* ckpt;
    int64_t ckpt_slots;
    int ckpt_K;
    // forward record for the adjoint (lbm_set_recording): every step from 0 on
    void* rec_all;
    int64_t rec_steps;
    // the per-device context of lbm_init_static (lbm_destroy leaves it alone)
    bool is_static;
    // LBM_VARIANT_AA: one population buffer updated in place (buf[0] == buf[1]) and the psi
    // plane of the workspace
    bool aa;
    void* aa_psi;
};


namespace lbmk {
bool hip_ok(hipError_t e, const char* what);
bool launch_reduce(lbm_ctx* c, double* out, long long step, int with_step, hipStream_t s);
bool launch_reduce_n(lbm_ctx* c, int n, double* out, long long step, int with_step, hipStream_t s);
bool launch_record_step(lbm_ctx* c, void* rec, hipStream_t s);
// two recorded steps in one launch (two-step variant only): records of steps t and t+1 in
// consecutive slots from rec
bool launch_record_pair(lbm_ctx* c, void* rec, hipStream_t s);
int decompose(const lbm_params& p, int* strips, int* seg_h, int* nseg, int* blk);
// LBM_VARIANT_AA (lbm_aa.hip): partial-sum slots of a reducing step, bytes of the psi plane,
// one step of c->step's parity in place (MODE_STEP or MODE_STEP_REDUCE), the macroscopic
// fields (out: rho, ux, uy, psi, p, Fx, Fy, any NULL) and the FP64 populations
int aa_slots(const lbm_params& p);
size_t aa_psi_bytes(const lbm_params& p, int ld);
bool aa_init(lbm_ctx* c, const double* rho0, const double* ux0, const double* uy0, hipStream_t s);
bool aa_step(lbm_ctx* c, int mode, hipStream_t s);
bool aa_macros(lbm_ctx* c, double* const out[7], hipStream_t s);
bool aa_populations(lbm_ctx* c, double* f_out, hipStream_t s);
int resolve_variant(const lbm_params& p);
}  // namespace lbmk
