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
int resolve_variant(const lbm_params& p);
}  // namespace lbmk
