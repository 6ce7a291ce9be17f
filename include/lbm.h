/*
 * lbm.h -- C ABI of the MI355X (gfx950) shaped-EOS pseudopotential lattice
 * Boltzmann library (liblbm.so).
 *
 * Method: Czelusniak, Mapelli, Cabezas Gomez, Wagner, "Shaping the equation
 * of state to improve numerical accuracy and stability of the
 * pseudopotential lattice Boltzmann method".  One time step is Eq. LBE with
 * the MRT operator (Eq. OperatorMRT, Eq. MatrixMRT, Eq. RelaxationMatrix),
 * the equilibrium of Eq. EquilibriumDistribution, the Shan-Chen force
 * (Eq. ShanChenForce) on the pseudopotential of Eq. InteractionPotential
 * with a shaped EOS (Sec. III.D "Smooth", Eq. PengEOS), and the forcing of
 * Eq. LiFS (Eq. GFS at sigma = 0).
 *
 * Conventions common to every entry point
 *  - Device pointers are CALLER-OWNED (typically torch tensors).  The library
 *    never allocates or frees device memory; it keeps a small host context.
 *  - Layouts.  Scalar fields are [ny][nx] row-major float64 (x fastest).
 *    Population buffers are planes of [ny][ld] (ld = row pitch >= nx, chosen
 *    by lbm_layout): for LBM_FP64, 9 float64 planes in the D2Q9 order of
 *    Eq. VelocitySet; for LBM_FP32_SHIFTED, planes 1..8 hold float32
 *    g_i = f_i - w_i rho_ref and a final float64 plane holds g_0 (the rest
 *    population, kept in FP64 so that each node's mass is exact).
 *  - The population buffers hold POST-collision values (pull streaming):
 *    the distributions of Eq. LBE at time t are obtained by pulling from
 *    the neighbours, with half-way bounce-back at walls.
 *  - `stream` is a hipStream_t passed as void*; 0 means the null stream.
 *    Calls are asynchronous unless stated.
 *  - Return value: 0 (LBM_OK) or a negative lbm_status; lbm_last_error()
 *    returns a thread-local message for the last failure.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility: exactly the declarations of
 * this header are its exported interface. */
#pragma GCC visibility push(default)

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument or parameter combination */
    LBM_EUNSTABLE = -2, /* psi^2 < 0, non-finite or non-positive density met on the device */
    LBM_EHIP = -3,      /* a HIP runtime call failed */
    LBM_ESTATE = -4,    /* call out of order (e.g. adjoint without checkpointing) */
    LBM_ENOROOT = -5    /* host thermodynamics: no root in the admissible bracket */
} lbm_status;

typedef enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 } lbm_prec;
/* Step-kernel decompositions (identical node arithmetic; results agree up to
 * the compiler's FMA contraction choices):
 * MARCH: one wavefront marches up a band of rows of a 62-column strip with
 * two rows of loads in flight; BLOCK: a 12-wavefront workgroup loads 12 rows
 * of a strip, one per wavefront, and shares psi through LDS; BLOCK2: a
 * workgroup advances a tile 58 columns wide by two time steps per launch and
 * keeps the intermediate populations in LDS (temporal blocking; a reducing
 * step ends a launch, and checkpoint boundaries and odd counts run single
 * steps on BLOCK).  The tile: FP64, 8 wavefronts of two rows each, 10 rows;
 * FP32, 16 wavefronts of one row, 10 rows, or on lattices of at least 4096
 * such tiles 12 wavefronts of two rows, 18 rows.  AUTO is BLOCK2.
 * AA: one population buffer updated in place with the AA access pattern
 * (even steps read and write each node's own slots, odd steps read from and
 * write to the neighbours, bounce-back included), for lattices whose second
 * buffer would not fit.  psi of the neighbours cannot be formed in the same
 * pass, so each step is two launches (psi of every node into a workspace
 * plane, then the update): about 1.6x the HBM traffic of the pull variants.
 * No adjoint (recording and checkpointing refuse it) and no batched use. */
typedef enum {
    LBM_VARIANT_AUTO = 0,
    LBM_VARIANT_MARCH = 1,
    LBM_VARIANT_BLOCK = 2,
    LBM_VARIANT_BLOCK2 = 3,
    LBM_VARIANT_AA = 4
} lbm_variant;
typedef enum { LBM_BASE_CS = 0, LBM_BASE_PR = 1 } lbm_base;
typedef enum {
    LBM_SHAPE_NONE = 0,      /* the base EOS itself */
    LBM_SHAPE_SMOOTH = 1,    /* Sec. III.D: ellipse / cubic / ellipse, p_max from Eq. MaxwellRule */
    LBM_SHAPE_MODSMOOTH = 2, /* Sec. IV.C: same loop, p_max from Eq. ShanVaporLiqEq (eps = 0) */
    LBM_SHAPE_PENG = 3       /* Eq. PengEOS with Eq. PengTheta, rho_m from Eq. ShanVaporLiqEq */
} lbm_shape;

/*
 * Equation of state.  Inputs are set by the caller; lbm_eos_build fills the
 * derived block (FP64, host only).  Base EOS: Carnahan-Starling (Eq. CS) or
 * the textbook Peng-Robinson form, times `scale` (the "standard procedure"
 * of Sec. III.B).  The shaped loop replaces the base EOS on (rho_v, rho_l);
 * the vapor branch is k_vap times the base EOS and the liquid branch is the
 * base EOS plus dP_liq = (k_vap - 1) p_sat (raised vapor sound speed,
 * Sec. III.D); p_min = p_sat_new - alpha (p_sat - p_min_base).
 */
typedef struct {
    /* inputs */
    int base, shape;
    double a, b, R, omega, Tr, scale, alpha, k_vap, r_theta;
    /* derived by lbm_eos_build */
    double Tc, T;
    double rho_v, rho_l, p_sat;       /* Maxwell coexistence of the scaled base EOS */
    double rho_max, p_max_base;       /* local maximum (spinodal) of the base EOS */
    double rho_min, p_min_base;       /* local minimum (spinodal) of the base EOS */
    double p_sat_new, dP_liq;
    double slope_v, slope_l;          /* dp/drho of the shaped EOS at rho_v, rho_l */
    double p_max, p_min;              /* interior knots (rho_max, p_max), (rho_min, p_min) */
    double a1sq, b1, a3sq, b3;        /* ellipse coefficients of regions 1 and 3 */
    double rho_m, theta;              /* Peng loop */
    double eps;                       /* root of Eq. VaporLiqEq (0 for the Guo-forcing shapes) */
} lbm_eos;

/* Host precompute (Sec. III.A, III.D, IV.C): critical point, Maxwell
 * coexistence, spinodals, shaped-loop coefficients, eps and
 * sigma = -eps/(16 G).  G must be negative.  Returns LBM_EINVAL for bad
 * inputs or a non-real ellipse, LBM_ENOROOT when a root is not bracketed. */
int lbm_eos_build(lbm_eos* e, double G, double* sigma_out);
/* Host evaluation of the built EOS p(rho) and dp/drho (FP64). */
double lbm_eos_pressure(const lbm_eos* e, double rho);
double lbm_eos_slope(const lbm_eos* e, double rho);

typedef struct {
    int nx, ny;          /* lattice size (nx, ny >= 1) */
    int walls;           /* 0: periodic in y; 1: half-way bounce-back below row 0 and above row ny-1 */
    int prec;            /* lbm_prec */
    int var_tau;         /* 1: s[7] = s[8] = 1/tau(rho) of Eq. RelaxationTime (clamped to [tau_v, tau_l]) */
    int reduce_every;    /* >0: FP64 mass/momentum reduction every this many steps (history in workspace) */
    int band_rows;       /* row-march kernel: rows per wavefront band (0 = automatic) */
    int kernel_variant;  /* lbm_variant: step-kernel decomposition (0 = automatic) */
    double rho_wall_lo, rho_wall_hi; /* densities of the solid nodes in Eq. ShanChenForce (walls = 1) */
    double G, sigma;     /* interaction constant (< 0) and Eq. LiFS sigma (0 = Eq. GFS) */
    double tau[9];       /* relaxation times, moment order of Eq. RelaxationMatrix; tau > 1/2 */
    double tau_l, tau_v, rho_v_tau, rho_l_tau; /* Eq. RelaxationTime */
    double rho_ref;      /* shift of the FP32 storage (LBM_FP32_SHIFTED), > 0 */
    lbm_eos eos;         /* built by lbm_eos_build */
    int tile_rows;       /* LBM_VARIANT_BLOCK2 tile height: 0 = the library's choice (below);
                          * -1 = the fastest candidate, timed on the device by lbm_init
                          * (FP32: one-row tiles and two-row heights 14..18; FP64: 7..10);
                          * > 0 = that height (FP32: 10 = one row per wavefront, 11..18 =
                          * two rows; FP64: 5..10).  Populations do not depend on it beyond
                          * the compiler's FMA contraction between the one- and two-row
                          * kernels; the order of the FP64 reduction partials does. */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Layout query: row pitch, bytes of ONE population buffer (the caller
 * allocates two; one for LBM_VARIANT_AA), and bytes of the workspace.  LBM_EINVAL when a population
 * plane (64-aligned row pitch x ny x 8 bytes) would reach 4 GiB: offsets
 * inside a plane are 32-bit (the largest square lattice is 23168^2). */
int lbm_layout(const lbm_params* p, int* ld_out, size_t* pop_bytes_out, size_t* ws_bytes_out);

/* Which step-kernel decomposition the parameters select (the automatic
 * choice resolved), the rows per band or block, and the wavefront count; for
 * BLOCK2 the output rows of a two-step tile and the wavefronts of its
 * workgroup (rows + 6 = wavefronts x rows per wavefront; two rows per
 * wavefront when rows + 6 < 2 x wavefronts + 1, i.e. rows > wavefronts - 6).
 * With tile_rows = -1 this is the shape before lbm_init times the candidates:
 * lbm_tile_shape reports the one a context runs.  LBM_VARIANT_AA: 4 rows and
 * 4 wavefronts per workgroup. */
int lbm_describe(const lbm_params* p, int* variant_out, int* band_rows_out, int* waves_out);

/* Create a context over caller buffers f_a, f_b (lbm_layout bytes each) and
 * workspace ws, and write the initial state f_i(0) = f^eq_i(rho0, u0)
 * (Sec. III.A) into f_a; in LBM_FP32_SHIFTED the FP64 rest population takes
 * what the eight FP32-rounded moving populations leave of rho0, so that each
 * node's mass is rho0 exactly.  rho0, ux0, uy0: device float64 [ny][nx]; ux0/uy0
 * may be NULL (u = 0).  Validates parameters (LBM_EINVAL): tau > 1/2,
 * rho_ref > 0 in FP32 mode, G < 0, buffers non-NULL and distinct
 * (LBM_VARIANT_AA: f_a only, f_b NULL; it holds f^eq(rho0, u0) at each node
 * itself, where the other variants store it one node upstream for their
 * first pull). */
int lbm_init(lbm_ctx** ctx, const lbm_params* p, void* f_a, void* f_b, void* ws, size_t ws_bytes,
             const double* rho0, const double* ux0, const double* uy0, void* stream);

/* lbm_init for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the workspace is the
 * library's own static array of 16 MiB per GPU instead of a caller buffer,
 * and the context is the library's one static context for the current
 * device.  Allocates nothing, host or device; the caller still passes f_a,
 * f_b and the initial fields, and lbm_step, lbm_macros and the rest take the
 * returned context as usual.  Each call re-initialises the device's context
 * (a later call on the same device ends the earlier one; lbm_destroy on it
 * does nothing).  LBM_EINVAL when the lattice needs more workspace than
 * 16 MiB (lbm_layout's ws_bytes: two-step lattices up to about 4096 x 4096
 * fit) or for tile_rows = -1 (its timing creates HIP events), LBM_EHIP when
 * the array's device address cannot be looked up.  The
 * array keeps the last call's contents, and every call on one GPU shares it:
 * calls that overlap on one GPU race. */
int lbm_init_static(lbm_ctx** ctx, const lbm_params* p, void* f_a, void* f_b, const double* rho0,
                    const double* ux0, const double* uy0, void* stream);

/* The two-step tile a context runs (LBM_VARIANT_BLOCK2): output rows and
 * wavefronts per workgroup, as lbm_describe reports them, after lbm_init's
 * timing when tile_rows = -1 (lbm_init then runs the lattice from its
 * initial state for a few launches of each candidate, alternating f_a and f_b
 * as lbm_step does, times them with HIP events, writes the initial state
 * again and synchronises the stream).  LBM_EINVAL for a null context or
 * another variant. */
int lbm_tile_shape(const lbm_ctx* ctx, int* rows_out, int* waves_out);

/* Advance nsteps time steps (Eq. LBE).  Asynchronous: device-side
 * instability is latched in the workspace and reported by lbm_status_check
 * or lbm_macros.  Steps t with t % reduce_every == 0 also add (t, mass, j_x,
 * j_y) of the state entering step t to the history (Eq. Density, Eq. Momentum,
 * FP64 in a fixed order: the same inputs and decomposition give the same bits).
 * LBM_ESTATE, before any launch, when the steps would pass the end of a
 * recording (lbm_set_recording) or of the checkpoint buffer. */
int lbm_step(lbm_ctx* ctx, int64_t nsteps, void* stream);

/* Synchronise `stream` and return LBM_EUNSTABLE if the device error word is
 * set (the message names the first failing step), else LBM_OK. */
int lbm_status_check(lbm_ctx* ctx, void* stream);

/* Macroscopic fields at the current time t: rho (Eq. Density), u (Eq.
 * Momentum, forced velocity), psi (Eq. InteractionPotential), p_EOS and the
 * Shan-Chen force F.  Any output may be NULL.  host_mass_mom (may be NULL)
 * receives {sum rho, sum rho u_x, sum rho u_y} (FP64, fixed-order
 * reduction).  Synchronises `stream`. */
int lbm_macros(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* psi, double* p,
               double* Fx, double* Fy, double* host_mass_mom, void* stream);

/* Distributions f_i(t, x) of Eq. LBE at the current time (pulled), as
 * float64 [9][ny][nx] on the device, whichever variant and (AA) layout
 * holds them.  Asynchronous. */
int lbm_populations(lbm_ctx* ctx, double* f_out, void* stream);

/* FP64 reduction history written by lbm_step when reduce_every > 0:
 * copies up to max_rows rows {step, mass, mom_x, mom_y} to host memory and
 * returns the row count through n_out.  Synchronises `stream`. */
int lbm_history(lbm_ctx* ctx, double* host_rows, int max_rows, int* n_out, void* stream);

/* Current step counter and the buffer that holds the current state (0: f_a, 1: f_b;
 * always 0 for LBM_VARIANT_AA, whose layout follows the parity of the step). */
int lbm_state(lbm_ctx* ctx, int64_t* step_out, int* cur_out);

/* Checkpoint / restore of the whole population state to caller memory
 * (device or host pointer of lbm_layout bytes).  Synchronous.  lbm_load sets
 * the step counter to `step`; with step != 0 it also turns recording and
 * checkpointing off (their contents belong to the trajectory before the
 * load), so a later lbm_adjoint returns LBM_ESTATE until the forward is run
 * again from step 0 with them re-enabled.  LBM_VARIANT_AA saves its buffer as
 * it lies, in the layout of the current step's parity: load it with a step of
 * the same parity. */
int lbm_save(lbm_ctx* ctx, void* dst, void* stream);
int lbm_load(lbm_ctx* ctx, const void* src, int64_t step, void* stream);

void lbm_destroy(lbm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Adjoint (discrete adjoint of lbm_step).  The loss is a function of the
 * final density field; the caller supplies dL/drho(x, T).  Gradients are
 * returned with respect to the four knots of the Smooth loop (Sec. III.D:
 * rho_max, p_max, rho_min, p_min, as independent parameters; the ellipse
 * coefficients follow them), the interaction constant G and the Eq. LiFS
 * sigma (held fixed while G varies).  The forward must run from step 0 with
 * recording or checkpointing enabled.  Recording keeps every step's record
 * (drho, j, psi) in HBM and the adjoint only runs the transposed steps;
 * checkpointing keeps the state every K steps and the adjoint recomputes each
 * K-step segment from its checkpoint (memory O(T/K) states + K records instead
 * of O(T) records).  Eq. RelaxationTime (var_tau) is not differentiated.
 * ------------------------------------------------------------------------ */

/* Bytes of the per-segment record (K steps of drho, j, psi) and of the
 * adjoint workspace for parameters p and checkpoint interval K. */
int lbm_adjoint_layout(const lbm_params* p, int K, size_t* rec_bytes, size_t* adj_bytes);
/* Store the state every K steps into ckpt_buf (device, ckpt_bytes; one slot
 * is lbm_layout's pop_bytes).  Call before the first lbm_step; K = 0 turns
 * checkpointing off.  lbm_step returns LBM_ESTATE when the slots run out. */
int lbm_set_checkpointing(lbm_ctx* ctx, void* ckpt_buf, size_t ckpt_bytes, int K);
/* Keep the record of every step 0 .. max_steps-1 of the forward in rec_buf
 * (device, caller-owned, rec_bytes >= the rec_bytes lbm_adjoint_layout gives
 * for K = max_steps: 4 planes of [ny][nx] in the storage precision per step,
 * step after step).  Call before the first lbm_step; max_steps = 0 turns it
 * off.  lbm_step returns LBM_ESTATE rather than step past max_steps.  A
 * recording forward runs the same node arithmetic and also writes 16 B (FP32)
 * or 32 B (FP64) per node and step. */
int lbm_set_recording(lbm_ctx* ctx, void* rec_buf, size_t rec_bytes, int64_t max_steps);
/* Gradient of L(rho(T)) given dL_drho_T (device float64 [ny][nx]).
 * grad_out (host, 6 doubles): dL/d{rho_max, p_max, rho_min, p_min, G, sigma}
 * (knot entries are 0 unless the shape is Smooth or Modified Smooth).
 * dL_drho0 (device [ny][nx], may be NULL): gradient with respect to the
 * initial density of f^eq(rho0, u = 0).  Synchronises; the forward state at
 * T is restored on return.  After a recorded forward rec_buf may be NULL (the
 * records are read from the recording buffer); after a checkpointed one it
 * holds one segment (lbm_adjoint_layout's rec_bytes for the same K), or two
 * (twice those bytes or more): then the recomputation of each segment runs on
 * a second stream of the library's,
 * beside the transposed steps of the one after it, ordered against `stream` by
 * events.  The result is the same either way. */
int lbm_adjoint(lbm_ctx* ctx, const double* dL_drho_T, void* rec_buf, size_t rec_bytes, void* adj_buf, size_t adj_bytes,
                double* grad_out, double* dL_drho0, void* stream);
/* lbm_adjoint for a loss on the final density and velocity: dL_drho_T, dL_dux_T,
 * dL_duy_T (device float64 [ny][nx], any of them NULL for zero, not all) with
 * u = (j + F/2)/rho of Eq. Momentum, F = psi F~ of Eq. ShanChenForce evaluated on
 * the final state (what lbm_macros returns).  Same workspaces, outputs and
 * errors as lbm_adjoint, which is this call with both velocity terms NULL. */
int lbm_adjoint_fields(lbm_ctx* ctx, const double* dL_drho_T, const double* dL_dux_T, const double* dL_duy_T,
                       void* rec_buf, size_t rec_bytes, void* adj_buf, size_t adj_bytes, double* grad_out,
                       double* dL_drho0, void* stream);
/* Replace the four interior knots of a built Smooth / Modified Smooth EOS and
 * recompute its ellipse coefficients (Sec. III.D); LBM_EINVAL when the knots
 * are out of order or an ellipse would not be real. */
int lbm_eos_set_knots(lbm_eos* e, double rho_max, double p_max, double rho_min, double p_min);

/* ------------------------------------------------------------------------
 * Batched lattices: B independent lattices (own size, EOS, relaxation times,
 * FP32 shift; one storage precision for all) advanced together, either by
 * grouped launches over every lattice at once or by one persistent launch in
 * which one workgroup owns one lattice and loops over the steps (see
 * lbm_step_batched and lbm_set_batch_mode for which runs when).  Either is
 * captured in HIP graphs and replayed.  Population buffers
 * hold the lattices back to back (lbm_batch_layout gives the sizes); scalar
 * fields are packed in lattice order, lattice b occupying
 * [cell_offsets[b], cell_offsets[b+1]) as [ny_b][nx_b].
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Sizes for B lattices with parameters p[0..B-1]: bytes of ONE population
 * buffer, bytes of the workspace, and (if non-NULL) cell_offsets[B+1]. */
int lbm_batch_layout(int B, const lbm_params* p, size_t* pop_bytes_out, size_t* ws_bytes_out, int64_t* cell_offsets);
/* Initial state f^eq(rho0, u0) of every lattice; rho0/ux0/uy0 packed device
 * float64 fields (ux0, uy0 may be NULL).  Validates every lattice. */
int lbm_init_batched(lbm_batch** ctx, int B, const lbm_params* p, void* f_a, void* f_b, void* ws, size_t ws_bytes,
                     const double* rho0, const double* ux0, const double* uy0, void* stream);
/* nsteps time steps of every lattice (asynchronous).  Persistent mode: one
 * launch in which one workgroup per lattice loops over the steps.  Grouped
 * mode: launches over all lattices at once, two steps per launch (whole
 * columns per workgroup when every lattice is periodic and at most 16 rows
 * tall, else the two-step tiles), an odd last step on its own, replayed as
 * HIP graphs of 128 steps.  Launches replayed from a graph keep the step
 * numbers of their capture, so the step that lbm_status_batched names is
 * exact only within the first capture. */
int lbm_step_batched(lbm_batch* ctx, int64_t nsteps, void* stream);
/* Choose how lbm_step_batched runs: LBM_BATCH_AUTO (default: grouped when some
 * lattice has more than 32 strip-rows, i.e. more than two per wavefront of
 * its persistent workgroup), LBM_BATCH_PERSISTENT or LBM_BATCH_GROUPED. */
typedef enum { LBM_BATCH_AUTO = 0, LBM_BATCH_PERSISTENT = 1, LBM_BATCH_GROUPED = 2 } lbm_batch_mode;
int lbm_set_batch_mode(lbm_batch* ctx, int mode);
/* Packed rho and forced u of every lattice (outputs may be NULL); synchronises. */
int lbm_macros_batched(lbm_batch* ctx, double* rho, double* ux, double* uy, void* stream);
/* LBM_EUNSTABLE if any lattice met psi^2 < 0; first_bad_out = its index or -1. */
int lbm_status_batched(lbm_batch* ctx, int* first_bad_out, void* stream);
void lbm_destroy_batched(lbm_batch* ctx);

/* ------------------------------------------------------------------------
 * Finite-difference reference solver (appendix "Finite Difference Method"):
 * the mass equation and Eq. FDmomentum for rho, u, v on a mesh of spacing h
 * (LBM units, c = 1, c_s^2 = 1/3), periodic in x and, in y, periodic or
 * bounded by the wall layers described below; viscous stress of
 * Eq. StressTensor with Eq. DynamicViscosity (tau_nu(rho) of
 * Eq. RelaxationTime when var_tau), pseudopotential pressure tensor through
 * Eq. FDforce, MacCormack predictor (forward one-sided first derivatives) and
 * corrector (backward), central second and higher derivatives.  FP64.
 * Walls (appendix "Grid-Dependency Study"): the layer b1 one node below row 0
 * lies on the bottom wall (u = v = 0, rho and psi extrapolated from rows 0 and
 * 1), b2 below it holds psi of Eq. B2 with psi_l = psi(eos.rho_l); row ny-1 lies
 * on the top wall and the layers above mirror rows ny-2 and ny-3 with the
 * velocity reversed.
 * ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny;           /* mesh nodes (>= 3 each), periodic in x */
    int var_tau;          /* 1: tau_nu from Eq. RelaxationTime (tau_l, tau_v, rho_*_tau) */
    int walls;            /* 0: periodic in y; 1: the wall layers above */
    double h, dt;         /* mesh spacing and time step (LBM units) */
    double G, eps;        /* interaction constant (< 0); eps of the pressure tensor (Li: -16 G sigma, Guo: 0) */
    double tau_e, tau_nu; /* relaxation times of Eq. DynamicViscosity */
    double tau_l, tau_v, rho_v_tau, rho_l_tau;
    lbm_eos eos;          /* built by lbm_eos_build */
} lbm_fd_params;
typedef struct lbm_fd_ctx lbm_fd_ctx;

/* Bytes of the caller-owned device buffer (an error word and 6 float64 fields
 * [ny][nx]: the state and the predicted state); LBM_EINVAL for bad sizes, h, dt or G. */
int lbm_fd_layout(const lbm_fd_params* p, size_t* bytes);
/* Initial state: rho0, u0, v0 device float64 [ny][nx] (u0, v0 may be NULL for
 * rest).  The buffer holds all solver state; the context holds only pointers. */
int lbm_fd_init(lbm_fd_ctx** ctx, const lbm_fd_params* p, void* buf, size_t buf_bytes, const double* rho0,
                const double* u0, const double* v0, void* stream);
/* nsteps predictor-corrector steps (asynchronous; one launch per step, the
 * predicted state kept in LDS). */
int lbm_fd_step(lbm_fd_ctx* ctx, int64_t nsteps, void* stream);
/* Copy rho, u, v (device float64 [ny][nx], any may be NULL); asynchronous. */
int lbm_fd_fields(lbm_fd_ctx* ctx, double* rho, double* u, double* v, void* stream);
/* LBM_EUNSTABLE once a node met psi^2 < 0 or rho <= 0; synchronises. */
int lbm_fd_status(lbm_fd_ctx* ctx, void* stream);
void lbm_fd_destroy(lbm_fd_ctx* ctx);

const char* lbm_strerror(int code);
const char* lbm_last_error(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
