/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of the shaped-EOS pseudopotential
 * lattice Boltzmann method (Czelusniak, Mapelli, Cabezas Gomez, Wagner,
 * "Shaping the equation of state to improve numerical accuracy and
 * stability of the pseudopotential lattice Boltzmann method").
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load or call this library.  It shares no code, header, table or constant
 * with the HIP product path under paper_2107_06355_amd/.
 *
 * Every routine follows the paper's equations in the paper's order:
 *   Sec. II.A  Eq. LBE, Eq. OperatorMRT, Eq. VelocitySet, Eq. MatrixMRT,
 *              Eq. RelaxationMatrix, Eq. Density, Eq. Momentum, Eq. GFS,
 *              Eq. EquilibriumDistribution
 *   Sec. II.B  Eq. ShanChenForce, Eq. InteractionPotential, Eq. MaxwellRule,
 *              Eq. ShanVaporLiqEq
 *   Sec. II.C  Eq. VaporLiqEq, Eq. LiFS, eps = -16 G sigma
 *   Sec. II.D  Eq. PengEOS, Eq. PengTheta
 *   Sec. III   Eq. CS, Sec. III.D (Smooth vdW-loop replacement)
 *   Sec. IV    Eq. RelaxationTime, bounce-back walls with ghost densities
 *
 * Readings of passages that are ambiguous or garbled are listed in the
 * header comment of lbm_oracle.c.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_EINVAL = -1, OR_EUNSTABLE = -2, OR_ENOROOT = -5 };
enum { OR_BASE_CS = 0, OR_BASE_PR = 1 };
enum { OR_SHAPE_NONE = 0, OR_SHAPE_SMOOTH = 1, OR_SHAPE_MODSMOOTH = 2, OR_SHAPE_PENG = 3 };
enum { OR_FORCING_GUO = 0, OR_FORCING_LI = 1 };

typedef struct {
    /* inputs */
    int base;          /* OR_BASE_CS (Eq. CS) or OR_BASE_PR (textbook Peng-Robinson) */
    int shape;         /* OR_SHAPE_* */
    double a, b, R, omega;
    double Tr;         /* reduced temperature T/Tc */
    double scale;      /* multiplies the whole base EOS ("standard procedure", Sec. III.B) */
    double alpha;      /* Smooth: p_min = p_sat_new - alpha (p_sat - p_min_base) */
    double k_vap;      /* Smooth: vapor branch = k_vap * base EOS (Sec. III.D, raised vapor slope) */
    double r_theta;    /* Peng: Eq. PengTheta */
    /* outputs of or_eos_build */
    double Tc, T;
    double rho_v, rho_l, p_sat;          /* Maxwell coexistence of the (scaled) base EOS */
    double rho_max, p_max_base;          /* local maximum of the base EOS (vdW loop) */
    double rho_min, p_min_base;          /* local minimum of the base EOS */
    double p_sat_new, dP_liq;            /* shaped saturation pressure, liquid offset */
    double slope_v, slope_l;             /* dp/drho of the shaped EOS at rho_v and rho_l */
    double p_max, p_min;                 /* interior knots of the shaped loop */
    double a1sq, b1, a3sq, b3;           /* ellipse coefficients, regions 1 and 3 */
    double rho_m, theta;                 /* Peng loop */
    double eps;                          /* root of Eq. VaporLiqEq (0 for Guo-forcing shapes) */
} or_eos;

typedef struct {
    int nx, ny;
    int walls;            /* 0: periodic in y; 1: half-way bounce-back below row 0 and above row ny-1 */
    int forcing;          /* OR_FORCING_GUO or OR_FORCING_LI */
    int var_tau;          /* 1: tau_nu from Eq. RelaxationTime */
    int pad_;
    double rho_wall_lo, rho_wall_hi;  /* densities given to the solid nodes in the force sum */
    double G, sigma;
    double tau[9];        /* relaxation times in the moment order of Eq. RelaxationMatrix */
    double tau_l, tau_v;  /* Eq. RelaxationTime */
    double rho_v_tau, rho_l_tau;
    or_eos eos;
} or_params;

/* thermodynamics (host precompute, FP64) */
int    or_eos_build(or_eos* e, double G, double* sigma_out);
int    or_eos_set_knots(or_eos* e, double rho_max, double p_max, double rho_min, double p_min);
double or_base_p(const or_eos* e, double rho);
double or_base_dp(const or_eos* e, double rho);
double or_eos_p(const or_eos* e, double rho);
double or_eos_dp(const or_eos* e, double rho);
double or_cs_critical_eta(void);
double or_maxwell_residual(const or_eos* e, double p0, double rho_lo, double rho_hi, int shaped);
double or_mech_residual(const or_eos* e, double eps, double G);

/* lattice */
typedef struct or_lattice or_lattice;
or_lattice* or_lattice_new(const or_params* p);
void   or_lattice_free(or_lattice* L);
void   or_init_eq(or_lattice* L, const double* rho, const double* ux, const double* uy);
void   or_set_f(or_lattice* L, const double* f);
void   or_get_f(const or_lattice* L, double* f);
int    or_run(or_lattice* L, long long nsteps);
int    or_threads(void);  /* threads of a time step: 1, or OpenMP's count in the -DOR_OMP build */
int    or_run_window(or_lattice* L, long long nsteps); /* psi^2 < 0 gives NaN psi instead of stopping */
long long or_fail_step(const or_lattice* L);
int    or_macros(or_lattice* L, double* rho, double* ux, double* uy, double* psi, double* p,
                 double* Fx, double* Fy);

/* one collision of one node (Eq. LBE right-hand side), for algebra tests */
void   or_collide_node(const or_params* p, const double* f, double Fx, double Fy, double psi,
                       double Ftx, double Fty, double* fout);
void   or_force_tilde_field(int nx, int ny, const double* psi, int walls, double psi_lo, double psi_hi,
                            double G, double* Ftx, double* Fty);
void   or_feq(double rho, double ux, double uy, double* feq);
void   or_matrix(double* M, double* Minv);

/* Finite-difference reference solver (Appendix "Finite Difference Method"), fd_oracle.c */
typedef struct {
    int nx, ny;           /* mesh nodes; periodic in x */
    int var_tau;          /* 1: tau_nu from Eq. RelaxationTime */
    int walls;            /* 0: periodic in y; 1: wall layers of the appendix (bottom b1/b2, top on row ny-1) */
    double h, dt;         /* mesh spacing and time step, LBM units */
    double G, eps;        /* interaction constant; eps of the pressure tensor (Li: -16 G sigma; Guo: 0) */
    double tau_e, tau_nu; /* Eq. DynamicViscosity */
    double tau_l, tau_v, rho_v_tau, rho_l_tau;
    double psi_wall;      /* psi_l of Eq. B2 (solid layer below the bottom wall) */
    or_eos eos;
} or_fd_params;
typedef struct or_fd or_fd;
or_fd* or_fd_new(const or_fd_params* p);
void   or_fd_free(or_fd* f);
void   or_fd_set(or_fd* f, const double* rho, const double* u, const double* v);
void   or_fd_get(const or_fd* f, double* rho, double* u, double* v);
int    or_fd_run(or_fd* f, long long nsteps);

#ifdef __cplusplus
}
#endif
#endif
