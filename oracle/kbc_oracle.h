/*
 * kbc_oracle.h -- FP64 CPU oracle for the D2Q9 lattice Boltzmann step with the
 * entropic multi-relaxation (KBC) collision of Boesch, Chikatamarla and Karlin,
 * "Entropic Multi-Relaxation Models for Simulation of Fluid Turbulence"
 * (arXiv:1507.02509), and the LBGK baseline.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * GPU results are checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Conventions (the interface the GPU library also documents):
 *   - velocity order i = 0..8: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *     (-1,-1) (1,-1), the D2Q9 set v_(i,j) = (i,j) of section "Moment
 *     Representation";
 *   - a lattice state is double f[9][ny][nx], x fastest, holding the
 *     pre-collision populations f_i(x, t) of eq. (Egeneral);
 *   - one step collides every node and pushes f_i' to x + v_i, wrapping
 *     periodically in both directions.
 *
 * Parity status of each function is stated in the repository's design notes;
 * every function here is pinned by a CPU test except where a comment says
 * "parity unpinned".
 */
#ifndef KBC_ORACLE_H
#define KBC_ORACLE_H

#include <stdint.h>

#define ORC_Q 9
#define ORC_NDIAG 16

enum { ORC_LBGK = 0, ORC_KBC = 1 };
enum { ORC_KBC_A = 0, ORC_KBC_B = 1, ORC_KBC_C = 2, ORC_KBC_D = 3 };
enum { ORC_GAMMA_ESTIMATE = 0, ORC_GAMMA_FIXED = 1, ORC_GAMMA_EXACT = 2 };
enum { ORC_INIT_EQ = 0, ORC_INIT_GRAD_CD = 1, ORC_INIT_GRAD_GIVEN = 2 };

/* diagnostics slots written by orc_diagnostics */
enum {
    ORC_D_MASS = 0, ORC_D_JX, ORC_D_JY,
    ORC_D_E, ORC_D_E_STD, ORC_D_Z, ORC_D_Z_STD, ORC_D_P, ORC_D_P_STD,
    ORC_D_S, ORC_D_GAMMA, ORC_D_GAMMA_STD,
    ORC_D_NONFINITE, ORC_D_FEQ_NONPOS, ORC_D_RHO_STD, ORC_D_UNUSED
};

typedef struct {
    int32_t nx, ny;
    double beta;          /* relaxation parameter, nu = cs2 (1/(2 beta) - 1/2) */
    int32_t collision;    /* ORC_LBGK or ORC_KBC */
    int32_t variant;      /* ORC_KBC_A .. ORC_KBC_D, Table kbc_moment_grouping */
    int32_t gamma_mode;   /* ORC_GAMMA_* */
    double gamma_guard;   /* gamma = 2 when <dh|dh> <= gamma_guard * <ds|ds> */
    double gamma_fixed;   /* used by ORC_GAMMA_FIXED */
    int32_t threads;      /* OpenMP threads for lattice loops (<= 0: 1) */
} orc_params;

/* ---- lattice constants ---- */
double orc_cs2(void);
void orc_velocities(int32_t cx[ORC_Q], int32_t cy[ORC_Q]);
void orc_weights(double W[ORC_Q]);

/* ---- single-node functions (pins and the adjoint oracle use these) ---- */
void orc_node_equilibrium(double rho, double ux, double uy, double feq[ORC_Q]);
void orc_node_natural(const double f[ORC_Q], double r[ORC_Q]);
void orc_node_central(const double f[ORC_Q], double ct[6]);
void orc_node_central_to_natural(double ux, double uy, const double ct[6], int32_t kin,
                                 double nat[6]);
void orc_node_populations(const double r[ORC_Q], double f[ORC_Q]);
void orc_node_split(int32_t variant, const double f[ORC_Q], double k[ORC_Q], double s[ORC_Q],
                    double h[ORC_Q]);
/* deviations ds = s(f) - s(feq), dh = h(f) - h(feq) and the entropic scalar
 * products out = (<ds|dh>, <dh|dh>, <ds|ds>) */
void orc_node_deviations(int32_t variant, const double f[ORC_Q], double ds[ORC_Q],
                         double dh[ORC_Q], double out[3]);
double orc_node_collide(const orc_params* p, const double f[ORC_Q], double out[ORC_Q]);
double orc_node_result1(const orc_params* p, const double f[ORC_Q], double gamma);
void orc_node_grad(double rho, double ux, double uy, const double du[4], double beta,
                   double f[ORC_Q]);

/* ---- lattice functions; all fields are [ny][nx] doubles, states [9][ny][nx] ---- */
int orc_init(const orc_params* p, const double* rho, double rho0, const double* ux,
             const double* uy, const double* grad, int32_t mode, double* f);
int orc_step(const orc_params* p, const double* fin, double* fout, double* gamma);
int orc_run(const orc_params* p, double* f, double* work, int32_t nsteps);

/* ---- storage rounding (emulation of reduced-precision state storage) ----
 * ORC_STORE_F32: the deviation g_i = f_i - W_i rho0 rounded to binary32;
 * ORC_STORE_F16: g_i 2^s_i rounded to binary16 (s = 1 for the rest
 * population, 3 for the axis ones, 5 for the diagonals) and scaled back.
 * Rounding is to nearest, ties to even.  orc_round_storage rounds a state in
 * place; orc_run_stored runs nsteps steps rounding the state after each (the
 * initial state is rounded by the caller). */
enum { ORC_STORE_F64 = 0, ORC_STORE_F32 = 1, ORC_STORE_F16 = 2 };
double orc_round_f16(double x);
int orc_round_storage(const orc_params* p, double rho0, int32_t storage, double* f);
int orc_run_stored(const orc_params* p, double rho0, int32_t storage, double* f, double* work, int32_t nsteps);
int orc_moments(const orc_params* p, const double* f, double* rho, double* ux, double* uy);
int orc_gamma_field(const orc_params* p, const double* f, double* gamma);
int orc_diagnostics(const orc_params* p, const double* f, double out[ORC_NDIAG]);

/* ---- adjoint oracle (kbc_oracle_adj.c) ---- */
void orc_node_jacobian(const orc_params* p, const double f[ORC_Q], double J[ORC_Q * ORC_Q],
                       double dbeta[ORC_Q]);
int orc_adjoint_step(const orc_params* p, const double* f, const double* lam_next,
                     double* lam, double* dbeta);
int orc_init_adjoint(const orc_params* p, double rho0, const double* ux, const double* uy,
                     int32_t mode, const double* lam0, double* gux, double* guy,
                     double* dbeta);

#endif
