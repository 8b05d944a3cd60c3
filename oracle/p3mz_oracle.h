/*
 * p3mz_oracle.h -- plain CPU FP64 reference of the P3MaZe mesh step.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes (Theory section of the paper):
 *   charge assignment with cardinal B-splines of order p, diffusion-type
 *   smoothing of the mesh charges, the Verlet prediction of the mesh
 *   potential and the constraint residual at the prediction (Eqs. 16-17),
 *   the correction problem M y = sigma_p solved by multigrid V-cycles with a
 *   max-norm residual test (Eq. 26), the field update of the Supporting
 *   Information ("Numerical integration"), the long-range force by
 *   interpolating a central-difference mesh gradient (Eq. 21), the screened
 *   short-range pair force (Eq. 20) and the energy split of Eq. 5 with
 *   Eqs. 6 and 7.  Every number is IEEE double; nothing is emulated in FP32.
 *
 * Units: lengths in the caller's length unit (Angstrom in the tests), charges
 * in e, energies and forces scaled by coulomb_k.
 */
#ifndef P3MZ_ORACLE_H
#define P3MZ_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_CYCLES 64
#define ORC_MAX_LEVELS 16

enum {
  ORC_OK = 0,
  ORC_WARN_NOT_CONVERGED = 1,
  ORC_ERR_INVALID_ARG = -1,
  ORC_ERR_NOT_NEUTRAL = -2,
  ORC_ERR_MESH_SHAPE = -3,
  ORC_ERR_OUT_OF_MEMORY = -4
};

enum { ORC_MESH_Q = 0, ORC_MESH_QS = 1, ORC_MESH_SIGMA_P = 2, ORC_MESH_Y = 3,
       ORC_MESH_PHI = 4, ORC_MESH_PHI_PREV = 5, ORC_MESH_Y_START = 6 };

typedef struct {
  double box;          /* cubic edge L                                        */
  double alpha;        /* Ewald splitting; Gaussian width sigma = 1/(sqrt2 a) */
  double r_cut;        /* real-space cutoff, 0 < r_cut <= L/2                 */
  int32_t mesh;        /* N points per edge, N = 4 * 2^m, m >= 1              */
  int32_t order;       /* B-spline order p, 2..7                              */
  double tol;          /* residual tolerance                                  */
  int32_t tol_mode;    /* 0: max|r| <= tol*max|q^s|; 1: max|r| <= tol         */
  int32_t max_cycles;  /* V-cycle cap per step, 0..ORC_MAX_CYCLES             */
  int32_t predictor;   /* multiplier predictor 0..3                           */
  double coulomb_k;    /* Coulomb constant                                    */
  int32_t nu_pre;      /* red-black Gauss-Seidel sweeps before restriction   */
  int32_t nu_post;     /* ... after prolongation                             */
  int32_t excl_group;  /* 0: none; g > 0: atoms i, j with i/g == j/g excluded */
  int32_t stencil;     /* 0: 7-point Laplacian, 2-point central gradient;
                          1: 19-point Mehrstellen (Hermitian) Laplacian with
                          its right-hand-side operator, 4-point gradient     */
} orc_params;

typedef struct {
  double h, sigma, sigma_s2, nu_smooth;
  int32_t K;                 /* smoothing steps per dimension   */
  int32_t levels;            /* multigrid levels down to 4^3    */
  int32_t nl[ORC_MAX_LEVELS];
} orc_plan;

typedef struct {
  int32_t status;            /* ORC_OK or ORC_WARN_NOT_CONVERGED */
  int32_t cycles;            /* V-cycles used in the last step   */
  int32_t cold;              /* 1 if the last step was a cold solve */
  int32_t m_eff;             /* predictor order actually used    */
  double thresh;             /* residual threshold of the last step */
  double norm_qs;            /* max|q^s|                         */
  double res_hist[ORC_MAX_CYCLES + 1]; /* residual before cycle c  */
  double e_sr, e_lr, e_self, e_total;
  double t_spread, t_solve, t_gather, t_sr;   /* wall seconds, last step */
  int64_t steps;             /* completed compute calls          */
} orc_stats;

typedef struct {
  int32_t model;       /* 0 none, 1 NaCl stand-in repulsion, 2 flexible water */
  double bm_a, bm_rho; /* stand-in repulsion A*exp(-r/rho) between all pairs  */
  double lj_eps, lj_sigma;   /* O-O Lennard-Jones                             */
  double k_bond, r0;   /* harmonic O-H bond: 0.5*k*(r-r0)^2                   */
  double k_angle, theta0;    /* harmonic H-O-H angle: 0.5*k*(th-th0)^2 [rad]  */
  double force_to_acc; /* acceleration = force / mass * force_to_acc          */
  double mv2_to_energy;/* kinetic energy = 0.5 * m v^2 * mv2_to_energy        */
} orc_mdterms;

typedef struct orc_state orc_state;

/* --- building blocks (exported so the tests can pin each one) ----------- */
int    orc_plan_make(const orc_params* p, orc_plan* out);
double orc_bspline(int p, double x);
void   orc_stencil_1d(int p, int n, double u, int32_t* idx, double* w);
void   orc_assign(int p, int n, double box, int64_t n_atoms, const double* pos,
                  const double* q_atoms, double* q_mesh);
void   orc_smooth(int n, int k_steps, double nu, double* v);
void   orc_apply_m(int n, const double* v, double* out);
void   orc_rbgs(int n, double* e, const double* r, int colour);
void   orc_restrict(int n, const double* rho, double* rc);
void   orc_prolong_add(int nc, const double* ec, double* e);
void   orc_coarsest(const double* r, double* e);
int    orc_vcycle_apply(orc_state* s, const double* r, double* e);
void   orc_sr(int64_t n_atoms, const double* pos, const double* q, double box,
              double alpha, double r_cut, double k_e, int32_t excl_group,
              const int64_t* targets, int64_t n_targets, double* force, double* e_atom);
int    orc_ewald(int64_t n_atoms, const double* pos, const double* q, double box,
                 double alpha, double k_e, double eps, double* energy3, double* force);

/* --- the mesh step ------------------------------------------------------ */
int  orc_create(const orc_params* p, int64_t n_atoms, const double* charges, orc_state** out);
void orc_destroy(orc_state* s);
int  orc_compute(orc_state* s, const double* pos, double* force, double* energy4);
/* Short-range subset for large systems: with n_targets >= 0 the pair term
 * is formed only for the listed atoms (against all partners); the other
 * atoms' forces are long-range only and e_sr / e_total become NaN.
 * n_targets = 0 skips the pair term; n_targets = -1 restores the full sum. */
int  orc_set_sr_targets(orc_state* s, const int64_t* targets, int64_t n_targets);
int  orc_get_stats(const orc_state* s, orc_stats* out);
int  orc_get_plan(const orc_state* s, orc_plan* out);
int  orc_get_mesh(const orc_state* s, int which, double* out);
int  orc_reset_history(orc_state* s);
int  orc_save_state(const orc_state* s, void* buf, size_t* bytes);
int  orc_load_state(orc_state* s, const void* buf, size_t bytes);
int  orc_md_run(orc_state* s, double* pos, double* vel, const double* mass,
                const orc_mdterms* t, double dt, int32_t n_steps,
                double* energy_log /* [n_steps][6] */, int32_t* cycles_log);
/* OVRVO Langevin thermostat for orc_md_run (gamma 0: none); resets its step
 * counter.  The generator and the normals are exported for their pins. */
int  orc_set_thermostat(orc_state* s, double gamma, double kt, uint64_t seed);
void orc_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4]);
void orc_thermo_normals(uint64_t seed, int64_t a, int64_t step, int half, double z[3]);
int  orc_nonelectrostatic(const orc_mdterms* t, int64_t n_atoms, const double* pos,
                          double box, double r_cut, double* force, double* energy);

/* Fourth-order (Hermitian, Mehrstellen) mesh operators of the stencil-1
 * discretisation: out = A v with A = (1/6)(2 sum_faces + sum_edges - 24),
 * the 19-point Laplacian times h^2, and out = B v with
 * B = 1/2 + (1/12) sum_faces, its right-hand-side operator; the discrete
 * Poisson equation is then A phi = -(4 pi / h) B q. */
void orc_apply_a19(int n, const double* v, double* out);
void orc_apply_b(int n, const double* v, double* out);

#ifdef __cplusplus
}
#endif
#endif
