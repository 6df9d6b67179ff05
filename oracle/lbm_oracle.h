/*
 * lbm_oracle.h -- plain FP64 CPU oracle for the two-component immiscible
 * pseudopotential (Shan-Chen) MRT lattice Boltzmann step with the corrected
 * open boundaries of Chen, Pan, Wang, Li & Chen, "A corrected open boundary
 * framework for lattice Boltzmann immiscible pseudopotential models"
 * (arXiv:2512.12934).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP product library.
 *
 * Conventions
 *   - dim = 2 (D2Q9) or 3 (D3Q19); in 2-D n[2] == 1.
 *   - node index  n = x + n0*(y + n1*z).
 *   - distribution arrays are [component k][direction i][node]  (k in {0,1}).
 *   - vectors are [component][axis][node] with 3 axes even in 2-D.
 *   - D2Q9 order (Sec. II B, App. B):  0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0);
 *     4 (0,-1); 5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1).
 *   - D3Q19 order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),
 *     (-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
 *     (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *   The state f is the post-streaming, post-boundary distribution; a "step"
 *   takes f(t) to f(t+1).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_INLETS 8

/* An inlet patch: fluid nodes of the face layer (axis, side) whose two
 * tangential coordinates lie in [lo, hi).  Later patches take precedence
 * over earlier ones where rectangles overlap.  rho[k] and u_n (speed along
 * the inward normal) are the prescribed inlet quantities of eq. (13). */
typedef struct {
    int axis, side;          /* side 0: coordinate 0 ; side 1: n[axis]-1 */
    int lo[3], hi[3];        /* tangential extent (normal axis ignored) */
    double rho[2];
    double u_n;
    int alpha_on;            /* 1: eqs. (15)-(19) correction, 0: eq. (13) only */
} orc_inlet;

/* The outlet: fluid nodes of the face layer (axis, side) inside [lo, hi). */
typedef struct {
    int axis, side;
    int lo[3], hi[3];
    int chi_on;              /* 1: eqs. (22)-(23) velocity correction */
} orc_outlet;

typedef struct {
    int dim;
    int n[3];
    int periodic[3];
    double nu[2];            /* kinematic viscosities, eq. (5) */
    double s_q;              /* energy-flux relaxation rate */
    int s_eps_policy;        /* 0: s_eps from the most viscous phase; 1: s_eps = s_nu,k */
    double G12;              /* fluid-fluid strength, eq. (10) */
    double Gw[2];            /* constant adhesion strengths, eq. (11) */
    double Fb[3];            /* body-force density (split by rho_k / rho) */
    int n_inlets;
    orc_inlet inlets[ORC_MAX_INLETS];
    int has_outlet;
    orc_outlet outlet;
} orc_params;

typedef struct orc_sim orc_sim;

/* Diagnostics of the last step (FP64). */
typedef struct {
    int64_t step;
    double q_in;      /* sum over inlet nodes of rho u . n_inward          */
    double q_out;     /* sum over the x_{N-1} column of rho u . n_outward  */
    double chi;       /* eq. (23) coefficient applied this step (1 if none) */
    double u_conv;    /* eq. (21) convective velocity (after clamp >= 0)    */
    double mass[2];
    double mass0[2];
    int64_t uc_clamps;
} orc_diag;

/* ---- tables and per-node building blocks (used by the pins) ---- */
int  orc_Q(int dim);
/* e: [Q][3] (int), w: [Q], T: [Q][Q] row-major, Tinv: [Q][Q]. */
void orc_tables(int dim, int *e, double *w, double *T, double *Tinv);
/* Relaxation rates for component k, [Q]. */
void orc_relaxation(const orc_params *p, int k, double *s);
void orc_feq(int dim, double rho, const double *u, double *feq);
void orc_forcing(int dim, const double *u, const double *F, double *Fbar);
/* eq. (1): post-collision populations of one node and one component. */
void orc_collide_node(int dim, const double *s, const double *f, double rho,
                      const double *u, const double *F, double *fout);
/* Force stencil: returns the number of neighbours; off [K][3], w [K]. */
int  orc_stencil(int dim, int *off, double *w);

/* Moving walls: uw [3][N] is the velocity of every solid node (ignored on
 * fluid nodes); NULL makes every wall rest again.  A population bounced back
 * from a solid node s at the fluid node x picks up the wall's momentum,
 * f_ibar(x, t+1) = f*_i(x) - 2 w_i rho_k(x) (e_i . u_w(s)) / cs^2
 * (halfway bounce-back with a moving wall, Ladd; rho_k is the component's
 * density at x).  Copied. */
void orc_set_wall_velocity(orc_sim *s, const double *uw);

/* ---- OpenMP threads of the node loops (timing only) ---- */
int  orc_threads(void);
void orc_set_threads(int n);

/* ---- whole-domain simulation ---- */
orc_sim *orc_create(const orc_params *p, const uint8_t *solid,
                    const double *rho0, const double *u0);
void orc_destroy(orc_sim *s);
void orc_step(orc_sim *s, int64_t nsteps);
void orc_get_f(const orc_sim *s, double *f);
void orc_set_f(orc_sim *s, const double *f);
/* rho [2][N], u [3][N] (common velocity eq. (7)-(8), before any outlet
 * override), F [2][3][N] (total force on each component).  Any may be NULL. */
void orc_moments(orc_sim *s, double *rho, double *u, double *F);
void orc_diagnostics(orc_sim *s, orc_diag *d);

/* ---- test hooks: single stages of a step on a planted state ----
 * fn is the buffer of f(t+1) that streaming fills and stages 7-8 complete
 * ([2][Q][N]); F is the force of stage 2 ([2][3][N]).  orc_stage runs one
 * stage of the step on the current buffers without swapping them:
 * 1 = stages 1-3 (densities, forces, velocity from f), 4 = outlet velocity
 * correction, 5 = collision and streaming (stages 5-6), 7 = inlet,
 * 8 = convective outflow. */
void orc_set_next(orc_sim *s, const double *fn);
void orc_get_next(const orc_sim *s, double *fn);
void orc_set_force(orc_sim *s, const double *F);
void orc_stage(orc_sim *s, int stage);
int64_t orc_nodes(const orc_sim *s);

#ifdef __cplusplus
}
#endif
#endif
