/*
 * lbm_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * One lattice step of the two-component immiscible pseudopotential MRT LBM
 * with the corrected open boundaries of arXiv:2512.12934, written stage by
 * stage in the paper's order and notation:
 *
 *   1. densities rho_k = sum_i f_i^k and pseudopotentials psi_k = rho_k
 *      (Sec. II A, eq. 8); mirror ghost layers at open faces (eqs. 24-25);
 *   2. forces: fluid-fluid 8th-order stencil (eq. 10, weights of Sec. II A),
 *      wall adhesion (eq. 11) and a body force;
 *   3. common velocity with the half-force term (eqs. 7-8);
 *   4. outlet velocity correction from the inlet/outlet mass-flow balance
 *      (eqs. 22-23, App. A);
 *   5. MRT collision with the forcing term (eqs. 1, 3-6, 9);
 *   6. streaming with halfway bounce-back and periodic wrap (eq. 2, App. B);
 *   7. non-equilibrium extrapolation inlet and its alpha correction
 *      (eqs. 13-19, App. A);
 *   8. convective outflow (eqs. 20-21).
 *
 * Nothing here is blocked, fused or reordered for speed: every stage is a
 * full loop over nodes with OpenMP, and eq. (1) is applied literally as
 * f - (T^-1 S T)(f - feq) + (T^-1 (I - S/2) T) Fbar with dense matrices.
 *
 * Readings of passages that are garbled or silent are stated where used.
 * This file shares no code with the HIP product library.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19
#define KMAX 92

/* ------------------------------------------------------------------ */
/* Lattices                                                           */
/* ------------------------------------------------------------------ */

/* D2Q9 velocities in the order implied by the unknown sets {1,5,8} (left
 * inflow), {4,7,8} (top inflow) and {3,6,7} (right outlet) of Sec. II B
 * and the periodic sets of eq. (B2). */
static const int E2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};

/* D3Q19 (not given in the paper): rest, 6 faces, 12 edges. */
static const int E3[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

int orc_Q(int dim) { return dim == 2 ? 9 : 19; }

#ifdef _OPENMP
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif

static const int (*lat_e(int dim))[3] { return dim == 2 ? E2 : E3; }

/* Weights: D2Q9 4/9, 1/9, 1/36 (Sec. II A); D3Q19 1/3, 1/18, 1/36. */
static double lat_w(int dim, int i)
{
    const int (*e)[3] = lat_e(dim);
    int e2 = e[i][0] * e[i][0] + e[i][1] * e[i][1] + e[i][2] * e[i][2];
    if (dim == 2) return e2 == 0 ? 4.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    return e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* Row r of the moment matrix T evaluated at velocity e.
 *
 * D2Q9 (eq. 3): the printed rows 0-2 are 1, -4+3|e|^2, 4-21|e|^2/2+9|e|^4/2;
 * the printed rows 3-8 are not mutually orthogonal, so they are taken as the
 * orthogonal polynomial basis whose order matches S of eq. (4):
 * j_x = e_x, q_x = (3|e|^2-5) e_x, j_y, q_y, p_xx = e_x^2 - e_y^2,
 * p_xy = e_x e_y.
 *
 * D3Q19 (absent from the paper): the 19 orthogonal polynomials
 * 1, 19|e|^2-30, (21|e|^4-53|e|^2+24)/2, e_x, (5|e|^2-9)e_x, e_y, ..., e_z,
 * ..., 3e_x^2-|e|^2, (3|e|^2-5)(3e_x^2-|e|^2), e_y^2-e_z^2,
 * (3|e|^2-5)(e_y^2-e_z^2), e_xe_y, e_ye_z, e_xe_z, (e_y^2-e_z^2)e_x,
 * (e_z^2-e_x^2)e_y, (e_x^2-e_y^2)e_z. */
static double moment_row(int dim, int r, const int *e)
{
    double x = e[0], y = e[1], z = e[2];
    double e2 = x * x + y * y + z * z;
    if (dim == 2) {
        switch (r) {
        case 0: return 1.0;
        case 1: return -4.0 + 3.0 * e2;
        case 2: return 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
        case 3: return x;
        case 4: return (3.0 * e2 - 5.0) * x;
        case 5: return y;
        case 6: return (3.0 * e2 - 5.0) * y;
        case 7: return x * x - y * y;
        case 8: return x * y;
        }
        return 0.0;
    }
    switch (r) {
    case 0: return 1.0;
    case 1: return 19.0 * e2 - 30.0;
    case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * e2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * e2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * e2 - 9.0) * z;
    case 9: return 3.0 * x * x - e2;
    case 10: return (3.0 * e2 - 5.0) * (3.0 * x * x - e2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * e2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    case 18: return (x * x - y * y) * z;
    }
    return 0.0;
}

void orc_tables(int dim, int *e, double *w, double *T, double *Tinv)
{
    int Q = orc_Q(dim);
    const int (*E)[3] = lat_e(dim);
    for (int i = 0; i < Q; i++) {
        if (e) for (int d = 0; d < 3; d++) e[3 * i + d] = E[i][d];
        if (w) w[i] = lat_w(dim, i);
    }
    double Tl[QMAX][QMAX];
    for (int r = 0; r < Q; r++)
        for (int i = 0; i < Q; i++) Tl[r][i] = moment_row(dim, r, E[i]);
    if (T)
        for (int r = 0; r < Q; r++)
            for (int i = 0; i < Q; i++) T[r * Q + i] = Tl[r][i];
    if (Tinv) {
        /* Rows of T are mutually orthogonal, so T^-1 = T^T diag(1/|row|^2). */
        for (int r = 0; r < Q; r++) {
            double nr = 0.0;
            for (int i = 0; i < Q; i++) nr += Tl[r][i] * Tl[r][i];
            for (int i = 0; i < Q; i++) Tinv[i * Q + r] = Tl[r][i] / nr;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Relaxation matrix S (eqs. 4-5, Sec. III A)                          */
/* ------------------------------------------------------------------ */

/* s_nu,k from eq. (5); s_e,k = s_nu,k; s_rho = s_j = 1; s_q both q slots.
 * s_eps: policy 0 takes it from the most viscous phase, shared by both
 * components (Sec. II A and III A); policy 1 keeps s_eps = s_nu,k.
 * D3Q19: s_pi = s_nu,k and s_m = s_q. */
void orc_relaxation(const orc_params *p, int k, double *s)
{
    double snu = 1.0 / (3.0 * p->nu[k] + 0.5);
    double numax = p->nu[0] > p->nu[1] ? p->nu[0] : p->nu[1];
    double seps = p->s_eps_policy == 0 ? 1.0 / (3.0 * numax + 0.5) : snu;
    double se = p->s_eps_policy == 0 ? seps : snu;
    if (p->dim == 2) {
        double S[9] = {1.0, se, seps, 1.0, p->s_q, 1.0, p->s_q, snu, snu};
        memcpy(s, S, sizeof S);
    } else {
        double S[19] = {1.0, se, seps, 1.0, p->s_q, 1.0, p->s_q, 1.0, p->s_q,
                        snu, snu, snu, snu, snu, snu, snu,
                        p->s_q, p->s_q, p->s_q};
        memcpy(s, S, sizeof S);
    }
}

/* ------------------------------------------------------------------ */
/* Equilibrium (eq. 6) and forcing (eq. 9)                             */
/* ------------------------------------------------------------------ */

static const double CS2 = 1.0 / 3.0;

/* eq. (6) with the second-order term read as (e.u)^2 / (2 cs^4): the printed
 * denominator 2 cs^2 does not recover rho from sum_i feq_i. */
void orc_feq(int dim, double rho, const double *u, double *feq)
{
    int Q = orc_Q(dim);
    const int (*E)[3] = lat_e(dim);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; i++) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        feq[i] = rho * lat_w(dim, i) *
                 (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* eq. (9): Fbar_i = w_i [ (e_i - u)/cs^2 + (e_i . u) e_i / cs^4 ] . F */
void orc_forcing(int dim, const double *u, const double *F, double *Fbar)
{
    int Q = orc_Q(dim);
    const int (*E)[3] = lat_e(dim);
    for (int i = 0; i < Q; i++) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double acc = 0.0;
        for (int d = 0; d < 3; d++)
            acc += ((E[i][d] - u[d]) / CS2 + eu * E[i][d] / (CS2 * CS2)) * F[d];
        Fbar[i] = lat_w(dim, i) * acc;
    }
}

/* Dense operators of eq. (1) for a given S: A = T^-1 S T, B = T^-1 (I-S/2) T. */
static void collision_operators(int dim, const double *s, double *A, double *B)
{
    int Q = orc_Q(dim);
    double T[QMAX * QMAX], Ti[QMAX * QMAX];
    orc_tables(dim, NULL, NULL, T, Ti);
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++) {
            double a = 0.0, b = 0.0;
            for (int r = 0; r < Q; r++) {
                a += Ti[i * Q + r] * s[r] * T[r * Q + j];
                b += Ti[i * Q + r] * (1.0 - 0.5 * s[r]) * T[r * Q + j];
            }
            A[i * Q + j] = a;
            B[i * Q + j] = b;
        }
}

static void collide_with(int dim, const double *A, const double *B,
                         const double *f, double rho, const double *u,
                         const double *F, double *fout)
{
    int Q = orc_Q(dim);
    double feq[QMAX], Fb[QMAX];
    orc_feq(dim, rho, u, feq);
    orc_forcing(dim, u, F, Fb);
    for (int i = 0; i < Q; i++) {
        double acc = f[i];
        for (int j = 0; j < Q; j++)
            acc += -A[i * Q + j] * (f[j] - feq[j]) + B[i * Q + j] * Fb[j];
        fout[i] = acc;
    }
}

void orc_collide_node(int dim, const double *s, const double *f, double rho,
                      const double *u, const double *F, double *fout)
{
    double A[QMAX * QMAX], B[QMAX * QMAX];
    collision_operators(dim, s, A, B);
    collide_with(dim, A, B, f, rho, u, F, fout);
}

/* ------------------------------------------------------------------ */
/* Interaction stencil (eqs. 10-11)                                    */
/* ------------------------------------------------------------------ */

/* 8th-order isotropic weights by squared length.  2-D: printed in Sec. II A
 * (w(1)=4/21, w(2)=4/45, w(4)=1/60, w(5)=2/315, w(8)=1/5040) over the 24
 * nonzero offsets of the 5x5 square.  3-D (not given in the paper): the
 * unique positive solution of the same normalisation and isotropy
 * conditions on the shells 1,2,3,4,5,6,8 of the 5x5x5 cube (92 offsets). */
static double stencil_weight(int dim, int r2)
{
    if (dim == 2) {
        switch (r2) {
        case 1: return 4.0 / 21.0;
        case 2: return 4.0 / 45.0;
        case 4: return 1.0 / 60.0;
        case 5: return 2.0 / 315.0;
        case 8: return 1.0 / 5040.0;
        }
        return 0.0;
    }
    switch (r2) {
    case 1: return 4.0 / 45.0;
    case 2: return 1.0 / 21.0;
    case 3: return 2.0 / 105.0;
    case 4: return 5.0 / 504.0;
    case 5: return 1.0 / 315.0;
    case 6: return 1.0 / 630.0;
    case 8: return 1.0 / 5040.0;
    }
    return 0.0;
}

int orc_stencil(int dim, int *off, double *w)
{
    int K = 0;
    int zr = dim == 2 ? 0 : 2;
    for (int dz = -zr; dz <= zr; dz++)
        for (int dy = -2; dy <= 2; dy++)
            for (int dx = -2; dx <= 2; dx++) {
                int r2 = dx * dx + dy * dy + dz * dz;
                double ww = stencil_weight(dim, r2);
                if (r2 == 0 || ww == 0.0) continue;
                if (off) { off[3 * K] = dx; off[3 * K + 1] = dy; off[3 * K + 2] = dz; }
                if (w) w[K] = ww;
                K++;
            }
    return K;
}

/* ------------------------------------------------------------------ */
/* Simulation state                                                    */
/* ------------------------------------------------------------------ */

struct orc_sim {
    orc_params p;
    int Q, K;
    int64_t N;
    int e[QMAX][3];
    int opp[QMAX];
    double w[QMAX];
    int off[KMAX][3];
    double ws[KMAX];
    double A[2][QMAX * QMAX], B[2][QMAX * QMAX];
    uint8_t *solid;      /* [N] */
    int8_t *inlet_of;    /* [N] owning inlet patch or -1 */
    uint8_t *is_outlet;  /* [N] */
    double *f;           /* [2][Q][N] state f(t) */
    double *fn;          /* [2][Q][N] scratch for f(t+1) */
    double *rho;         /* [2][N] */
    double *psi;         /* [2][N] */
    double *F;           /* [2][3][N] */
    double *u;           /* [3][N] common velocity (eqs. 7-8) */
    double *uc;          /* [3][N] velocity used in the collision */
    double *uw;          /* [3][N] wall velocity of solid nodes, or NULL */
    orc_diag diag;
};

#define IDX(s, x, y, z) ((int64_t)(x) + (int64_t)(s)->p.n[0] * ((int64_t)(y) + (int64_t)(s)->p.n[1] * (int64_t)(z)))
#define FI(s, k, i, n) (((int64_t)(k) * (s)->Q + (i)) * (s)->N + (n))

static void coords(const orc_sim *s, int64_t n, int *c)
{
    c[0] = (int)(n % s->p.n[0]);
    c[1] = (int)((n / s->p.n[0]) % s->p.n[1]);
    c[2] = (int)(n / ((int64_t)s->p.n[0] * s->p.n[1]));
}

/* Position used to read psi and the solid flag at x+e: periodic axes wrap;
 * positions beyond a non-periodic face take the value of their mirror image
 * about that face (ghost layers of eqs. 24-25: g1 <- x1, g2 <- x2 at the low
 * face; gN <- xN, g(N-1) <- x(N-1) at the high face). */
static int64_t field_pos(const orc_sim *s, const int *c)
{
    int q[3];
    for (int a = 0; a < 3; a++) {
        int n = s->p.n[a], v = c[a];
        if (v < 0 || v >= n) {
            if (s->p.periodic[a]) v = ((v % n) + n) % n;
            else if (v < 0) v = -1 - v;
            else v = 2 * n - 1 - v;
        }
        q[a] = v;
    }
    return IDX(s, q[0], q[1], q[2]);
}

/* Streaming target x+e_i; returns -1 if the link leaves the box through a
 * non-periodic face (the population is discarded and later supplied by the
 * inlet or outlet treatment). */
static int64_t stream_target(const orc_sim *s, const int *c, const int *e)
{
    int q[3];
    for (int a = 0; a < 3; a++) {
        int n = s->p.n[a], v = c[a] + e[a];
        if (v < 0 || v >= n) {
            if (!s->p.periodic[a]) return -1;
            v = ((v % n) + n) % n;
        }
        q[a] = v;
    }
    return IDX(s, q[0], q[1], q[2]);
}

static void face_normal(int axis, int side, int inward, int *nv)
{
    nv[0] = nv[1] = nv[2] = 0;
    int sgn = side == 0 ? 1 : -1;  /* inward normal of the low face is +e_axis */
    nv[axis] = inward ? sgn : -sgn;
}

static int on_face(const orc_sim *s, const int *c, int axis, int side,
                   const int *lo, const int *hi)
{
    int layer = side == 0 ? 0 : s->p.n[axis] - 1;
    if (c[axis] != layer) return 0;
    for (int a = 0; a < s->p.dim; a++) {
        if (a == axis) continue;
        if (c[a] < lo[a] || c[a] >= hi[a]) return 0;
    }
    return 1;
}

int64_t orc_nodes(const orc_sim *s) { return s->N; }

/* ------------------------------------------------------------------ */
/* Stages 1-3: densities, forces, common velocity                      */
/* ------------------------------------------------------------------ */

static void stage_moments_forces(orc_sim *s)
{
    const int Q = s->Q;
    const int64_t N = s->N;

    /* Stage 1: rho_k = sum_i f_i^k (eq. 8); psi_k = rho_k, zero on solids. */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        for (int k = 0; k < 2; k++) {
            double r = 0.0;
            if (!s->solid[n])
                for (int i = 0; i < Q; i++) r += s->f[FI(s, k, i, n)];
            s->rho[k * N + n] = r;
            s->psi[k * N + n] = s->solid[n] ? 0.0 : r;
        }
    }

    /* Stage 2 and 3. */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        if (s->solid[n]) {
            for (int k = 0; k < 2; k++)
                for (int d = 0; d < 3; d++) s->F[(k * 3 + d) * N + n] = 0.0;
            for (int d = 0; d < 3; d++) s->u[d * N + n] = 0.0;
            continue;
        }
        int c[3];
        coords(s, n, c);
        /* sum_e w(|e|^2) psi_kbar(x+e) e  and  sum_e w(|e|^2) s(x+e) e */
        double gp[2][3] = {{0, 0, 0}, {0, 0, 0}}, gs[3] = {0, 0, 0};
        for (int j = 0; j < s->K; j++) {
            int cc[3] = {c[0] + s->off[j][0], c[1] + s->off[j][1], c[2] + s->off[j][2]};
            int64_t m = field_pos(s, cc);
            for (int d = 0; d < 3; d++) {
                gp[0][d] += s->ws[j] * s->psi[m] * s->off[j][d];
                gp[1][d] += s->ws[j] * s->psi[N + m] * s->off[j][d];
                gs[d] += s->ws[j] * (double)s->solid[m] * s->off[j][d];
            }
        }
        double rtot = s->rho[n] + s->rho[N + n];
        for (int k = 0; k < 2; k++) {
            int kb = 1 - k;
            double psik = s->psi[k * N + n];
            for (int d = 0; d < 3; d++) {
                /* eq. (10), read with the other component's psi at x+e */
                double Ff = -s->p.G12 * psik * gp[kb][d];
                /* eq. (11) with a constant G_w,k */
                double Fa = -s->p.Gw[k] * psik * gs[d];
                double Fbk = (s->rho[k * N + n] / rtot) * s->p.Fb[d];
                s->F[(k * 3 + d) * N + n] = Ff + Fa + Fbk;
            }
        }
        /* eqs. (7)-(8): u = (sum_k sum_i e_i f_i^k + 1/2 sum_k F^k) / sum_k rho_k */
        for (int d = 0; d < 3; d++) {
            double J = 0.0;
            for (int k = 0; k < 2; k++) {
                for (int i = 0; i < Q; i++) J += s->e[i][d] * s->f[FI(s, k, i, n)];
                J += 0.5 * s->F[(k * 3 + d) * N + n];
            }
            s->u[d * N + n] = J / rtot;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Stage 4: outlet velocity correction (eqs. 22-23, App. A)            */
/* ------------------------------------------------------------------ */

static void stage_outlet_velocity(orc_sim *s)
{
    const int64_t N = s->N;
    memcpy(s->uc, s->u, sizeof(double) * 3 * N);
    s->diag.q_in = 0.0;
    s->diag.q_out = 0.0;
    s->diag.chi = 1.0;

    /* Q_in: all inlet nodes, rho u . n_inward (eq. 23 numerator summed over
     * every inlet patch). */
    double qin = 0.0;
    for (int64_t n = 0; n < N; n++) {
        int p = s->inlet_of[n];
        if (p < 0) continue;
        int nv[3];
        face_normal(s->p.inlets[p].axis, s->p.inlets[p].side, 1, nv);
        double un = 0.0;
        for (int d = 0; d < 3; d++) un += s->u[d * N + n] * nv[d];
        qin += (s->rho[n] + s->rho[N + n]) * un;
    }
    s->diag.q_in = qin;
    if (!s->p.has_outlet) return;

    const orc_outlet *o = &s->p.outlet;
    int no[3];
    face_normal(o->axis, o->side, 0, no);
    /* Q': the x_{N-1} column next to every outlet node (eq. 23 denominator). */
    double qout = 0.0;
    for (int64_t n = 0; n < N; n++) {
        if (!s->is_outlet[n]) continue;
        int c[3];
        coords(s, n, c);
        int cp[3] = {c[0] - no[0], c[1] - no[1], c[2] - no[2]};
        int64_t m = IDX(s, cp[0], cp[1], cp[2]);
        if (s->solid[m]) continue;
        double un = 0.0;
        for (int d = 0; d < 3; d++) un += s->u[d * N + m] * no[d];
        qout += (s->rho[m] + s->rho[N + m]) * un;
    }
    s->diag.q_out = qout;
    /* eq. (23); when the x_{N-1} column carries no outflow (or flows against
     * the inlets) the ratio is undefined and the outlet is left uncorrected. */
    double chi = (fabs(qout) < 1e-30 || qin * qout <= 0.0) ? 1.0 : qin / qout;
    if (!o->chi_on) return;
    s->diag.chi = chi;
    /* eq. (22): the normal velocity on the outlet column becomes chi times
     * that of its x_{N-1} neighbour; tangential components are unchanged. */
    for (int64_t n = 0; n < N; n++) {
        if (!s->is_outlet[n]) continue;
        int c[3];
        coords(s, n, c);
        int64_t m = IDX(s, c[0] - no[0], c[1] - no[1], c[2] - no[2]);
        if (s->solid[m]) continue;
        s->uc[o->axis * N + n] = chi * s->u[o->axis * N + m];
    }
}

/* ------------------------------------------------------------------ */
/* Stages 5-6: collision (eq. 1) and streaming (eq. 2, App. B)         */
/* ------------------------------------------------------------------ */

static void stage_collide_stream(orc_sim *s)
{
    const int Q = s->Q;
    const int64_t N = s->N;
    /* populations that no streaming link supplies stay NaN until stages 7/8 */
    for (int64_t j = 0; j < 2 * (int64_t)Q * N; j++) s->fn[j] = NAN;

#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        if (s->solid[n]) continue;
        int c[3];
        coords(s, n, c);
        double u[3] = {s->uc[n], s->uc[N + n], s->uc[2 * N + n]};
        for (int k = 0; k < 2; k++) {
            double f[QMAX], fs[QMAX], F[3];
            for (int i = 0; i < Q; i++) f[i] = s->f[FI(s, k, i, n)];
            for (int d = 0; d < 3; d++) F[d] = s->F[(k * 3 + d) * N + n];
            collide_with(s->p.dim, s->A[k], s->B[k], f, s->rho[k * N + n], u, F, fs);
            for (int i = 0; i < Q; i++) {
                int64_t m = stream_target(s, c, s->e[i]);
                if (m < 0) continue;                    /* leaves through an open face */
                if (s->solid[m]) {
                    /* eq. (B1); a moving wall adds -2 w_i rho_k (e_i . u_w) / cs^2 */
                    double mw = 0.0;
                    if (s->uw)
                        for (int d = 0; d < 3; d++) mw += s->e[i][d] * s->uw[d * N + m];
                    s->fn[FI(s, k, s->opp[i], n)] = fs[i] - 2.0 * s->w[i] * s->rho[k * N + n] * mw / CS2;
                } else {
                    s->fn[FI(s, k, i, m)] = fs[i];      /* eq. (2) */
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Stage 7: corrected non-equilibrium extrapolation inlet              */
/* ------------------------------------------------------------------ */

static void stage_inlet(orc_sim *s)
{
    const int Q = s->Q;
    const int64_t N = s->N;
    const int dim = s->p.dim;
    for (int64_t n = 0; n < N; n++) {
        int p = s->inlet_of[n];
        if (p < 0) continue;
        const orc_inlet *in = &s->p.inlets[p];
        int nv[3], c[3];
        face_normal(in->axis, in->side, 1, nv);
        coords(s, n, c);
        int64_t m = IDX(s, c[0] + nv[0], c[1] + nv[1], c[2] + nv[2]);   /* x2 */
        double up[3] = {in->u_n * nv[0], in->u_n * nv[1], in->u_n * nv[2]};

        /* rho_k(x2) and u(x2) from the streamed f at t+1 with this step's
         * force (the force at t+1 does not exist yet). */
        double r2[2] = {0, 0}, u2[3] = {0, 0, 0};
        int x2_fluid = !s->solid[m];
        if (x2_fluid) {
            for (int k = 0; k < 2; k++)
                for (int i = 0; i < Q; i++) r2[k] += s->fn[FI(s, k, i, m)];
            for (int d = 0; d < 3; d++) {
                double J = 0.0;
                for (int k = 0; k < 2; k++) {
                    for (int i = 0; i < Q; i++) J += s->e[i][d] * s->fn[FI(s, k, i, m)];
                    J += 0.5 * s->F[(k * 3 + d) * N + m];
                }
                u2[d] = J / (r2[0] + r2[1]);
            }
        }
        for (int k = 0; k < 2; k++) {
            double feq_p[QMAX], feq_2[QMAX];
            orc_feq(dim, in->rho[k], up, feq_p);
            orc_feq(dim, r2[k], u2, feq_2);
            /* eq. (13)/(14) for the populations entering the domain */
            for (int i = 0; i < Q; i++) {
                int ein = s->e[i][0] * nv[0] + s->e[i][1] * nv[1] + s->e[i][2] * nv[2];
                if (ein <= 0) continue;
                double neq = x2_fluid ? s->fn[FI(s, k, i, m)] - feq_2[i] : 0.0;
                s->fn[FI(s, k, i, n)] = feq_p[i] + neq;
            }
            if (!in->alpha_on) continue;
            /* eqs. (15)-(19), read as a momentum correction: the entering
             * populations are shifted by alpha_i = w_i sum_d e_id dJ_d / D_d,
             * D_d = sum_{j entering} w_j e_jd^2, with
             * dJ = rho_k^p u^p - (sum_i e_i f_i(x1) + F^k(x1)/2). */
            double dJ[3], D[3] = {0, 0, 0};
            for (int d = 0; d < 3; d++) {
                double J = 0.0;
                for (int i = 0; i < Q; i++) J += s->e[i][d] * s->fn[FI(s, k, i, n)];
                J += 0.5 * s->F[(k * 3 + d) * N + n];
                dJ[d] = in->rho[k] * up[d] - J;
            }
            for (int i = 0; i < Q; i++) {
                int ein = s->e[i][0] * nv[0] + s->e[i][1] * nv[1] + s->e[i][2] * nv[2];
                if (ein <= 0) continue;
                for (int d = 0; d < 3; d++) D[d] += s->w[i] * s->e[i][d] * s->e[i][d];
            }
            for (int i = 0; i < Q; i++) {
                int ein = s->e[i][0] * nv[0] + s->e[i][1] * nv[1] + s->e[i][2] * nv[2];
                if (ein <= 0) continue;
                double a = 0.0;
                for (int d = 0; d < dim; d++)
                    if (D[d] > 0.0) a += s->w[i] * s->e[i][d] * dJ[d] / D[d];
                s->fn[FI(s, k, i, n)] += a;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Stage 8: convective outflow (eqs. 20-21)                            */
/* ------------------------------------------------------------------ */

static void stage_outlet_fill(orc_sim *s)
{
    const int Q = s->Q;
    const int64_t N = s->N;
    s->diag.u_conv = 0.0;
    if (!s->p.has_outlet) return;
    const orc_outlet *o = &s->p.outlet;
    int no[3];
    face_normal(o->axis, o->side, 0, no);

    /* eq. (21): mean normal velocity over the fluid x_{N-1} column, from the
     * streamed f at t+1 with this step's force. */
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t n = 0; n < N; n++) {
        if (!s->is_outlet[n]) continue;
        int c[3];
        coords(s, n, c);
        int64_t m = IDX(s, c[0] - no[0], c[1] - no[1], c[2] - no[2]);
        if (s->solid[m]) continue;
        double r = 0.0, J = 0.0;
        for (int k = 0; k < 2; k++) {
            for (int i = 0; i < Q; i++) {
                double fv = s->fn[FI(s, k, i, m)];
                r += fv;
                J += (s->e[i][0] * no[0] + s->e[i][1] * no[1] + s->e[i][2] * no[2]) * fv;
            }
            for (int d = 0; d < 3; d++) J += 0.5 * s->F[(k * 3 + d) * N + m] * no[d];
        }
        sum += J / r;
        cnt++;
    }
    double Uc = cnt ? sum / (double)cnt : 0.0;
    /* U_c < 0 would make eq. (20) singular at U_c = -1; it is clamped. */
    if (Uc < 0.0) { Uc = 0.0; s->diag.uc_clamps++; }
    s->diag.u_conv = Uc;

    /* eq. (20) for the populations entering through the outlet face. */
    for (int64_t n = 0; n < N; n++) {
        if (!s->is_outlet[n]) continue;
        int c[3];
        coords(s, n, c);
        int64_t m = IDX(s, c[0] - no[0], c[1] - no[1], c[2] - no[2]);
        for (int k = 0; k < 2; k++)
            for (int i = 0; i < Q; i++) {
                int eo = s->e[i][0] * no[0] + s->e[i][1] * no[1] + s->e[i][2] * no[2];
                if (eo >= 0) continue;
                double prev = s->f[FI(s, k, i, n)];    /* f_i(x_N, t) */
                double val = s->solid[m] ? prev
                                         : (prev + Uc * s->fn[FI(s, k, i, m)]) / (1.0 + Uc);
                s->fn[FI(s, k, i, n)] = val;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Public driver                                                       */
/* ------------------------------------------------------------------ */

static void total_mass(const orc_sim *s, double *mass)
{
    const int Q = s->Q;
    const int64_t N = s->N;
    for (int k = 0; k < 2; k++) {
        double acc = 0.0;
        for (int64_t n = 0; n < N; n++) {
            if (s->solid[n]) continue;
            for (int i = 0; i < Q; i++) acc += s->f[FI(s, k, i, n)];
        }
        mass[k] = acc;
    }
}

orc_sim *orc_create(const orc_params *p, const uint8_t *solid,
                    const double *rho0, const double *u0)
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    if (s->p.dim == 2) s->p.n[2] = 1;
    s->Q = orc_Q(p->dim);
    s->N = (int64_t)s->p.n[0] * s->p.n[1] * s->p.n[2];
    const int Q = s->Q;
    const int64_t N = s->N;
    const int (*E)[3] = lat_e(p->dim);
    for (int i = 0; i < Q; i++) {
        for (int d = 0; d < 3; d++) s->e[i][d] = E[i][d];
        s->w[i] = lat_w(p->dim, i);
    }
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++)
            if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2]) s->opp[i] = j;
    {
        int off[KMAX * 3];
        double w[KMAX];
        s->K = orc_stencil(p->dim, off, w);
        for (int j = 0; j < s->K; j++) {
            for (int d = 0; d < 3; d++) s->off[j][d] = off[3 * j + d];
            s->ws[j] = w[j];
        }
    }
    for (int k = 0; k < 2; k++) {
        double sk[QMAX];
        orc_relaxation(&s->p, k, sk);
        collision_operators(p->dim, sk, s->A[k], s->B[k]);
    }
    s->solid = (uint8_t *)malloc(N);
    memcpy(s->solid, solid, N);
    s->inlet_of = (int8_t *)malloc(N);
    s->is_outlet = (uint8_t *)calloc(N, 1);
    for (int64_t n = 0; n < N; n++) {
        s->inlet_of[n] = -1;
        if (s->solid[n]) continue;
        int c[3];
        coords(s, n, c);
        for (int q = 0; q < p->n_inlets; q++)
            if (on_face(s, c, p->inlets[q].axis, p->inlets[q].side, p->inlets[q].lo, p->inlets[q].hi))
                s->inlet_of[n] = (int8_t)q;
        if (p->has_outlet &&
            on_face(s, c, p->outlet.axis, p->outlet.side, p->outlet.lo, p->outlet.hi))
            s->is_outlet[n] = 1;
    }
    s->f = (double *)calloc(2 * (size_t)Q * N, sizeof(double));
    s->fn = (double *)calloc(2 * (size_t)Q * N, sizeof(double));
    s->rho = (double *)calloc(2 * (size_t)N, sizeof(double));
    s->psi = (double *)calloc(2 * (size_t)N, sizeof(double));
    s->F = (double *)calloc(6 * (size_t)N, sizeof(double));
    s->u = (double *)calloc(3 * (size_t)N, sizeof(double));
    s->uc = (double *)calloc(3 * (size_t)N, sizeof(double));
    /* initial state f = feq(rho_k, u0) */
    for (int64_t n = 0; n < N; n++) {
        if (s->solid[n]) continue;
        double u[3] = {0, 0, 0};
        if (u0) for (int d = 0; d < 3; d++) u[d] = u0[d * N + n];
        for (int k = 0; k < 2; k++) {
            double feq[QMAX];
            orc_feq(p->dim, rho0[k * N + n], u, feq);
            for (int i = 0; i < Q; i++) s->f[FI(s, k, i, n)] = feq[i];
        }
    }
    s->diag.chi = 1.0;
    total_mass(s, s->diag.mass0);
    total_mass(s, s->diag.mass);
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->solid); free(s->inlet_of); free(s->is_outlet);
    free(s->f); free(s->fn); free(s->rho); free(s->psi);
    free(s->F); free(s->u); free(s->uc); free(s->uw);
    free(s);
}

void orc_step(orc_sim *s, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; t++) {
        stage_moments_forces(s);      /* stages 1-3 */
        stage_outlet_velocity(s);     /* stage 4 */
        stage_collide_stream(s);      /* stages 5-6 */
        stage_inlet(s);               /* stage 7 */
        stage_outlet_fill(s);         /* stage 8 */
        double *tmp = s->f; s->f = s->fn; s->fn = tmp;
        s->diag.step++;
    }
    total_mass(s, s->diag.mass);
}

void orc_get_f(const orc_sim *s, double *f)
{
    memcpy(f, s->f, sizeof(double) * 2 * (size_t)s->Q * s->N);
}

void orc_set_f(orc_sim *s, const double *f)
{
    memcpy(s->f, f, sizeof(double) * 2 * (size_t)s->Q * s->N);
    total_mass(s, s->diag.mass);
}

void orc_moments(orc_sim *s, double *rho, double *u, double *F)
{
    stage_moments_forces(s);
    const int64_t N = s->N;
    if (rho) memcpy(rho, s->rho, sizeof(double) * 2 * N);
    if (u) memcpy(u, s->u, sizeof(double) * 3 * N);
    if (F) memcpy(F, s->F, sizeof(double) * 6 * N);
}

void orc_diagnostics(orc_sim *s, orc_diag *d) { *d = s->diag; }

void orc_set_wall_velocity(orc_sim *s, const double *uw)
{
    free(s->uw);
    s->uw = NULL;
    if (!uw) return;
    s->uw = (double *)malloc(sizeof(double) * 3 * (size_t)s->N);
    memcpy(s->uw, uw, sizeof(double) * 3 * (size_t)s->N);
}

void orc_set_next(orc_sim *s, const double *fn)
{
    memcpy(s->fn, fn, sizeof(double) * 2 * (size_t)s->Q * s->N);
}

void orc_get_next(const orc_sim *s, double *fn)
{
    memcpy(fn, s->fn, sizeof(double) * 2 * (size_t)s->Q * s->N);
}

void orc_set_force(orc_sim *s, const double *F)
{
    memcpy(s->F, F, sizeof(double) * 6 * (size_t)s->N);
}

void orc_stage(orc_sim *s, int stage)
{
    switch (stage) {
    case 1: stage_moments_forces(s); break;
    case 4: stage_outlet_velocity(s); break;
    case 5: stage_collide_stream(s); break;
    case 7: stage_inlet(s); break;
    case 8: stage_outlet_fill(s); break;
    default: break;
    }
}
