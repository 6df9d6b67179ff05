/*
 * lbm.h -- C ABI of the MI355X (gfx950) two-component immiscible
 * pseudopotential MRT lattice Boltzmann solver with corrected open boundaries
 * (Chen, Pan, Wang, Li & Chen, arXiv:2512.12934).
 *
 * One call of lbm_step advances the lattice by whole time steps of the method
 * of Sec. II: densities and pseudopotentials (eq. 8; psi_k = rho_k) with
 * mirror ghost layers at open faces (eqs. 24-25), the fluid-fluid force of
 * eq. (10) with the 8th-order weights of Sec. II A and the wall adhesion of
 * eq. (11), the common velocity (eqs. 7-8), the outlet velocity correction
 * from the inlet/outlet mass-flow ratio (eqs. 22-23, App. A), the MRT
 * collision with forcing (eqs. 1, 3-6, 9) with s_e and s_eps taken from the
 * most viscous phase (Sec. III A), streaming with halfway bounce-back and
 * periodic wrap (eq. 2, App. B), the alpha-corrected non-equilibrium
 * extrapolation inlet (eqs. 13-19) and the convective outflow (eqs. 20-21).
 *
 * Conventions shared by every entry point
 *   - All calls return lbm_status; nothing throws across the ABI.
 *   - Node index n = x + n[0]*(y + n[1]*z) over the box; 2-D uses n[2] = 1.
 *   - Component k in {0, 1} is the paper's component k+1.
 *   - Populations: D2Q9 order 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1);
 *     5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1)  (the unknown sets of Sec. II B).
 *     D3Q19 order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),
 *     (-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
 *     (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *   - The state of a context is the post-streaming, post-boundary
 *     distribution f(t); lbm_get_state/lbm_set_state exchange it as
 *     double f[2][Q][N] (solid nodes ignored on input, zero on output).
 *   - Lattice units throughout.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,     /* invalid argument or configuration; nothing changed   */
    LBM_ENOMEM = 2,     /* workspace too small or device allocation failed      */
    LBM_EDEVICE = 3,    /* a HIP runtime call failed (message in lbm_last_error) */
    LBM_EUNSTABLE = 4,  /* a non-finite or non-positive density was produced    */
    LBM_ESTATE = 5      /* the context was already flagged unstable             */
} lbm_status;

/* Storage of the populations between steps (all arithmetic is FP32):
 *   LBM_STORE_F32         f_i - w_i in FP32;
 *   LBM_STORE_F16_OFFSET  f_i - w_i r in binary16 (round to nearest even),
 *                         r the previous step's density of the component at
 *                         the node that reads the value (its reference
 *                         density), so the stored numbers stay small in both
 *                         phases;
 *   LBM_STORE_F16_FIXED   f_i - w_i in binary16: the fixed offset of the
 *                         precision extension as stated, kept to report its
 *                         error beside the reference-density form. */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16_OFFSET = 1, LBM_STORE_F16_FIXED = 2 };
enum { LBM_SEPS_MAXVISC = 0, LBM_SEPS_FIXED = 1 };
#define LBM_MAX_INLETS 8

/* Inlet patch (eqs. 13-19): the fluid nodes of the face layer (axis, side)
 * whose two tangential coordinates lie in [lo, hi) (the normal coordinate of
 * lo/hi is ignored).  side 0 is coordinate 0, side 1 is n[axis]-1.  Later
 * patches take precedence where rectangles overlap.  rho[k] and the speed
 * u_n along the inward normal are the prescribed inlet quantities. */
typedef struct {
    int axis, side;
    int lo[3], hi[3];
    double rho[2];
    double u_n;
    int alpha_on;       /* 1: eqs. (15)-(19) correction; 0: eq. (13)/(14) only */
} lbm_inlet;

/* Outlet (eqs. 20-23): fluid nodes of the face layer (axis, side) in [lo, hi). */
typedef struct {
    int axis, side;
    int lo[3], hi[3];
    int chi_on;         /* 1: mass-flow velocity correction of eqs. (22)-(23) */
} lbm_outlet;

/* Problem description.  Every array is host memory owned by the caller and
 * copied by lbm_create. */
enum { LBM_LAYOUT_CALLER = 0, LBM_LAYOUT_FACE_LAST = 1 };

typedef struct {
    int dim;                 /* 2: D2Q9, 3: D3Q19 */
    int storage;             /* LBM_STORE_F32, LBM_STORE_F16_OFFSET or LBM_STORE_F16_FIXED */
    int n[3];                /* box size; n[2] = 1 in 2-D; non-periodic axes need n >= 3 */
    int periodic[3];
    double nu[2];            /* kinematic viscosities, eq. (5); > 0 */
    double s_q;              /* energy-flux relaxation rate, in (0, 2) */
    int s_eps_policy;        /* LBM_SEPS_MAXVISC (paper) or LBM_SEPS_FIXED */
    double G12;              /* eq. (10) */
    double Gw[2];            /* eq. (11), constant per component */
    double Fb[3];            /* body-force density, shared as (rho_k/rho) Fb */
    int n_inlets;
    lbm_inlet inlets[LBM_MAX_INLETS];
    int has_outlet;
    lbm_outlet outlet;
    int tile_config;         /* node-update configuration, -1 = library default
                                (an index into the tuning space; the autotuner
                                measures them) */
    int layout;              /* LBM_LAYOUT_CALLER: memory axes are the caller's;
                                LBM_LAYOUT_FACE_LAST (3-D): the axis normal to the
                                open faces is stored last, so face nodes are
                                contiguous (faster face kernels, slower node
                                update on the 600x120x120 device).  Outputs are
                                in the caller's frame either way. */
    const uint8_t *solid;    /* [N], 1 = solid; every fluid node on a
                                non-periodic face must belong to a patch */
    const double *rho0;      /* [2][N] initial component densities (> 0 on fluid) */
    const double *u0;        /* [3][N] initial velocity, or NULL for rest */
    const double *wall_u;    /* [3][N] velocity of every solid node (moving
                                walls, read on solid nodes only), or NULL for
                                resting walls.  A population bounced back from
                                a moving solid node s at the fluid node x
                                gains -2 w_i rho_k(x) (e_i . u_w(s)) / cs^2
                                (halfway bounce-back with a moving wall, as
                                the sheared plates of the Taylor deformation
                                test of Sec. III A need).  Not supported next
                                to the outlet column (LBM_EINVAL). */
} lbm_config;

/* FP64 diagnostics of the most recent step (device-side reductions). */
typedef struct {
    int64_t step;
    double q_in;     /* sum over inlet nodes of rho u . n_inward      (eq. 23 numerator)   */
    double q_out;    /* sum over the x_{N-1} column of rho u . n_out  (eq. 23 denominator) */
                     /* (both summed exactly with every term on a grid of 2^-40, so they do
                      * not depend on the launch shape; |q| < 2^23) */
    double chi;      /* eq. (23) coefficient applied (1 if uncorrected or undefined) */
    double u_conv;   /* eq. (21) convective velocity after the clamp at 0 */
    double mass[2];  /* current total mass of each component over fluid nodes */
    double mass0[2]; /* total mass at creation */
    int64_t uc_clamps;
} lbm_flux;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace lbm_create needs for cfg; 0 if cfg is invalid. */
size_t lbm_workspace_bytes(const lbm_config *cfg);

/* Validates cfg, carves the caller-owned device buffer dev_ws (ws_bytes long,
 * 256-byte aligned, it must outlive the context), uploads the static node
 * maps and initialises f = feq(rho0, u0) on hip_stream (a hipStream_t owned
 * by the caller; NULL = default stream).  Returns LBM_EINVAL for an invalid
 * configuration, LBM_ENOMEM when ws_bytes is too small, LBM_EDEVICE on a HIP
 * error.  On success *out receives the context. */
lbm_status lbm_create(const lbm_config *cfg, void *dev_ws, size_t ws_bytes,
                      void *hip_stream, lbm_ctx **out);

/* Enqueues n >= 0 time steps on the context stream and returns without
 * waiting.  Errors raised on the device surface at the next synchronising
 * call.  LBM_ESTATE if the context was already flagged unstable.  Whole
 * groups of lbm_set_graph_steps() steps are replayed from a HIP graph
 * (captured on a private stream the first time, launched on the context
 * stream); the remainder, and every step enqueued while the context stream is
 * itself being captured by the caller, are launched one kernel at a time.
 * Both routes run the same kernels on the same data.  Under the caller's
 * capture n must be even (LBM_EINVAL otherwise): the two population arrays
 * swap every step, and an even count leaves them where every replay of the
 * caller's graph expects them; the replays advance the device state, while
 * lbm_steps_done counts the steps enqueued at capture once. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Steps per replayed graph (0 = never use graphs; default 16; at most 4096).
 * Drops graphs captured so far, then captures, instantiates and uploads the
 * graphs of both A/B parities at once, so that later lbm_step calls replay
 * them without a capture (set-up work, not to be called inside the caller's
 * own capture).  LBM_EINVAL for a value out of range, LBM_EDEVICE if a
 * capture fails. */
lbm_status lbm_set_graph_steps(lbm_ctx *ctx, int steps_per_graph);

/* Synchronises the stream and writes rho [2][N] and the common velocity
 * u [3][N] of eqs. (7)-(8) (half-force included, before any outlet
 * override) of the current state; solid nodes get 0.  Buffers are caller
 * owned, device memory if dst_on_device != 0, else host memory.  Returns
 * LBM_EUNSTABLE if the instability flag is set (the fields are still
 * written). */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *u, int dst_on_device);

/* Synchronises and fills *out (host) with the FP64 diagnostics. */
lbm_status lbm_mass_flux(lbm_ctx *ctx, lbm_flux *out);

/* Checkpoint of the current state as host double f[2][Q][N] (bytes must be
 * 16*Q*N).  lbm_set_state replaces the state (used for restarts and to plant
 * values from the host); it also clears the instability flag. */
lbm_status lbm_get_state(lbm_ctx *ctx, double *f_host, size_t bytes);
lbm_status lbm_set_state(lbm_ctx *ctx, const double *f_host, size_t bytes);

/* Measurement hook: enqueues n steps like lbm_step, bracketing every kernel
 * launch with HIP events on the context stream, then synchronises and writes
 * the mean duration in milliseconds of each launch kind into ms[5]:
 * [0] the node update, [1] the first face launch (chi of eq. 23, the outlet
 * collision and, unless one of them streams from the outlet column, the inlet
 * nodes), [2] the inlet nodes left over and the partial sums of eq. (21),
 * [3] the outlet fill, [4] the density pass that precedes the node update in
 * the two-pass mode (0 where a kind is not launched). */
lbm_status lbm_time_kernels(lbm_ctx *ctx, int64_t n, double *ms);

/* Number of node-update configurations of the tuning space for dim (2 or 3),
 * valid values of lbm_config.tile_config being -1 .. count-1; 0 for any other
 * dim.  Every configuration computes the same arithmetic per node. */
int lbm_tile_configs(int dim);

/* Describes configuration i of dim in out[6] (caller-owned): the density
 * source (0: recomputed inside the node update, 1: a density pass before it),
 * the lateral tile (x, then y; y is 1 in 2-D), the sweep planes per
 * iteration, the sweep planes per work item and whether both components stay
 * in registers.  Returns LBM_EINVAL for an unknown dim or index. */
lbm_status lbm_tile_config_desc(int dim, int i, int *out);

/* Number of steps taken; the stream is not synchronised. */
int64_t lbm_steps_done(const lbm_ctx *ctx);

/* Releases the context (not the caller's workspace).  NULL is ignored. */
void lbm_destroy(lbm_ctx *ctx);

/* Last error message of ctx (or of the last failed lbm_create if ctx is NULL). */
const char *lbm_last_error(const lbm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent contexts advanced together, one launch per stage
 * of the step for all members (the node update as one persistent launch over
 * the members' concatenated work items), with the step loop replayed from a
 * HIP graph.  Members share dim and storage; the node-update configuration
 * is cfgs[0].tile_config for every member.  They differ in everything else
 * (size, geometry, viscosities, forces, faces).  Each member computes exactly
 * what its own context would compute with lbm_step (same kernels, same
 * arithmetic, bitwise identical results).
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Device workspace bytes for the n members cfgs[0..n); 0 if any is invalid
 * or the members do not share dim and storage. */
size_t lbm_batch_workspace_bytes(const lbm_config *cfgs, int n);

/* Creates every member (as lbm_create would, inside the one caller-owned
 * workspace: 256-byte aligned, ws_bytes long, outliving the batch) and the
 * device tables of the batched launches.  Same status codes as lbm_create;
 * the message names the failing member. */
lbm_status lbm_batch_create(const lbm_config *cfgs, int n, void *dev_ws, size_t ws_bytes,
                            void *hip_stream, lbm_batch **out);

/* Enqueues n steps of every member on the batch stream without waiting.
 * LBM_ESTATE if a member is flagged unstable or was stepped on its own since
 * the last batch step (its A/B parity differs from the batch's).  Under a
 * capture of the batch stream by the caller, n must be even (as for
 * lbm_step). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);

/* Steps per replayed graph for lbm_batch_step (0 = plain launches; default
 * 16).  As lbm_set_graph_steps: both parities are captured and uploaded at
 * once. */
lbm_status lbm_batch_set_graph_steps(lbm_batch *b, int steps_per_graph);

/* Number of members; 0 for NULL. */
int lbm_batch_size(const lbm_batch *b);

/* Member i as a context, for lbm_moments, lbm_mass_flux, lbm_get_state and
 * lbm_set_state (owned by the batch: do not destroy it).  NULL if i is out of
 * range. */
lbm_ctx *lbm_batch_member(lbm_batch *b, int i);

/* Releases the batch and its members (not the workspace).  NULL is ignored. */
void lbm_batch_destroy(lbm_batch *b);

/* Last error of b (or of the last failed lbm_batch_create if b is NULL). */
const char *lbm_batch_last_error(const lbm_batch *b);

/* ------------------------------------------------------------------------
 * Droplet labels (droplet size and generation period, Sec. III D).  The
 * dispersed phase is the set of fluid nodes inside a box whose component-k
 * density, summed from the current populations in FP32, exceeds threshold.
 * ------------------------------------------------------------------------ */

/* An axis-aligned box of nodes [lo, hi) in the caller's frame (2-D: lo[2] = 0,
 * hi[2] = 1). */
typedef struct {
    int lo[3], hi[3];
} lbm_box;

/* One face-connected component (4-neighbour in 2-D, 6-neighbour in 3-D). */
typedef struct {
    int64_t first;   /* smallest node index (x fastest) of the component */
    int64_t size;    /* nodes: the area (2-D) or volume (3-D) of the droplet */
    int lo[3], hi[3];/* bounding box [lo, hi) */
} lbm_component;

/* Enqueues on the context stream (no synchronisation, graph-capturable) the
 * count of dispersed nodes of component k in box into *dev_count (an int64 in
 * device memory owned by the caller, overwritten).  A thin box across a
 * channel gives a time series whose rising edges are droplet passages.
 * LBM_EINVAL for k not in {0, 1} or a box outside the domain. */
lbm_status lbm_probe(lbm_ctx *ctx, int k, const lbm_box *box, double threshold, int64_t *dev_count);

/* Synchronises and labels the face-connected components of the dispersed
 * phase of component k in box.  *n_out receives their number; the first
 * min(n, max_out) of them, ordered by their smallest node index, are written
 * to out (host memory, caller owned).  Allocates and frees its own device
 * scratch (4 bytes x 2 per node); not for use inside a graph capture. */
lbm_status lbm_components(lbm_ctx *ctx, int k, const lbm_box *box, double threshold,
                          lbm_component *out, int max_out, int *n_out);

/* Allocation-free variant of lbm_components, for callers that cannot
 * allocate device memory (tight serving or analysis loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and ordering as
 * lbm_components; its device scratch is a fixed array inside the library
 * (about 32.2 MiB per device, held by every device the library runs on
 * until the process ends), so it allocates and frees nothing.  Limits: the
 * context's domain may hold at most LBM_COMPONENTS_STATIC_MAX_NODES nodes
 * and the phase at most LBM_COMPONENTS_STATIC_MAX_COMPONENTS components;
 * beyond either it returns LBM_EINVAL with the reason in lbm_last_error
 * (the second check comes after the labelling, and *n_out is then left
 * unchanged).  The context's device must be the current device.  It
 * synchronises the context stream, so it cannot be captured into a graph.
 * Every call on one device shares that device's scratch: calls that overlap
 * on one device (two host threads, or different streams) race and must be
 * serialised by the caller. */
#define LBM_COMPONENTS_STATIC_MAX_NODES (1 << 22)
#define LBM_COMPONENTS_STATIC_MAX_COMPONENTS 4096
lbm_status lbm_components_static(lbm_ctx *ctx, int k, const lbm_box *box, double threshold,
                                 lbm_component *out, int max_out, int *n_out);

/* ------------------------------------------------------------------------
 * Surrogate: an ensemble of MLPs 4 -> hidden -> hidden -> 2 (tanh) that maps
 * the parameters of a channel run to its droplet labels.  Training (full
 * batch, mean squared error, Adam) runs in FP32 on the GPU with hand-written
 * forward and backward kernels; inference uses BF16 matrix cores with FP32
 * accumulation.  A query whose members disagree (standard deviation above
 * threshold x |mean| for an output) is flagged for the lattice Boltzmann
 * solver.  X [n][4], Y [n][2], mean/std [n][2] and fallback [n] are device
 * memory owned by the caller; every call only enqueues work on the context
 * stream unless stated.
 * ------------------------------------------------------------------------ */
typedef struct surr_ctx surr_ctx;

/* Device workspace bytes for members (1..64) of width hidden (128) trained on
 * up to max_n samples; 0 if the arguments are invalid. */
size_t surr_workspace_bytes(int members, int hidden, int max_n);

/* Parameters per member (17410 for hidden = 128; 0 for another width). */
int surr_param_count(int hidden);

/* Initialises every member from seed (counter-based, so the same seed gives
 * the same weights) and synchronises.  LBM_EINVAL / LBM_ENOMEM / LBM_EDEVICE
 * as lbm_create. */
lbm_status surr_create(int members, int hidden, int max_n, uint64_t seed, void *dev_ws, size_t ws_bytes,
                       void *hip_stream, surr_ctx **out);

/* epochs full-batch Adam steps (learning rate lr) on n <= max_n samples.  If
 * loss_host is not NULL it synchronises and receives each member's loss
 * before the last update. */
lbm_status surr_train(surr_ctx *ctx, const float *X, const float *Y, int n, int epochs, float lr,
                      float *loss_host);

/* Test hook: the gradient of the loss with respect to every parameter,
 * grads [members][P] (device), and the loss per member (device, or NULL),
 * without updating anything. */
lbm_status surr_forward_backward(surr_ctx *ctx, const float *X, const float *Y, int n, float *grads,
                                 float *loss);

/* Ensemble prediction of n queries (X, mean, std, fallback on the device).
 * Each member's outputs are first mapped to the caller's units,
 * y * out_scale[o] + out_shift[o] (host float[2] each; NULL = 1 and 0), so a
 * network trained on normalised targets reports physical values.  In those
 * units: mean [n][2] and (population) standard deviation [n][2] over the
 * members, and fallback[i] = 1 where some output has std > threshold * |mean|
 * (the query goes back to the lattice Boltzmann solver).  Asynchronous on the
 * context stream.  LBM_EINVAL for bad sizes, a negative threshold or a
 * non-finite scale or shift. */
lbm_status surr_predict(surr_ctx *ctx, const float *X, int n, float *mean, float *std, uint8_t *fallback,
                        float threshold, const float *out_scale, const float *out_shift);

/* Copy every member's parameters (host float [members][P], bytes exact) out
 * or in; both synchronise. */
lbm_status surr_get_params(surr_ctx *ctx, float *host, size_t bytes);
lbm_status surr_set_params(surr_ctx *ctx, const float *host, size_t bytes);

/* Releases the context (not the workspace); NULL is ignored. */
void surr_destroy(surr_ctx *ctx);

/* Last error of ctx (or of the last failed surr_create if ctx is NULL). */
const char *surr_last_error(const surr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
