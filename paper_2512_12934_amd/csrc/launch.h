// launch.h -- host-side launchers of the step kernels.  Each lattice has its
// own translation unit (k2d.hip, k3d.hip) that instantiates Launcher<DIM>;
// the runtime (lbm_api.hip) sees only these declarations.
#pragma once

#include <hip/hip_runtime.h>

#include "params.h"

namespace lbm {

// One configuration of the node update: where psi comes from (1 = the psi
// array written by k_psi, 0 = recomputed in k_main), the lateral tile
// (tx, or tx x ty in 3-D), the planes per sweep iteration w, the planes per
// block zc, and whether both components stay in registers (keepb).
struct TileCfg {
    int psrc, tx, ty, w, zc, keepb;
};

// The tuning space.  Entry 0 is the default when no measured choice exists.
constexpr TileCfg CFG2[] = {
    {1, 64, 1, 4, 16, 1},
    {1, 64, 1, 4, 32, 1},
    {1, 128, 1, 2, 16, 1},
    {1, 256, 1, 1, 16, 1},
    {0, 64, 1, 4, 16, 1},
    {1, 64, 1, 8, 16, 1},
    {1, 64, 1, 16, 32, 1},
    {1, 32, 1, 16, 32, 1},
    // shallow chunks: four times the work items, for small domains whose
    // deeper items would leave most CUs idle
    {1, 32, 1, 8, 8, 1},
    {1, 64, 1, 4, 8, 1},
    {0, 32, 1, 8, 8, 1},
};
constexpr TileCfg CFG3[] = {
    {1, 32, 8, 4, 16, 1},
    {1, 32, 8, 4, 16, 0},
    {1, 32, 8, 2, 16, 1},
    {1, 64, 4, 4, 16, 1},
    {1, 32, 8, 4, 32, 1},
    {1, 32, 8, 8, 16, 1},
    {0, 32, 8, 4, 16, 1},
    // shallow chunks: four (eight) times the work items of the 16-plane
    // shapes, so the last wave of blocks leaves fewer CUs idle (the picks for
    // the co-flow device at full and at quarter scale)
    {1, 32, 8, 4, 4, 1},
    {1, 64, 4, 4, 4, 1},
    {1, 32, 8, 2, 2, 1},
};
constexpr int NCFG2 = sizeof(CFG2) / sizeof(CFG2[0]);
constexpr int NCFG3 = sizeof(CFG3) / sizeof(CFG3[0]);

inline const TileCfg &tile_cfg(int dim, int i) { return dim == 2 ? CFG2[i] : CFG3[i]; }
inline int n_tile_cfg(int dim) { return dim == 2 ? NCFG2 : NCFG3; }

struct StepArgs {
    const void *src;
    void *dst;
    const uint32_t *type;
    float2 *psi;        // psi(t) (written by k_psi, or by the fused node update)
    const float2 *ref;  // reference densities of the stored state (psi(t-1))
    Geometry g;
    Physics ph;
    Boundary bd;
    int tiles_x, tiles_y, items;
    const int *item_list;
    unsigned grid;
    double *orho, *ou;
    int *flag;
    unsigned long long *qacc;   // eq. (23) sums of this step (Boundary::qacc at the step's parity)
    unsigned long long *qnext;  // those of the other parity, cleared by the first face launch
    hipStream_t stream;
};

// One step of a whole batch: launch sizes of each stage (0 = skip).
struct BatchArgs {
    BatchTab t;
    int cur;
    unsigned g_psi, g_main, g_chi, g_out, g_inl, g_fill;
    hipStream_t stream;
};

template <int DIM> struct Launcher {
    static void psi(int storage, const StepArgs &a);
    static void moments(int storage, const StepArgs &a);
    static void main(int storage, int cfg, const StepArgs &a);
    // chi; nb_out blocks of outlet collision and nb_in blocks of inlet nodes
    static void faces(int storage, const StepArgs &a, int nb_out, int nb_in);
    static void inlet(int storage, const StepArgs &a, unsigned nb, int nb_in);
    static void outlet_fill(int storage, const StepArgs &a, unsigned nb);
    static void scatter(int storage, const StepArgs &a, const double *f, float2 *ref_out);
    static void gather_state(int storage, const StepArgs &a, double *f);
    static void feq_state(const double *rho0, const double *u0, int64_t N, double *f, hipStream_t s);
    static void mass(int storage, const StepArgs &a, double *part, int nb, double *out);
    static void batch_step(int storage, int cfg, const BatchArgs &b);
    // droplet labels
    static void probe(int storage, const StepArgs &a, int k, const Box3 &bx, float thr, unsigned long long *out);
    static void lab_init(int storage, const StepArgs &a, int k, const Box3 &bx, float thr, int *lab);
    static void lab_prop(const StepArgs &a, int *lab, int *changed, int passes);
    static void lab_roots(const StepArgs &a, const int *lab, int *slot, int *n_roots);
    static void lab_stats(const StepArgs &a, const int *lab, const int *slot, CompStat *st, int n);
};

extern template struct Launcher<2>;
extern template struct Launcher<3>;

}  // namespace lbm
