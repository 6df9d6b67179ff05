// params.h -- launch parameters shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace lbm {

// Per-node type word (box node order).
enum : uint32_t {
    T_BBMASK = (1u << 19) - 1,  // bit i: population i at this node comes back by bounce-back
    T_EDGE = 1u << 19,          // node on a periodic boundary layer: gathers wrap
    T_NEARWALL = 1u << 20,      // a solid lies within the interaction stencil
    T_SOLID = 1u << 21,
    T_INLET = 1u << 22,         // x1 of an inlet patch
    T_OUTLET = 1u << 23,        // x_N of the outlet
    T_XPRIME = 1u << 24,        // x_{N-1}: neighbour of an outlet node
    T_X2 = 1u << 25,            // x2: neighbour of an inlet node
    T_PATCH_SHIFT = 26,         // 3 bits: inlet patch of an x1 / x2 node
    T_PATCH_MASK = 7u << 26,
    T_MOVWALL = 1u << 29,       // a bounce-back link of this node meets a moving wall
    T_ROLE = T_INLET | T_OUTLET | T_XPRIME | T_X2,
};

constexpr int MAX_PATCH = 8;

// One inlet node x1 and its partner x2 = x1 + n.
struct InletRec {
    int64_t b1, b2;     // box indices
    int slot1, slot2;   // face-buffer slots
    int patch;
    int pad;
};

// One outlet node x_N and its partner x' = x_N - n_o.
struct OutletRec {
    int64_t bN, bP;
    int slotN, slotP;   // slotP < 0 when x' is solid
};

struct Physics {
    float se[2], seps[2], sq, snu[2];
    float G12, Gw[2], Fb[3];
    int adhesion;
};

// Rows of a population plane are padded to whole 128-byte lines and x = 0
// starts a line, so the unit-stride loads of a wave cover whole lines.
struct Geometry {
    int n[3];
    int P[3];              // padded sizes: rows of xoff + n + 1 rounded up to a
                           // whole number of lines, n + 2 on the other lattice axes
    int xoff;              // elements before x = 0 in every row
    int periodic[3];
    int64_t N;             // box nodes
    int64_t Ppad;          // padded nodes (stride between population planes)
    // The caller's frame: memory axis a holds the caller's lattice axis ax[a]
    // (the axis normal to the open faces of a 3-D domain is put last, so face
    // nodes are contiguous in memory).  ostride[a] is the caller-frame linear
    // stride of memory axis a and dmap[i] the caller-frame index of memory
    // direction i; used only where state enters or leaves the context.
    int ax[3];
    int64_t ostride[3];
    signed char dmap[19];
};

struct Patch {
    int axis, sign;        // inward normal = sign * e_axis
    float rho[2];
    float u_n;
    int alpha_on;
};

struct Boundary {
    int n_patch;
    const Patch *patch;       // [n_patch] device copy of the inlet patches
    int has_outlet, chi_on;
    int out_axis, out_sign;   // outward normal = out_sign * e_axis
    int n_in, n_out;          // record counts
    const InletRec *in;
    const OutletRec *out;
    const int *bslot;         // [N] face-buffer slot of role nodes, -1 elsewhere
    int n_xp;                 // fluid x_{N-1} nodes; face slots [0, n_in) are the inlet nodes and
                              // [n_in, n_in + n_xp) the x_{N-1} nodes, both in record order
    float *faceF;             // [slots][2][3] force of this step at role nodes
    float *faceU;             // [slots] normal velocity at x' (outward)
    // [2 parities][2] the eq. 23 sums Q_in and Q' of a step as integers in
    // units of 2^-40 (see flow_fix): the node update adds into the pair of
    // the step's parity, the first face launch reads it and clears the other
    unsigned long long *qacc;
    double *ucpart;           // [inlet-kernel blocks][2] partial sum of u.n at x' and count
    int n_ucpart;
    double *scal;             // device scalars, see SC_* below
    // [2][Q][slots] FP32 history of eq. (20): the populations entering through
    // the outlet at the previous step, at the face slot of each outlet node
    // (kept in FP32 whatever the storage: eq. 20 is a recursive filter with a
    // memory of 1 / U_c steps, so re-reading a rounded value every step would
    // hold it up to 1 / U_c rounding units from its fixed point)
    float *hist;
    int n_slots;
    // [slots][Q] moving-wall term per stored direction j of a T_MOVWALL node,
    // to be multiplied by the component's density: -2 w_j (e_j . u_w) / cs^2
    // where x + e_j is a moving solid node, 0 elsewhere
    const float *wallc;
};

// Threads per block of the face kernels (one wave: the face node counts are
// small, so narrow blocks spread the uncoalesced face gathers over more CUs).
constexpr int FACE_NT = 64;
// Consecutive node-update work items that one XCD takes per turn.
constexpr int MAIN_XCD_GROUP = 4;

// One member of a batch: what a single context passes to its step kernels.
struct Member {
    void *f[2];                // population arrays A and B
    const uint32_t *type;
    void *psi[2];              // float2 per box node: psi(t) in psi[cur], the reference
                               // densities of the stored state (psi(t-1)) in psi[cur ^ 1]
    Geometry g;
    Physics ph;
    Boundary bd;
    int tiles_x, tiles_y, n_items;
    const int *item_list;      // [n_items] tiles of the node update that hold fluid
    int nb_in, nb_out;         // face-kernel blocks
    int *flag;
};

// Device tables of a batch.  Every *0 array holds n + 1 prefix sums of the
// per-member block (or work-item) counts of one launch, so a block finds its
// member by a binary search and its local block index by a subtraction.
struct BatchTab {
    const Member *m;
    int n;
    const int *item0;          // node-update work items
    const int *item_mem;       // the member of each node-update work item
    const int *psi0;           // k_psi blocks
    const int *out0;           // outlet-collision blocks
    const int *inl0;           // inlet-kernel blocks (inlet nodes, then U_c partials)
    const int *fill0;          // outlet-fill blocks
};

// An axis-aligned box of nodes [lo, hi) in the memory frame.
struct Box3 {
    int lo[3], hi[3];
};

// Aggregates of one connected component (caller frame).
struct CompStat {
    unsigned long long size;
    unsigned long long first;  // smallest node index
    int lo[3], hi[3];          // bounding box [lo, hi)
};

enum { SC_QIN = 0, SC_QOUT = 1, SC_CHI = 2, SC_UC = 3, SC_CLAMPS = 4, SC_COUNT = 8 };

}  // namespace lbm
