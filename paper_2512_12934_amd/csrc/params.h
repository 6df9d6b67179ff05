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

// Elements of padding before x = 0 in every row of a population plane: one
// ghost slot is needed; 32 keeps x = 0 on a 128-byte boundary for FP32.
constexpr int XOFF = 32;

struct Geometry {
    int n[3];
    int P[3];              // padded sizes: rows of XOFF + n + 1 rounded up to 32
                           // elements, n + 2 on the other lattice axes
    int periodic[3];
    int64_t N;             // box nodes
    int64_t Ppad;          // padded nodes (stride between population planes)
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
    float *faceF;             // [slots][2][3] force of this step at role nodes
    float *faceU;             // [slots] normal velocity at x' (outward)
    double *faceQ;            // [slots] rho u.n at inlet and x' nodes (eq. 23 terms)
    double *ucpart;           // [inlet-kernel blocks][2] partial sum of u.n at x' and count
    int n_ucpart;
    double *scal;             // device scalars, see SC_* below
};

// Node-update kernel modes: a time step, or moments output only.
enum { MODE_STEP = 0, MODE_MOMENTS = 1 };

enum { SC_QIN = 0, SC_QOUT = 1, SC_CHI = 2, SC_UC = 3, SC_CLAMPS = 4, SC_COUNT = 8 };

}  // namespace lbm
