// lbm_api.hip -- host runtime and C ABI of the HIP lattice Boltzmann solver.
//
// The context owns nothing but a carve-up of the caller's device workspace:
// two population arrays (source / destination of the pull-scheme step), the
// static node map, the face buffers of the open boundaries and the FP64
// reduction scratch.  lbm_step only enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "launch.h"
#include "lattice.h"
#include "params.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;

thread_local std::string g_create_error;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    int dim = 0, Q = 0, storage = 0;
    Geometry g{};
    int tiles[3] = {1, 1, 1};      // lateral x tiles, lateral y tiles, sweep chunks
    int64_t nblocks_main = 0;      // work items of the node update (tiles holding fluid)
    std::vector<int> item_list;    // their tile indices
    int64_t grid_main = 0;         // launched blocks (a multiple of 8 * MAIN_XCD_GROUP)
    int64_t n_slots = 0, n_in = 0, n_out = 0;
    int nb_in = 0, nb_out = 0;
    int nb_mass = 0;
    bool boundary = false;
    // byte offsets into the workspace
    size_t o_fA, o_fB, o_type, o_bslot, o_faceF, o_faceU, o_in, o_out, o_qacc, o_ucpart, o_scal,
        o_flag, o_mpart, o_mout, o_patch, o_psi[2], o_items, o_hist, o_wallc, total;
    bool moving = false;
    int cfg = 0;                   // node-update configuration (launch.h)
    int psi_mode = 1;              // 1: psi array written by k_psi, 0: recomputed in k_main
    bool inlet_early = true;       // no inlet node pulls from the collided outlet column, so the
                                   // inlet nodes run in the outlet collision's launch
};

// Host-side static maps built from the configuration.
struct Maps {
    std::vector<uint32_t> type;
    std::vector<int32_t> bslot;
    std::vector<std::vector<float>> wallc;   // [N] moving-wall term per stored direction (empty: none)
    bool moving = false;
    std::vector<InletRec> in;
    std::vector<OutletRec> out;
    int n_xp = 0;                  // fluid x_{N-1} nodes (slots n_in .. n_in + n_xp)
    bool inlet_pulls_outlet = false;   // an inlet node x1 or x2 streams from an outlet node
};

int lat_Q(int dim) { return dim == 2 ? 9 : 19; }

// Row layout of the population planes: elements per 128-byte line, the
// offset of x = 0 (the start of the second line of the row, so every row is
// line-aligned and the ghost slot x = -1 ends the first line) and the
// padded row pitch.
int line_elems(int storage) { return storage == LBM_STORE_F32 ? 32 : 64; }
int row_xoff(int storage)
{
    return line_elems(storage);
}
int row_pitch(int n0, int storage)
{
    const int le = line_elems(storage);
    return (row_xoff(storage) + n0 + 1 + le - 1) / le * le;
}

template <int DIM> void lat_e(int i, int *e)
{
    for (int d = 0; d < 3; d++) e[d] = Lat<DIM>::E[i][d];
}

void dir(int dim, int i, int *e)
{
    if (dim == 2) lat_e<2>(i, e);
    else lat_e<3>(i, e);
}

bool on_face(const lbm_config *c, const int *xc, int axis, int side, const int *lo, const int *hi)
{
    const int layer = side == 0 ? 0 : c->n[axis] - 1;
    if (xc[axis] != layer) return false;
    for (int a = 0; a < c->dim; a++) {
        if (a == axis) continue;
        if (xc[a] < lo[a] || xc[a] >= hi[a]) return false;
    }
    return true;
}

// The configuration in memory axis order.  With LBM_LAYOUT_FACE_LAST (3-D)
// the axis normal to the open faces (the outlet's, else the first inlet's)
// becomes the last memory axis, so the face nodes of the inlet and outlet
// kernels are contiguous planes instead of single elements strided by a row.  The lattice is closed under
// axis permutations and the collision operator commutes with them (equal
// rates within every moment group of one tensor order), so the permuted
// problem is the same problem; only entry and exit of state are remapped.
struct Canon {
    lbm_config c{};
    int ax[3] = {0, 1, 2};         // memory axis a holds the caller's axis ax[a]
    std::vector<uint8_t> solid;
    std::vector<double> wall_u;    // [3][N] in the memory frame, when permuted
};

std::string canonicalize(const lbm_config *in, Canon &k)
{
    if (!in) return "null configuration";
    if (in->dim != 2 && in->dim != 3) return "dim must be 2 or 3";
    if (in->dim == 2 && in->n[2] != 1) return "2-D boxes need n[2] == 1";
    for (int a = 0; a < in->dim; a++)
        if (in->n[a] < 3 || in->n[a] > (1 << 24)) return "every lattice axis needs 3 .. 2^24 nodes";
    if (!in->solid || !in->rho0) return "solid and rho0 arrays are required";
    const int64_t N = (int64_t)in->n[0] * in->n[1] * (in->dim == 3 ? in->n[2] : 1);
    for (int64_t b = 0; b < N; b++) {
        if (in->solid[b]) continue;
        if (!(in->rho0[b] > 0.0) || !(in->rho0[N + b] > 0.0))
            return "initial densities must be positive on fluid nodes";
    }
    int flow = -1;
    if (in->layout != LBM_LAYOUT_CALLER && in->layout != LBM_LAYOUT_FACE_LAST) return "unknown layout";
    if (in->dim == 3 && in->layout == LBM_LAYOUT_FACE_LAST) {
        if (in->has_outlet && in->outlet.axis >= 0 && in->outlet.axis < 3) flow = in->outlet.axis;
        else if (in->n_inlets > 0 && in->inlets[0].axis >= 0 && in->inlets[0].axis < 3) flow = in->inlets[0].axis;
    }
    if (flow >= 0 && flow != 2) {
        int j = 0;
        for (int a = 0; a < 3; a++)
            if (a != flow) k.ax[j++] = a;
        k.ax[2] = flow;
    }
    int inv[3];
    for (int a = 0; a < 3; a++) inv[k.ax[a]] = a;
    k.c = *in;
    lbm_config &c = k.c;
    for (int a = 0; a < 3; a++) {
        c.n[a] = in->n[k.ax[a]];
        c.periodic[a] = in->periodic[k.ax[a]];
        c.Fb[a] = in->Fb[k.ax[a]];
    }
    auto remap_face = [&](int &axis, int *lo, int *hi) {
        if (axis >= 0 && axis < 3) axis = inv[axis];
        int l[3], h[3];
        for (int a = 0; a < 3; a++) { l[a] = lo[k.ax[a]]; h[a] = hi[k.ax[a]]; }
        for (int a = 0; a < 3; a++) { lo[a] = l[a]; hi[a] = h[a]; }
    };
    for (int q = 0; q < c.n_inlets && q < LBM_MAX_INLETS; q++) remap_face(c.inlets[q].axis, c.inlets[q].lo, c.inlets[q].hi);
    if (c.has_outlet) remap_face(c.outlet.axis, c.outlet.lo, c.outlet.hi);
    if (k.ax[0] == 0 && k.ax[1] == 1 && k.ax[2] == 2) {
        c.solid = in->solid;
        c.wall_u = in->wall_u;
    } else {
        k.solid.resize(N);
        if (in->wall_u) k.wall_u.resize((size_t)3 * N);
        const int64_t st[3] = {1, in->n[0], (int64_t)in->n[0] * in->n[1]};
        const int64_t os[3] = {st[k.ax[0]], st[k.ax[1]], st[k.ax[2]]};
        int64_t b = 0;
        for (int z = 0; z < c.n[2]; z++)
            for (int y = 0; y < c.n[1]; y++)
                for (int x = 0; x < c.n[0]; x++, b++) {
                    const int64_t ob = x * os[0] + y * os[1] + z * os[2];
                    k.solid[b] = in->solid[ob];
                    if (in->wall_u)
                        for (int a = 0; a < 3; a++) k.wall_u[(size_t)a * N + b] = in->wall_u[(size_t)k.ax[a] * N + ob];
                }
        c.solid = k.solid.data();
        c.wall_u = in->wall_u ? k.wall_u.data() : nullptr;
    }
    // rho0 / u0 stay in the caller's frame: the initial state is built there
    // and scattered through the frame map
    return "";
}

// Validates the configuration and builds the node maps.  Returns an empty
// string on success, else the reason.
std::string build_maps(const lbm_config *c, Maps &m)
{
    if (!c) return "null configuration";
    if (c->dim != 2 && c->dim != 3) return "dim must be 2 or 3";
    if (c->storage != LBM_STORE_F32 && c->storage != LBM_STORE_F16_OFFSET && c->storage != LBM_STORE_F16_FIXED)
        return "unknown storage";
    const int nz = c->dim == 2 ? 1 : c->n[2];
    if (c->dim == 2 && c->n[2] != 1) return "2-D boxes need n[2] == 1";
    for (int a = 0; a < c->dim; a++) {
        if (c->n[a] < 3) return "every lattice axis needs at least 3 nodes";
        if (c->n[a] > (1 << 24)) return "axis too long";
    }
    if (!(c->nu[0] > 0.0) || !(c->nu[1] > 0.0)) return "viscosities must be positive";
    if (!(c->s_q > 0.0 && c->s_q < 2.0)) return "s_q must lie in (0, 2)";
    if (c->s_eps_policy != LBM_SEPS_MAXVISC && c->s_eps_policy != LBM_SEPS_FIXED) return "unknown s_eps policy";
    if (c->n_inlets < 0 || c->n_inlets > LBM_MAX_INLETS) return "bad inlet count";
    if (c->tile_config < -1 || c->tile_config >= n_tile_cfg(c->dim)) return "unknown tile configuration";
    if (!c->solid) return "the solid array is required";
    for (int q = 0; q < c->n_inlets; q++) {
        const lbm_inlet &p = c->inlets[q];
        if (p.axis < 0 || p.axis >= c->dim || (p.side != 0 && p.side != 1)) return "bad inlet face";
        if (c->periodic[p.axis]) return "inlet on a periodic axis";
        if (!(p.rho[0] >= 0.0) || !(p.rho[1] >= 0.0)) return "inlet densities must be >= 0";
    }
    if (c->has_outlet) {
        const lbm_outlet &o = c->outlet;
        if (o.axis < 0 || o.axis >= c->dim || (o.side != 0 && o.side != 1)) return "bad outlet face";
        if (c->periodic[o.axis]) return "outlet on a periodic axis";
    }
    const int64_t N = (int64_t)c->n[0] * c->n[1] * nz;
    const int Q = lat_Q(c->dim);
    {
        // each component array is addressed with 32-bit byte offsets
        const int64_t pad = (int64_t)row_pitch(c->n[0], c->storage) * (c->n[1] + 2) *
                            (c->dim == 3 ? c->n[2] + 2 : 1);
        const int64_t bytes = pad * Q * (c->storage == LBM_STORE_F32 ? 4 : 2);
        if (bytes >= ((int64_t)1 << 31)) return "domain too large for one context (2 GiB per component array)";
    }
    m.type.assign(N, 0);
    m.bslot.assign(N, -1);
    m.wallc.assign(c->wall_u ? N : 0, std::vector<float>());
    m.moving = false;
    m.in.clear();
    m.out.clear();
    auto solid_at = [&](const int *p) -> bool {
        int q[3] = {p[0], p[1], p[2]};
        for (int a = 0; a < c->dim; a++) {
            const int n = c->n[a];
            if (q[a] < 0) q[a] = c->periodic[a] ? q[a] + n : -1 - q[a];
            else if (q[a] >= n) q[a] = c->periodic[a] ? q[a] - n : 2 * n - 1 - q[a];
        }
        return c->solid[(int64_t)q[0] + (int64_t)c->n[0] * ((int64_t)q[1] + (int64_t)c->n[1] * q[2])] != 0;
    };
    std::vector<int8_t> inlet_of(N, -1);
    std::vector<uint8_t> is_out(N, 0);
    for (int64_t b = 0; b < N; b++) {
        if (c->solid[b]) continue;
        const int xc[3] = {(int)(b % c->n[0]), (int)((b / c->n[0]) % c->n[1]), (int)(b / ((int64_t)c->n[0] * c->n[1]))};
        for (int q = 0; q < c->n_inlets; q++)
            if (on_face(c, xc, c->inlets[q].axis, c->inlets[q].side, c->inlets[q].lo, c->inlets[q].hi))
                inlet_of[b] = (int8_t)q;
        if (c->has_outlet && on_face(c, xc, c->outlet.axis, c->outlet.side, c->outlet.lo, c->outlet.hi))
            is_out[b] = 1;
        if (inlet_of[b] >= 0 && is_out[b]) return "a node belongs to an inlet and the outlet";
    }
    for (int64_t b = 0; b < N; b++) {
        const int xc[3] = {(int)(b % c->n[0]), (int)((b / c->n[0]) % c->n[1]), (int)(b / ((int64_t)c->n[0] * c->n[1]))};
        if (c->solid[b]) {
            m.type[b] = T_SOLID;
            continue;
        }
        uint32_t tw = 0;
        for (int a = 0; a < c->dim; a++)
            if (c->periodic[a] && (xc[a] == 0 || xc[a] == c->n[a] - 1)) tw |= T_EDGE;
        for (int i = 0; i < Q; i++) {
            int e[3];
            dir(c->dim, i, e);
            int s[3] = {xc[0] - e[0], xc[1] - e[1], xc[2] - e[2]};
            bool outside = false;
            for (int a = 0; a < c->dim; a++) {
                if (s[a] < 0 || s[a] >= c->n[a]) {
                    if (c->periodic[a]) s[a] = (s[a] + c->n[a]) % c->n[a];
                    else outside = true;
                }
            }
            if (outside) {
                // the population arrives through a non-periodic face: an open
                // boundary has to supply it
                bool ok = false;
                const int q = inlet_of[b];
                if (q >= 0) ok = e[c->inlets[q].axis] * (c->inlets[q].side == 0 ? 1 : -1) > 0;
                if (is_out[b]) ok = ok || e[c->outlet.axis] * (c->outlet.side == 0 ? -1 : 1) < 0;
                if (!ok) return "a fluid node on a non-periodic face is not covered by an inlet or the outlet";
                continue;
            }
            const int64_t sb = (int64_t)s[0] + (int64_t)c->n[0] * ((int64_t)s[1] + (int64_t)c->n[1] * s[2]);
            if (c->solid[sb]) {
                tw |= 1u << i;
                if (c->wall_u) {
                    // population i comes back from the solid node s = x - e_i
                    // as the stored direction OPP[i] (= x + e_OPP[i]); a
                    // moving s adds -2 w (e_OPP[i] . u_w) / cs^2 times rho_k
                    double eu = 0.0;
                    for (int a = 0; a < c->dim; a++) eu += (double)e[a] * c->wall_u[(size_t)a * N + sb];
                    if (eu != 0.0) {
                        auto &wc = m.wallc[b];
                        if (wc.empty()) wc.assign(Q, 0.0f);
                        const int j = c->dim == 2 ? Lat<2>::OPP[i] : Lat<3>::OPP[i];
                        wc[j] = (float)(6.0 * (double)(c->dim == 2 ? weight<2>(i) : weight<3>(i)) * eu);
                    }
                }
            }
        }
        if (c->wall_u && !m.wallc[b].empty()) {
            tw |= T_MOVWALL;
            m.moving = true;
        }
        const int zr = c->dim == 3 ? 2 : 0;
        bool near = false;
        for (int dz = -zr; dz <= zr && !near; dz++)
            for (int dy = -2; dy <= 2 && !near; dy++)
                for (int dx = -2; dx <= 2 && !near; dx++) {
                    const int p[3] = {xc[0] + dx, xc[1] + dy, xc[2] + dz};
                    if (solid_at(p)) near = true;
                }
        if (near) tw |= T_NEARWALL;
        m.type[b] = tw;
    }
    // roles
    for (int64_t b = 0; b < N; b++) {
        const int q = inlet_of[b];
        if (q < 0) continue;
        const lbm_inlet &p = c->inlets[q];
        const int xc[3] = {(int)(b % c->n[0]), (int)((b / c->n[0]) % c->n[1]), (int)(b / ((int64_t)c->n[0] * c->n[1]))};
        int x2[3] = {xc[0], xc[1], xc[2]};
        x2[p.axis] += p.side == 0 ? 1 : -1;
        const int64_t b2 = (int64_t)x2[0] + (int64_t)c->n[0] * ((int64_t)x2[1] + (int64_t)c->n[1] * x2[2]);
        m.type[b] |= T_INLET | ((uint32_t)q << T_PATCH_SHIFT);
        if (!c->solid[b2]) {
            if (m.type[b2] & T_INLET) return "inlet patches are less than two nodes apart";
            m.type[b2] |= T_X2 | ((uint32_t)q << T_PATCH_SHIFT);
        }
        InletRec r{};
        r.b1 = b;
        r.b2 = b2;
        r.patch = q;
        m.in.push_back(r);
    }
    if (c->has_outlet) {
        const lbm_outlet &o = c->outlet;
        for (int64_t b = 0; b < N; b++) {
            if (!is_out[b]) continue;
            const int xc[3] = {(int)(b % c->n[0]), (int)((b / c->n[0]) % c->n[1]), (int)(b / ((int64_t)c->n[0] * c->n[1]))};
            int xp[3] = {xc[0], xc[1], xc[2]};
            xp[o.axis] += o.side == 0 ? 1 : -1;
            const int64_t bp = (int64_t)xp[0] + (int64_t)c->n[0] * ((int64_t)xp[1] + (int64_t)c->n[1] * xp[2]);
            m.type[b] |= T_OUTLET;
            OutletRec r{};
            r.bN = b;
            r.bP = bp;
            if (!c->solid[bp]) {
                if (m.type[bp] & (T_INLET | T_OUTLET)) return "the outlet is less than two nodes from an open face";
                m.type[bp] |= T_XPRIME;
            } else {
                r.bP = -1;
            }
            m.out.push_back(r);
        }
    }
    // face slots: the inlet nodes in record order, then the fluid x_{N-1}
    // nodes in outlet record order (so the eq. 23 sums read two contiguous
    // ranges in a fixed order), then every other role node in box order
    int32_t slot = 0;
    for (auto &r : m.in) m.bslot[r.b1] = slot++;
    m.n_xp = 0;
    for (auto &r : m.out)
        if (r.bP >= 0 && m.bslot[r.bP] < 0) {
            m.bslot[r.bP] = slot++;
            m.n_xp++;
        }
    for (int64_t b = 0; b < N; b++)
        if ((m.type[b] & (T_ROLE | T_MOVWALL)) && m.bslot[b] < 0) m.bslot[b] = slot++;
    for (int64_t b = 0; b < N; b++)
        if ((m.type[b] & T_MOVWALL) && (m.type[b] & T_OUTLET))
            return "a moving wall next to the outlet column is not supported";
    for (auto &r : m.in) {
        r.slot1 = m.bslot[r.b1];
        r.slot2 = c->solid[r.b2] ? r.slot1 : m.bslot[r.b2];
    }
    // does the inlet rule read a population that the outlet collision
    // writes?  It reads the streamed populations of x1 and x2, so it
    // depends on the outlet column when one of them pulls from it
    for (const auto &r : m.in) {
        for (int k = 0; k < 2 && !m.inlet_pulls_outlet; k++) {
            const int64_t b = k == 0 ? r.b1 : r.b2;
            if (c->solid[b]) continue;
            const int xc[3] = {(int)(b % c->n[0]), (int)((b / c->n[0]) % c->n[1]),
                               (int)(b / ((int64_t)c->n[0] * c->n[1]))};
            for (int i = 0; i < Q; i++) {
                int e[3];
                dir(c->dim, i, e);
                int sx[3] = {xc[0] - e[0], xc[1] - e[1], xc[2] - e[2]};
                bool inside = true;
                for (int a = 0; a < c->dim; a++)
                    if (sx[a] < 0 || sx[a] >= c->n[a]) {
                        if (c->periodic[a]) sx[a] = (sx[a] + c->n[a]) % c->n[a];
                        else inside = false;
                    }
                if (!inside) continue;
                const int64_t sb = (int64_t)sx[0] + (int64_t)c->n[0] * ((int64_t)sx[1] + (int64_t)c->n[1] * sx[2]);
                if (m.type[sb] & T_OUTLET) m.inlet_pulls_outlet = true;
            }
        }
    }
    for (auto &r : m.out) {
        r.slotN = m.bslot[r.bN];
        r.slotP = r.bP >= 0 ? m.bslot[r.bP] : -1;
        if (r.bP < 0) r.bP = r.bN;
    }
    return "";
}

// Default node-update configuration: the measured best of the tuning space
// for the lattice (see the autotuner), entry 0 otherwise.
int default_cfg(const lbm_config *c)
{
    (void)c;
    return 0;
}

Layout make_layout(const Canon &k, const Maps &m)
{
    const lbm_config *c = &k.c;
    Layout L;
    L.dim = c->dim;
    L.Q = lat_Q(c->dim);
    L.storage = c->storage;
    Geometry &g = L.g;
    for (int a = 0; a < 3; a++) {
        g.n[a] = a < c->dim ? c->n[a] : 1;
        g.P[a] = a == 0 ? row_pitch(c->n[0], c->storage) : (a < c->dim ? c->n[a] + 2 : 1);
        g.periodic[a] = a < c->dim ? (c->periodic[a] != 0) : 1;
    }
    g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    g.Ppad = (int64_t)g.P[0] * g.P[1] * g.P[2];
    g.xoff = row_xoff(c->storage);
    {
        // the caller's frame
        int on[3];
        for (int a = 0; a < 3; a++) on[k.ax[a]] = g.n[a];
        const int64_t st[3] = {1, on[0], (int64_t)on[0] * on[1]};
        for (int a = 0; a < 3; a++) {
            g.ax[a] = k.ax[a];
            g.ostride[a] = st[k.ax[a]];
        }
        const int Q = lat_Q(c->dim);
        for (int i = 0; i < 19; i++) g.dmap[i] = (signed char)i;
        for (int i = 0; i < Q; i++) {
            int e[3], p[3];
            dir(c->dim, i, e);
            for (int a = 0; a < 3; a++) p[k.ax[a]] = e[a];
            for (int j = 0; j < Q; j++) {
                int f[3];
                dir(c->dim, j, f);
                if (f[0] == p[0] && f[1] == p[1] && f[2] == p[2]) g.dmap[i] = (signed char)j;
            }
        }
    }
    L.cfg = c->tile_config >= 0 ? c->tile_config : default_cfg(c);
    const TileCfg &tc = tile_cfg(c->dim, L.cfg);
    L.psi_mode = tc.psrc;
    if (c->dim == 2) {
        L.tiles[0] = (g.n[0] + tc.tx - 1) / tc.tx;
        L.tiles[1] = 1;
        L.tiles[2] = (g.n[1] + tc.zc - 1) / tc.zc;
    } else {
        L.tiles[0] = (g.n[0] + tc.tx - 1) / tc.tx;
        L.tiles[1] = (g.n[1] + tc.ty - 1) / tc.ty;
        L.tiles[2] = (g.n[2] + tc.zc - 1) / tc.zc;
    }
    // the work list: every tile that holds a fluid node (all-solid tiles,
    // common in channel networks, are never launched)
    {
        const int64_t all = (int64_t)L.tiles[0] * L.tiles[1] * L.tiles[2];
        std::vector<uint8_t> live(all, 0);
        const int ny = c->dim == 3 ? g.n[1] : 1, nz = c->dim == 3 ? g.n[2] : g.n[1];
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < g.n[0]; x++) {
                    const int64_t b = (int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)ny * z);
                    if (m.type[b] & T_SOLID) continue;
                    const int64_t it = x / tc.tx + (int64_t)L.tiles[0] * ((c->dim == 3 ? y / tc.ty : 0) +
                                                                          (int64_t)L.tiles[1] * (z / tc.zc));
                    live[it] = 1;
                }
        L.item_list.clear();
        for (int64_t it = 0; it < all; it++)
            if (live[it]) L.item_list.push_back((int)it);
    }
    L.nblocks_main = (int64_t)L.item_list.size();
    L.grid_main = std::max<int64_t>((L.nblocks_main + 8 * MAIN_XCD_GROUP - 1) / (8 * MAIN_XCD_GROUP) *
                                        (8 * MAIN_XCD_GROUP), 8 * MAIN_XCD_GROUP);
    L.n_in = (int64_t)m.in.size();
    L.n_out = (int64_t)m.out.size();
    L.n_slots = 0;
    for (auto s : m.bslot) L.n_slots = std::max<int64_t>(L.n_slots, s + 1);
    L.moving = m.moving;
    L.boundary = L.n_in > 0 || c->has_outlet;
    L.nb_in = (int)((L.n_in + FACE_NT - 1) / FACE_NT);
    L.nb_out = (int)((L.n_out + FACE_NT - 1) / FACE_NT);
    L.inlet_early = !(c->has_outlet && c->outlet.chi_on) || !m.inlet_pulls_outlet;
    L.nb_mass = (int)std::min<int64_t>(1024, (g.N + 255) / 256);
    const size_t fbytes = (size_t)2 * L.Q * g.Ppad * (L.storage == LBM_STORE_F32 ? 4 : 2);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align_up(std::max<size_t>(bytes, 1)); return at; };
    L.o_fA = take(fbytes);
    L.o_fB = take(fbytes);
    L.o_type = take((size_t)g.N * 4);
    L.o_bslot = take((size_t)g.N * 4);
    L.o_faceF = take((size_t)L.n_slots * 6 * 4);
    L.o_faceU = take((size_t)L.n_slots * 4);
    L.o_in = take((size_t)L.n_in * sizeof(InletRec));
    L.o_out = take((size_t)L.n_out * sizeof(OutletRec));
    L.o_qacc = take(4 * sizeof(unsigned long long));
    L.o_ucpart = take((size_t)std::max(L.nb_out, 1) * 16);
    L.o_scal = take(SC_COUNT * 8);
    L.o_flag = take(4);
    L.o_mpart = take((size_t)L.nb_mass * 16);
    L.o_mout = take(16);
    L.o_patch = take(sizeof(Patch) * MAX_PATCH);
    L.o_psi[0] = take((size_t)g.N * 8);
    L.o_psi[1] = take((size_t)g.N * 8);
    L.o_items = take(L.item_list.size() * 4);
    L.o_hist = take(c->has_outlet ? (size_t)2 * L.Q * L.n_slots * 4 : 0);
    L.o_wallc = take(m.moving ? (size_t)L.Q * L.n_slots * 4 : 0);
    L.total = o;
    return L;
}

// Scratch of lbm_components_static: a file-scope device array, so that the
// entry point allocates nothing.  Each device holds its own copy for the
// life of the process; host code uses only the device address that
// hipGetSymbolAddress returns for it (the array's name is a host-side
// stand-in).  Layout: lab [MAX_NODES] int, slot [MAX_NODES] int, two int
// counters, MAX_COMPONENTS CompStat, MAX_COMPONENTS lbm_component (ordered).
constexpr size_t SCR_LAB = 0;
constexpr size_t SCR_SLOT = SCR_LAB + (size_t)LBM_COMPONENTS_STATIC_MAX_NODES * 4;
constexpr size_t SCR_FLAGS = SCR_SLOT + (size_t)LBM_COMPONENTS_STATIC_MAX_NODES * 4;
constexpr size_t SCR_STATS = SCR_FLAGS + 256;
constexpr size_t SCR_SORTED = SCR_STATS + (size_t)LBM_COMPONENTS_STATIC_MAX_COMPONENTS * sizeof(CompStat);
constexpr size_t SCR_BYTES = SCR_SORTED + (size_t)LBM_COMPONENTS_STATIC_MAX_COMPONENTS * sizeof(lbm_component);
static_assert(sizeof(CompStat) % 8 == 0 && sizeof(lbm_component) % 8 == 0, "scratch record alignment");

static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on device dev (current), resolved once.
std::string static_scratch_resolve(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return "device index out of range for the static scratch";
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return "";
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    g_scratch_ptr[dev] = ptr;
    return "";
}

void *static_scratch_ptr(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// Orders the n component records by their smallest node index (all distinct)
// into the caller's record layout: record i goes to the rank of its first
// index among all n.
__global__ __launch_bounds__(256) void k_lab_order(const CompStat *__restrict__ st, int n,
                                                   lbm_component *__restrict__ out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const unsigned long long fi = st[i].first;
    int rank = 0;
    for (int j = 0; j < n; j++) rank += st[j].first < fi ? 1 : 0;
    lbm_component r;
    r.first = (int64_t)fi;
    r.size = (int64_t)st[i].size;
    for (int d = 0; d < 3; d++) {
        r.lo[d] = st[i].lo[d];
        r.hi[d] = st[i].hi[d];
    }
    out[rank] = r;
}

}  // namespace

struct lbm_ctx {
    Layout L;
    lbm_config cfg;
    Physics ph{};
    Boundary bd{};
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int cur = 0;           // which array holds f(t): 0 = A, 1 = B
    int device = 0;        // the HIP device current at creation
    int64_t steps = 0;
    double mass0[2] = {0, 0};
    bool unstable = false;
    std::string err;
    // Step loop as a replayed HIP graph: graph_steps steps per graph, one
    // executable per parity of the A/B arrays at its start, captured on a
    // private stream the first time it is needed.
    int graph_steps = 16;
    hipStream_t cap = nullptr;
    hipGraphExec_t gx[2] = {nullptr, nullptr};
    ~lbm_ctx()
    {
        for (auto &g : gx)
            if (g) (void)hipGraphExecDestroy(g);
        if (cap) (void)hipStreamDestroy(cap);
    }
    void *fsrc() const { return ws + (cur == 0 ? L.o_fA : L.o_fB); }
    void *fdst() const { return ws + (cur == 0 ? L.o_fB : L.o_fA); }
    const uint32_t *type() const { return (const uint32_t *)(ws + L.o_type); }
    int *flag() const { return (int *)(ws + L.o_flag); }
};

namespace {

lbm_status fail(lbm_ctx *c, lbm_status st, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return st;
}

#define HIPCHECK(ctx, call)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

StepArgs step_args(const lbm_ctx *c, double *orho = nullptr, double *ou = nullptr)
{
    const Layout &L = c->L;
    StepArgs a{};
    a.src = c->fsrc();
    a.dst = c->fdst();
    a.type = c->type();
    // psi(t) and the reference densities of the stored state alternate
    // with the population arrays
    a.psi = (float2 *)(c->ws + L.o_psi[c->cur]);
    a.ref = (const float2 *)(c->ws + L.o_psi[c->cur ^ 1]);
    a.g = L.g;
    a.ph = c->ph;
    a.bd = c->bd;
    a.tiles_x = L.tiles[0];
    a.tiles_y = L.tiles[1];
    a.items = (int)L.nblocks_main;
    a.item_list = (const int *)(c->ws + L.o_items);
    a.grid = (unsigned)L.grid_main;
    a.orho = orho;
    a.ou = ou;
    a.flag = c->flag();
    a.qacc = c->bd.qacc + 2 * c->cur;
    a.qnext = c->bd.qacc + 2 * (c->cur ^ 1);
    a.stream = c->stream;
    return a;
}

template <int DIM> struct Ops {
    using Lx = Launcher<DIM>;

    // rho and u of the current state: psi of every node, then one thread per node
    static void moments(lbm_ctx *c, double *orho, double *ou)
    {
        StepArgs a = step_args(c, orho, ou);
        Lx::psi(c->L.storage, a);
        Lx::moments(c->L.storage, a);
    }

    // ev (optional): events bracketing k_psi (ev[8], ev[9]) and k_main (ev[0], ev[1])
    static void main_kernel(lbm_ctx *c, hipEvent_t *ev = nullptr)
    {
        const Layout &L = c->L;
        StepArgs a = step_args(c);
        if (L.psi_mode) {
            if (ev) (void)hipEventRecord(ev[8], c->stream);
            Lx::psi(L.storage, a);
            if (ev) (void)hipEventRecord(ev[9], c->stream);
        }
        if (ev) (void)hipEventRecord(ev[0], c->stream);
        Lx::main(L.storage, L.cfg, a);
        if (ev) (void)hipEventRecord(ev[1], c->stream);
    }

    // ev (optional): 10 events bracketing the launches of the step
    static void step(lbm_ctx *c, hipEvent_t *ev = nullptr)
    {
        const Layout &L = c->L;
        main_kernel(c, ev);
        if (L.boundary) {
            const StepArgs a = step_args(c);
            // chi, the outlet collision and (when independent of it) the inlet nodes
            const int nb_coll = c->bd.has_outlet && c->bd.chi_on ? L.nb_out : 0;
            const int nb_in_early = L.inlet_early ? L.nb_in : 0;
            if (ev) (void)hipEventRecord(ev[2], c->stream);
            Lx::faces(L.storage, a, nb_coll, nb_in_early);
            if (ev) (void)hipEventRecord(ev[3], c->stream);
            // the remaining inlet nodes, then the U_c partial sums of eq. (21)
            const int nb_in_late = L.nb_in - nb_in_early;
            if (nb_in_late + L.nb_out > 0) {
                if (ev) (void)hipEventRecord(ev[4], c->stream);
                Lx::inlet(L.storage, a, (unsigned)(nb_in_late + L.nb_out), nb_in_late);
                if (ev) (void)hipEventRecord(ev[5], c->stream);
            }
            if (L.nb_out > 0) {
                if (ev) (void)hipEventRecord(ev[6], c->stream);
                Lx::outlet_fill(L.storage, a, (unsigned)L.nb_out);
                if (ev) (void)hipEventRecord(ev[7], c->stream);
            }
        }
        c->cur ^= 1;
    }

    // the state and its reference densities, then psi of the state
    static void scatter(lbm_ctx *c, const double *dev_f)
    {
        const StepArgs a = step_args(c);
        Lx::scatter(c->L.storage, a, dev_f, (float2 *)(c->ws + c->L.o_psi[c->cur ^ 1]));
        Lx::psi(c->L.storage, a);
    }
    static void gather_state(lbm_ctx *c, double *dev_f) { Lx::gather_state(c->L.storage, step_args(c), dev_f); }
    static void mass(lbm_ctx *c, double *out)
    {
        Lx::mass(c->L.storage, step_args(c), (double *)(c->ws + c->L.o_mpart), c->L.nb_mass, out);
    }
    static void feq_state(lbm_ctx *c, const double *rho0, const double *u0, double *f)
    {
        Lx::feq_state(rho0, u0, c->L.g.N, f, c->stream);
    }
};

template <typename F> void dispatch(const lbm_ctx *c, F &&f)
{
    if (c->L.dim == 2) f(Ops<2>{});
    else f(Ops<3>{});
}

lbm_status current_mass(lbm_ctx *c, double *mass)
{
    double *out = (double *)(c->ws + c->L.o_mout);
    dispatch(c, [&](auto l) { decltype(l)::mass(c, out); });
    HIPCHECK(c, hipGetLastError());
    HIPCHECK(c, hipMemcpyAsync(mass, out, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status check_flag(lbm_ctx *c)
{
    int flag = 0;
    HIPCHECK(c, hipMemcpyAsync(&flag, c->flag(), 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (flag) c->unstable = true;
    return c->unstable ? LBM_EUNSTABLE : LBM_OK;
}

// Captures graph_steps steps starting from A/B parity `parity` on the
// private capture stream and instantiates them into gx[parity].
lbm_status capture_steps(lbm_ctx *c, int parity)
{
    const int G = c->graph_steps;
    hipGraphExec_t &gx = c->gx[parity];
    if (gx || G <= 0) return LBM_OK;
    if (!c->cap) HIPCHECK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    const int cur = c->cur;
    c->stream = c->cap;
    c->cur = parity;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int t = 0; t < G; t++) dispatch(c, [&](auto l) { decltype(l)::step(c); });
        e = hipStreamEndCapture(c->cap, &graph);
    }
    c->stream = user;
    c->cur = cur;
    if (e == hipSuccess) e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, std::string("step graph: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_config *cfg)
{
    Canon k;
    if (!canonicalize(cfg, k).empty()) return 0;
    Maps m;
    if (!build_maps(&k.c, m).empty()) return 0;
    return make_layout(k, m).total;
}

lbm_status lbm_create(const lbm_config *cfg, void *dev_ws, size_t ws_bytes, void *hip_stream, lbm_ctx **out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    Canon canon;
    std::string why = canonicalize(cfg, canon);
    if (!why.empty()) return fail(nullptr, LBM_EINVAL, why);
    const double *rho0 = cfg->rho0, *u0 = cfg->u0;   // caller's frame
    cfg = &canon.c;                                   // memory frame from here on
    Maps m;
    why = build_maps(cfg, m);
    if (!why.empty()) return fail(nullptr, LBM_EINVAL, why);
    Layout L = make_layout(canon, m);
    if (!dev_ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)dev_ws) % ALIGN) return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(nullptr, LBM_ENOMEM, "workspace too small");

    lbm_ctx *c = new lbm_ctx();
    c->L = L;
    c->cfg = *cfg;
    c->cfg.solid = nullptr;
    c->cfg.rho0 = nullptr;
    c->cfg.u0 = nullptr;
    c->cfg.wall_u = nullptr;
    c->ws = (char *)dev_ws;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LBM_EDEVICE, "hipGetDevice failed");
    }
    {
        // resolve the device address of the allocation-free labelling
        // scratch once per device, at set-up
        std::string why = static_scratch_resolve(c->device);
        if (!why.empty()) {
            delete c;
            return fail(nullptr, LBM_EDEVICE, why);
        }
    }

    // relaxation rates (eqs. 4-5, Sec. III A)
    Physics &ph = c->ph;
    const double numax = std::max(cfg->nu[0], cfg->nu[1]);
    for (int k = 0; k < 2; k++) {
        const double snu = 1.0 / (3.0 * cfg->nu[k] + 0.5);
        const double seps = cfg->s_eps_policy == LBM_SEPS_MAXVISC ? 1.0 / (3.0 * numax + 0.5) : snu;
        ph.snu[k] = (float)snu;
        ph.seps[k] = (float)seps;
        ph.se[k] = (float)seps;
    }
    ph.sq = (float)cfg->s_q;
    ph.G12 = (float)cfg->G12;
    ph.Gw[0] = (float)cfg->Gw[0];
    ph.Gw[1] = (float)cfg->Gw[1];
    for (int d = 0; d < 3; d++) ph.Fb[d] = (float)cfg->Fb[d];
    ph.adhesion = (cfg->Gw[0] != 0.0 || cfg->Gw[1] != 0.0) ? 1 : 0;

    Boundary &bd = c->bd;
    bd.n_patch = cfg->n_inlets;
    Patch patches[MAX_PATCH] = {};
    for (int q = 0; q < cfg->n_inlets; q++) {
        const lbm_inlet &p = cfg->inlets[q];
        patches[q].axis = p.axis;
        patches[q].sign = p.side == 0 ? 1 : -1;
        patches[q].rho[0] = (float)p.rho[0];
        patches[q].rho[1] = (float)p.rho[1];
        patches[q].u_n = (float)p.u_n;
        patches[q].alpha_on = p.alpha_on ? 1 : 0;
    }
    bd.has_outlet = cfg->has_outlet ? 1 : 0;
    bd.chi_on = cfg->has_outlet && cfg->outlet.chi_on ? 1 : 0;
    bd.out_axis = cfg->has_outlet ? cfg->outlet.axis : 0;
    bd.out_sign = cfg->has_outlet ? (cfg->outlet.side == 0 ? -1 : 1) : 1;
    bd.n_in = (int)L.n_in;
    bd.n_out = (int)L.n_out;
    char *ws = c->ws;
    bd.in = (const InletRec *)(ws + L.o_in);
    bd.out = (const OutletRec *)(ws + L.o_out);
    bd.bslot = (const int *)(ws + L.o_bslot);
    bd.n_xp = m.n_xp;
    bd.faceF = (float *)(ws + L.o_faceF);
    bd.faceU = (float *)(ws + L.o_faceU);
    bd.qacc = (unsigned long long *)(ws + L.o_qacc);
    bd.ucpart = (double *)(ws + L.o_ucpart);
    bd.n_ucpart = L.nb_out;
    bd.scal = (double *)(ws + L.o_scal);
    bd.patch = (const Patch *)(ws + L.o_patch);
    bd.hist = (float *)(ws + L.o_hist);
    bd.n_slots = (int)L.n_slots;
    bd.wallc = L.moving ? (const float *)(ws + L.o_wallc) : nullptr;

    auto st = [&]() -> lbm_status {
        hipStream_t s = c->stream;
        HIPCHECK(c, hipMemsetAsync(ws, 0, L.total, s));
        HIPCHECK(c, hipMemcpyAsync(ws + L.o_type, m.type.data(), m.type.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHECK(c, hipMemcpyAsync(ws + L.o_bslot, m.bslot.data(), m.bslot.size() * 4, hipMemcpyHostToDevice, s));
        if (L.n_in)
            HIPCHECK(c, hipMemcpyAsync(ws + L.o_in, m.in.data(), m.in.size() * sizeof(InletRec), hipMemcpyHostToDevice, s));
        if (L.n_out)
            HIPCHECK(c, hipMemcpyAsync(ws + L.o_out, m.out.data(), m.out.size() * sizeof(OutletRec), hipMemcpyHostToDevice, s));
        HIPCHECK(c, hipMemcpyAsync(ws + L.o_patch, patches, sizeof patches, hipMemcpyHostToDevice, s));
        std::vector<float> wallc;
        if (L.moving) {
            wallc.assign((size_t)L.n_slots * L.Q, 0.0f);
            for (int64_t b = 0; b < L.g.N; b++)
                if (!m.wallc[b].empty())
                    for (int j = 0; j < L.Q; j++) wallc[(size_t)m.bslot[b] * L.Q + j] = m.wallc[b][j];
            HIPCHECK(c, hipMemcpyAsync(ws + L.o_wallc, wallc.data(), wallc.size() * 4, hipMemcpyHostToDevice, s));
        }
        if (!L.item_list.empty())
            HIPCHECK(c, hipMemcpyAsync(ws + L.o_items, L.item_list.data(), L.item_list.size() * 4,
                                       hipMemcpyHostToDevice, s));
        const double one = 1.0;
        HIPCHECK(c, hipMemcpyAsync(ws + L.o_scal + SC_CHI * 8, &one, 8, hipMemcpyHostToDevice, s));
        // initial state f = feq(rho0, u0), scattered into the source slots
        const int64_t N = L.g.N;
        double *d_rho = nullptr, *d_u = nullptr, *d_f = nullptr;
        HIPCHECK(c, hipMalloc(&d_rho, (size_t)2 * N * 8));
        if (u0) HIPCHECK(c, hipMalloc(&d_u, (size_t)3 * N * 8));
        HIPCHECK(c, hipMalloc(&d_f, (size_t)2 * L.Q * N * 8));
        HIPCHECK(c, hipMemcpyAsync(d_rho, rho0, (size_t)2 * N * 8, hipMemcpyHostToDevice, s));
        if (u0) HIPCHECK(c, hipMemcpyAsync(d_u, u0, (size_t)3 * N * 8, hipMemcpyHostToDevice, s));
        dispatch(c, [&](auto l) { decltype(l)::feq_state(c, d_rho, d_u, d_f); });
        dispatch(c, [&](auto l) { decltype(l)::scatter(c, d_f); });
        HIPCHECK(c, hipGetLastError());
        HIPCHECK(c, hipStreamSynchronize(s));
        HIPCHECK(c, hipFree(d_rho));
        if (d_u) HIPCHECK(c, hipFree(d_u));
        HIPCHECK(c, hipFree(d_f));
        return current_mass(c, c->mass0);
    }();
    if (st != LBM_OK) {
        g_create_error = c->err;
        delete c;
        return st;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c || n < 0) return fail(c, LBM_EINVAL, "bad arguments to lbm_step");
    if (c->unstable) return fail(c, LBM_ESTATE, "context flagged unstable");
    const int64_t n0 = n;
    const int G = c->graph_steps;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHECK(c, hipStreamIsCapturing(c->stream, &cs));
    // inside the caller's own capture the kernels go straight into it; the
    // A/B arrays swap every step, so only an even count leaves the arrays
    // where every replay of the caller's graph expects them
    if (cs != hipStreamCaptureStatusNone && n % 2)
        return fail(c, LBM_EINVAL, "a captured lbm_step must enqueue an even number of steps");
    if (G > 0 && cs == hipStreamCaptureStatusNone) {
        while (n >= G) {
            hipGraphExec_t &gx = c->gx[c->cur];
            if (!gx) {
                const lbm_status st = capture_steps(c, c->cur);
                if (st != LBM_OK) return st;
            }
            HIPCHECK(c, hipGraphLaunch(gx, c->stream));
            if (G % 2) c->cur ^= 1;
            n -= G;
        }
    }
    for (int64_t t = 0; t < n; t++) dispatch(c, [&](auto l) { decltype(l)::step(c); });
    HIPCHECK(c, hipGetLastError());
    c->steps += n0;
    return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_ctx *c, int steps_per_graph)
{
    if (!c || steps_per_graph < 0 || steps_per_graph > 4096) return fail(c, LBM_EINVAL, "bad steps per graph");
    for (auto &g : c->gx)
        if (g) {
            HIPCHECK(c, hipGraphExecDestroy(g));
            g = nullptr;
        }
    c->graph_steps = steps_per_graph;
    // capture and upload both parities now, so that no later lbm_step pays
    // for a capture
    for (int p = 0; p < 2 && steps_per_graph > 0; p++) {
        const lbm_status st = capture_steps(c, p);
        if (st != LBM_OK) return st;
        HIPCHECK(c, hipGraphUpload(c->gx[p], c->stream));
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx *c, double *rho, double *u, int dst_on_device)
{
    if (!c || !rho || !u) return fail(c, LBM_EINVAL, "bad arguments to lbm_moments");
    const int64_t N = c->L.g.N;
    double *drho = rho, *du = u;
    if (!dst_on_device) {
        HIPCHECK(c, hipMalloc(&drho, (size_t)2 * N * 8));
        HIPCHECK(c, hipMalloc(&du, (size_t)3 * N * 8));
    }
    HIPCHECK(c, hipMemsetAsync(du, 0, (size_t)3 * N * 8, c->stream));
    dispatch(c, [&](auto l) { decltype(l)::moments(c, drho, du); });
    HIPCHECK(c, hipGetLastError());
    if (!dst_on_device) {
        HIPCHECK(c, hipMemcpyAsync(rho, drho, (size_t)2 * N * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipMemcpyAsync(u, du, (size_t)3 * N * 8, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (!dst_on_device) {
        HIPCHECK(c, hipFree(drho));
        HIPCHECK(c, hipFree(du));
    }
    return check_flag(c);
}

lbm_status lbm_mass_flux(lbm_ctx *c, lbm_flux *out)
{
    if (!c || !out) return fail(c, LBM_EINVAL, "bad arguments to lbm_mass_flux");
    double sc[SC_COUNT];
    HIPCHECK(c, hipMemcpyAsync(sc, c->ws + c->L.o_scal, sizeof sc, hipMemcpyDeviceToHost, c->stream));
    double mass[2];
    lbm_status st = current_mass(c, mass);
    if (st != LBM_OK) return st;
    out->step = c->steps;
    out->q_in = sc[SC_QIN];
    out->q_out = sc[SC_QOUT];
    out->chi = sc[SC_CHI];
    out->u_conv = sc[SC_UC];
    out->uc_clamps = (int64_t)sc[SC_CLAMPS];
    out->mass[0] = mass[0];
    out->mass[1] = mass[1];
    out->mass0[0] = c->mass0[0];
    out->mass0[1] = c->mass0[1];
    return check_flag(c);
}

lbm_status lbm_get_state(lbm_ctx *c, double *f_host, size_t bytes)
{
    if (!c || !f_host) return fail(c, LBM_EINVAL, "bad arguments to lbm_get_state");
    const size_t need = (size_t)16 * c->L.Q * c->L.g.N;
    if (bytes != need) return fail(c, LBM_EINVAL, "state buffer has the wrong size");
    double *d = nullptr;
    HIPCHECK(c, hipMalloc(&d, need));
    dispatch(c, [&](auto l) { decltype(l)::gather_state(c, d); });
    HIPCHECK(c, hipGetLastError());
    HIPCHECK(c, hipMemcpyAsync(f_host, d, need, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipFree(d));
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx *c, const double *f_host, size_t bytes)
{
    if (!c || !f_host) return fail(c, LBM_EINVAL, "bad arguments to lbm_set_state");
    const size_t need = (size_t)16 * c->L.Q * c->L.g.N;
    if (bytes != need) return fail(c, LBM_EINVAL, "state buffer has the wrong size");
    double *d = nullptr;
    HIPCHECK(c, hipMalloc(&d, need));
    HIPCHECK(c, hipMemcpyAsync(d, f_host, need, hipMemcpyHostToDevice, c->stream));
    dispatch(c, [&](auto l) { decltype(l)::scatter(c, d); });
    HIPCHECK(c, hipGetLastError());
    HIPCHECK(c, hipMemsetAsync(c->flag(), 0, 4, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipFree(d));
    c->unstable = false;
    return LBM_OK;
}

lbm_status lbm_time_kernels(lbm_ctx *c, int64_t n, double *ms)
{
    if (!c || n <= 0 || !ms) return fail(c, LBM_EINVAL, "bad arguments to lbm_time_kernels");
    if (c->unstable) return fail(c, LBM_ESTATE, "context flagged unstable");
    const int64_t total = n * 10;
    std::vector<hipEvent_t> ev(total);
    for (auto &e : ev) HIPCHECK(c, hipEventCreate(&e));
    for (int64_t t = 0; t < n; t++) dispatch(c, [&](auto l) { decltype(l)::step(c, ev.data() + 10 * t); });
    HIPCHECK(c, hipGetLastError());
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->steps += n;
    const bool used[5] = {true, c->L.boundary,
                          c->L.boundary && (c->L.inlet_early ? 0 : c->L.nb_in) + c->L.nb_out > 0,
                          c->L.boundary && c->L.nb_out > 0, c->L.psi_mode != 0};
    for (int k = 0; k < 5; k++) {
        double acc = 0.0;
        if (used[k])
            for (int64_t t = 0; t < n; t++) {
                float v = 0.0f;
                HIPCHECK(c, hipEventElapsedTime(&v, ev[10 * t + 2 * k], ev[10 * t + 2 * k + 1]));
                acc += v;
            }
        ms[k] = used[k] ? acc / (double)n : 0.0;
    }
    for (auto &e : ev) HIPCHECK(c, hipEventDestroy(e));
    return LBM_OK;
}

int lbm_tile_configs(int dim) { return (dim == 2 || dim == 3) ? n_tile_cfg(dim) : 0; }

lbm_status lbm_tile_config_desc(int dim, int i, int *out)
{
    if (!out || (dim != 2 && dim != 3) || i < 0 || i >= n_tile_cfg(dim)) return LBM_EINVAL;
    const TileCfg &t = tile_cfg(dim, i);
    out[0] = t.psrc;
    out[1] = t.tx;
    out[2] = t.ty;
    out[3] = t.w;
    out[4] = t.zc;
    out[5] = t.keepb;
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : -1; }

void lbm_destroy(lbm_ctx *c) { delete c; }

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

struct lbm_batch {
    std::vector<lbm_ctx *> m;
    int dim = 0, storage = 0, cfg = 0;
    BatchTab tab{};
    unsigned g_psi = 0, g_main = 0, g_chi = 0, g_out = 0, g_inl = 0, g_fill = 0;
    hipStream_t stream = nullptr;
    int cur = 0;
    int64_t steps = 0;
    std::string err;
    int graph_steps = 16;
    hipStream_t cap = nullptr;
    hipGraphExec_t gx[2] = {nullptr, nullptr};
    ~lbm_batch()
    {
        for (auto &g : gx)
            if (g) (void)hipGraphExecDestroy(g);
        if (cap) (void)hipStreamDestroy(cap);
        for (auto *c : m) delete c;
    }
};

namespace {

thread_local std::string g_batch_error;

lbm_status bfail(lbm_batch *b, lbm_status st, const std::string &msg)
{
    if (b) b->err = msg;
    else g_batch_error = msg;
    return st;
}

#define BHIPCHECK(b, call)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return bfail(b, LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

// Member configurations as the batch builds them: the batch's node-update
// configuration everywhere.  Returns the per-member workspace sizes (0 = invalid).
std::string batch_plan(const lbm_config *cfgs, int n, std::vector<lbm_config> &mc, std::vector<size_t> &bytes,
                       size_t &tables, size_t &total)
{
    if (!cfgs || n < 1 || n > (1 << 20)) return "bad member count";
    mc.assign(cfgs, cfgs + n);
    bytes.assign(n, 0);
    const int cfg = cfgs[0].tile_config;
    total = 0;
    int64_t items = 0;
    for (int i = 0; i < n; i++) {
        if (mc[i].dim != mc[0].dim || mc[i].storage != mc[0].storage)
            return "batch members must share the lattice and the storage";
        mc[i].tile_config = cfg;
        Canon k;
        std::string why = canonicalize(&mc[i], k);
        Maps m;
        if (why.empty()) why = build_maps(&k.c, m);
        if (!why.empty()) return "member " + std::to_string(i) + ": " + why;
        const Layout L = make_layout(k, m);
        bytes[i] = L.total;
        items += (int64_t)L.item_list.size();
        total += align_up(bytes[i]);
    }
    if (items > INT32_MAX) return "too many node-update work items";
    tables = align_up(sizeof(Member) * n) + 5 * align_up(sizeof(int) * (n + 1)) +
             align_up(sizeof(int) * std::max<int64_t>(items, 1));
    total += tables;
    return "";
}

void batch_launch(lbm_batch *b, hipStream_t s)
{
    BatchArgs a{};
    a.t = b->tab;
    a.cur = b->cur;
    a.g_psi = b->g_psi;
    a.g_main = b->g_main;
    a.g_chi = b->g_chi;
    a.g_out = b->g_out;
    a.g_inl = b->g_inl;
    a.g_fill = b->g_fill;
    a.stream = s;
    if (b->dim == 2) Launcher<2>::batch_step(b->storage, b->cfg, a);
    else Launcher<3>::batch_step(b->storage, b->cfg, a);
    b->cur ^= 1;
}

// Captures graph_steps batch steps starting from parity `parity` into gx[parity].
lbm_status batch_capture(lbm_batch *b, int parity)
{
    const int G = b->graph_steps;
    hipGraphExec_t &gx = b->gx[parity];
    if (gx || G <= 0) return LBM_OK;
    if (!b->cap) BHIPCHECK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    const int cur = b->cur;
    b->cur = parity;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int t = 0; t < G; t++) batch_launch(b, b->cap);
        e = hipStreamEndCapture(b->cap, &graph);
    }
    b->cur = cur;
    if (e == hipSuccess) e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch graph: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_config *cfgs, int n)
{
    std::vector<lbm_config> mc;
    std::vector<size_t> bytes;
    size_t tables = 0, total = 0;
    if (!batch_plan(cfgs, n, mc, bytes, tables, total).empty()) return 0;
    return total;
}

lbm_status lbm_batch_create(const lbm_config *cfgs, int n, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            lbm_batch **out)
{
    if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    std::vector<lbm_config> mc;
    std::vector<size_t> bytes;
    size_t tables = 0, total = 0;
    const std::string why = batch_plan(cfgs, n, mc, bytes, tables, total);
    if (!why.empty()) return bfail(nullptr, LBM_EINVAL, why);
    if (!dev_ws) return bfail(nullptr, LBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)dev_ws) % ALIGN) return bfail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < total) return bfail(nullptr, LBM_ENOMEM, "workspace too small");
    lbm_batch *b = new lbm_batch();
    b->stream = (hipStream_t)hip_stream;
    b->dim = mc[0].dim;
    b->storage = mc[0].storage;
    char *ws = (char *)dev_ws;
    size_t off = 0;
    std::vector<Member> mem(n);
    std::vector<int> item0(n + 1, 0), psi0(n + 1, 0), out0(n + 1, 0), inl0(n + 1, 0), fill0(n + 1, 0);
    bool faces = false;
    for (int i = 0; i < n; i++) {
        lbm_ctx *c = nullptr;
        const lbm_status st = lbm_create(&mc[i], ws + off, bytes[i], hip_stream, &c);
        if (st != LBM_OK) {
            const std::string msg = "member " + std::to_string(i) + ": " + g_create_error;
            delete b;
            return bfail(nullptr, st, msg);
        }
        b->m.push_back(c);
        off += align_up(bytes[i]);
        const Layout &L = c->L;
        b->cfg = L.cfg;
        Member &M = mem[i];
        M.f[0] = c->ws + L.o_fA;
        M.f[1] = c->ws + L.o_fB;
        M.type = c->type();
        M.psi[0] = c->ws + L.o_psi[0];
        M.psi[1] = c->ws + L.o_psi[1];
        M.g = L.g;
        M.ph = c->ph;
        M.bd = c->bd;
        M.tiles_x = L.tiles[0];
        M.tiles_y = L.tiles[1];
        M.n_items = (int)L.nblocks_main;
        M.item_list = (const int *)(c->ws + L.o_items);
        M.nb_in = L.nb_in;
        M.nb_out = L.nb_out;
        M.flag = c->flag();
        const bool chi_stage = L.boundary && c->bd.has_outlet && c->bd.chi_on;
        item0[i + 1] = item0[i] + M.n_items;
        psi0[i + 1] = psi0[i] + (L.psi_mode ? (int)((L.g.N + 255) / 256) : 0);
        out0[i + 1] = out0[i] + (chi_stage ? L.nb_out : 0);
        inl0[i + 1] = inl0[i] + (L.boundary ? L.nb_in + L.nb_out : 0);
        fill0[i + 1] = fill0[i] + (L.boundary ? L.nb_out : 0);
        faces = faces || L.boundary;
    }
    char *t = ws + off;
    auto put = [&](const void *src, size_t nbytes) -> char * {
        char *at = t;
        t += align_up(nbytes);
        return hipMemcpyAsync(at, src, nbytes, hipMemcpyHostToDevice, b->stream) == hipSuccess ? at : nullptr;
    };
    b->tab.n = n;
    b->tab.m = (const Member *)put(mem.data(), sizeof(Member) * n);
    b->tab.item0 = (const int *)put(item0.data(), sizeof(int) * (n + 1));
    std::vector<int> item_mem(std::max(item0[n], 1), 0);
    for (int i = 0; i < n; i++)
        for (int w = item0[i]; w < item0[i + 1]; w++) item_mem[w] = i;
    b->tab.item_mem = (const int *)put(item_mem.data(), sizeof(int) * item_mem.size());
    b->tab.psi0 = (const int *)put(psi0.data(), sizeof(int) * (n + 1));
    b->tab.out0 = (const int *)put(out0.data(), sizeof(int) * (n + 1));
    b->tab.inl0 = (const int *)put(inl0.data(), sizeof(int) * (n + 1));
    b->tab.fill0 = (const int *)put(fill0.data(), sizeof(int) * (n + 1));
    if (!b->tab.m || !b->tab.item0 || !b->tab.item_mem || !b->tab.psi0 || !b->tab.out0 || !b->tab.inl0 ||
        !b->tab.fill0) {
        delete b;
        return bfail(nullptr, LBM_EDEVICE, "upload of the batch tables failed");
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        delete b;
        return bfail(nullptr, LBM_EDEVICE, "batch set-up failed");
    }
    // launch sizes: the node update is persistent, at most two blocks per
    // resident slot (256 CUs x 4 blocks), a multiple of the 8 XCDs
    const int items = item0[n];
    b->g_main = (unsigned)std::min((items + 7) / 8 * 8, 2048);
    b->g_psi = (unsigned)psi0[n];
    b->g_chi = faces ? (unsigned)((n + 63) / 64) : 0u;
    b->g_out = (unsigned)out0[n];
    b->g_inl = (unsigned)inl0[n];
    b->g_fill = (unsigned)fill0[n];
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t n)
{
    if (!b || n < 0) return bfail(b, LBM_EINVAL, "bad arguments to lbm_batch_step");
    for (auto *c : b->m) {
        if (c->unstable) return bfail(b, LBM_ESTATE, "a member is flagged unstable");
        if (c->cur != b->cur) return bfail(b, LBM_ESTATE, "a member was stepped on its own; parities differ");
    }
    const int64_t n0 = n;
    const int G = b->graph_steps;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    BHIPCHECK(b, hipStreamIsCapturing(b->stream, &cs));
    if (cs != hipStreamCaptureStatusNone && n % 2)
        return bfail(b, LBM_EINVAL, "a captured lbm_batch_step must enqueue an even number of steps");
    if (G > 0 && cs == hipStreamCaptureStatusNone) {
        while (n >= G) {
            hipGraphExec_t &gx = b->gx[b->cur];
            if (!gx) {
                const lbm_status st = batch_capture(b, b->cur);
                if (st != LBM_OK) return st;
            }
            BHIPCHECK(b, hipGraphLaunch(gx, b->stream));
            if (G % 2) b->cur ^= 1;
            n -= G;
        }
    }
    for (int64_t t = 0; t < n; t++) batch_launch(b, b->stream);
    BHIPCHECK(b, hipGetLastError());
    b->steps += n0;
    for (auto *c : b->m) {
        c->cur = b->cur;
        c->steps += n0;
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_graph_steps(lbm_batch *b, int steps_per_graph)
{
    if (!b || steps_per_graph < 0 || steps_per_graph > 4096) return bfail(b, LBM_EINVAL, "bad steps per graph");
    for (auto &g : b->gx)
        if (g) {
            BHIPCHECK(b, hipGraphExecDestroy(g));
            g = nullptr;
        }
    b->graph_steps = steps_per_graph;
    for (int p = 0; p < 2 && steps_per_graph > 0; p++) {
        const lbm_status st = batch_capture(b, p);
        if (st != LBM_OK) return st;
        BHIPCHECK(b, hipGraphUpload(b->gx[p], b->stream));
    }
    return LBM_OK;
}

int lbm_batch_size(const lbm_batch *b) { return b ? (int)b->m.size() : 0; }

lbm_ctx *lbm_batch_member(lbm_batch *b, int i)
{
    if (!b || i < 0 || i >= (int)b->m.size()) return nullptr;
    return b->m[i];
}

void lbm_batch_destroy(lbm_batch *b) { delete b; }

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Droplet labels
// ---------------------------------------------------------------------------

namespace {

// caller-frame box -> memory-frame box; empty string if valid
std::string to_box(const lbm_ctx *c, const lbm_box *in, Box3 &bx)
{
    if (!in) return "box is NULL";
    const Geometry &g = c->L.g;
    for (int a = 0; a < 3; a++) {
        const int ca = g.ax[a];
        bx.lo[a] = in->lo[ca];
        bx.hi[a] = in->hi[ca];
        if (bx.lo[a] < 0 || bx.hi[a] > g.n[a] || bx.lo[a] > bx.hi[a]) return "box outside the domain";
    }
    return "";
}

}  // namespace

extern "C" {

lbm_status lbm_probe(lbm_ctx *c, int k, const lbm_box *box, double threshold, int64_t *dev_count)
{
    if (!c || (k != 0 && k != 1) || !dev_count) return fail(c, LBM_EINVAL, "bad arguments to lbm_probe");
    Box3 bx{};
    const std::string why = to_box(c, box, bx);
    if (!why.empty()) return fail(c, LBM_EINVAL, why);
    const StepArgs a = step_args(c);
    auto *out = (unsigned long long *)dev_count;
    if (c->L.dim == 2) Launcher<2>::probe(c->L.storage, a, k, bx, (float)threshold, out);
    else Launcher<3>::probe(c->L.storage, a, k, bx, (float)threshold, out);
    HIPCHECK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_components(lbm_ctx *c, int k, const lbm_box *box, double threshold, lbm_component *out, int max_out,
                          int *n_out)
{
    if (!c || (k != 0 && k != 1) || !n_out || max_out < 0 || (max_out > 0 && !out))
        return fail(c, LBM_EINVAL, "bad arguments to lbm_components");
    Box3 bx{};
    const std::string why = to_box(c, box, bx);
    if (!why.empty()) return fail(c, LBM_EINVAL, why);
    const StepArgs a = step_args(c);
    const int64_t N = c->L.g.N;
    int *lab = nullptr, *slot = nullptr, *flags = nullptr;
    CompStat *st = nullptr;
    auto release = [&]() {
        if (lab) (void)hipFree(lab);
        if (slot) (void)hipFree(slot);
        if (flags) (void)hipFree(flags);
        if (st) (void)hipFree(st);
    };
    auto run = [&]() -> lbm_status {
        HIPCHECK(c, hipMalloc(&lab, (size_t)N * 4));
        HIPCHECK(c, hipMalloc(&slot, (size_t)N * 4));
        HIPCHECK(c, hipMalloc(&flags, 8));
        const bool d2 = c->L.dim == 2;
        if (d2) Launcher<2>::lab_init(c->L.storage, a, k, bx, (float)threshold, lab);
        else Launcher<3>::lab_init(c->L.storage, a, k, bx, (float)threshold, lab);
        // propagate until no label changes (at most N rounds; pointer jumping
        // makes it a few dozen in practice)
        for (int64_t round = 0;; round++) {
            if (round > N) return fail(c, LBM_EDEVICE, "label propagation did not converge");
            HIPCHECK(c, hipMemsetAsync(flags, 0, 4, c->stream));
            if (d2) Launcher<2>::lab_prop(a, lab, flags, 4);
            else Launcher<3>::lab_prop(a, lab, flags, 4);
            int changed = 0;
            HIPCHECK(c, hipMemcpyAsync(&changed, flags, 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHECK(c, hipStreamSynchronize(c->stream));
            if (!changed) break;
        }
        HIPCHECK(c, hipMemsetAsync(flags + 1, 0, 4, c->stream));
        if (d2) Launcher<2>::lab_roots(a, lab, slot, flags + 1);
        else Launcher<3>::lab_roots(a, lab, slot, flags + 1);
        int nr = 0;
        HIPCHECK(c, hipMemcpyAsync(&nr, flags + 1, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        *n_out = nr;
        if (nr == 0) return LBM_OK;
        HIPCHECK(c, hipMalloc(&st, sizeof(CompStat) * nr));
        if (d2) Launcher<2>::lab_stats(a, lab, slot, st, nr);
        else Launcher<3>::lab_stats(a, lab, slot, st, nr);
        std::vector<CompStat> h(nr);
        HIPCHECK(c, hipMemcpyAsync(h.data(), st, sizeof(CompStat) * nr, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        std::sort(h.begin(), h.end(), [](const CompStat &p, const CompStat &q) { return p.first < q.first; });
        for (int i = 0; i < nr && i < max_out; i++) {
            out[i].first = (int64_t)h[i].first;
            out[i].size = (int64_t)h[i].size;
            for (int d = 0; d < 3; d++) {
                out[i].lo[d] = h[i].lo[d];
                out[i].hi[d] = h[i].hi[d];
            }
        }
        return LBM_OK;
    };
    const lbm_status r = run();
    release();
    return r;
}

lbm_status lbm_components_static(lbm_ctx *c, int k, const lbm_box *box, double threshold, lbm_component *out,
                                 int max_out, int *n_out)
{
    if (!c || (k != 0 && k != 1) || !n_out || max_out < 0 || (max_out > 0 && !out))
        return fail(c, LBM_EINVAL, "bad arguments to lbm_components_static");
    Box3 bx{};
    const std::string why = to_box(c, box, bx);
    if (!why.empty()) return fail(c, LBM_EINVAL, why);
    const int64_t N = c->L.g.N;
    if (N > LBM_COMPONENTS_STATIC_MAX_NODES)
        return fail(c, LBM_EINVAL, "domain has more nodes than the static labelling scratch holds (" +
                                       std::to_string(N) + " > " + std::to_string(LBM_COMPONENTS_STATIC_MAX_NODES) + ")");
    int dev = -1;
    HIPCHECK(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, LBM_EINVAL, "the context's device is not the current device");
    char *base = (char *)static_scratch_ptr(dev);
    if (!base) return fail(c, LBM_EDEVICE, "static scratch not resolved on this device");
    int *lab = (int *)(base + SCR_LAB);
    int *slot = (int *)(base + SCR_SLOT);
    int *flags = (int *)(base + SCR_FLAGS);
    CompStat *st = (CompStat *)(base + SCR_STATS);
    lbm_component *sorted = (lbm_component *)(base + SCR_SORTED);
    const StepArgs a = step_args(c);
    const bool d2 = c->L.dim == 2;
    if (d2) Launcher<2>::lab_init(c->L.storage, a, k, bx, (float)threshold, lab);
    else Launcher<3>::lab_init(c->L.storage, a, k, bx, (float)threshold, lab);
    for (int64_t round = 0;; round++) {
        if (round > N) return fail(c, LBM_EDEVICE, "label propagation did not converge");
        HIPCHECK(c, hipMemsetAsync(flags, 0, 4, c->stream));
        if (d2) Launcher<2>::lab_prop(a, lab, flags, 4);
        else Launcher<3>::lab_prop(a, lab, flags, 4);
        int changed = 0;
        HIPCHECK(c, hipMemcpyAsync(&changed, flags, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        if (!changed) break;
    }
    HIPCHECK(c, hipMemsetAsync(flags + 1, 0, 4, c->stream));
    if (d2) Launcher<2>::lab_roots(a, lab, slot, flags + 1);
    else Launcher<3>::lab_roots(a, lab, slot, flags + 1);
    int nr = 0;
    HIPCHECK(c, hipMemcpyAsync(&nr, flags + 1, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    if (nr > LBM_COMPONENTS_STATIC_MAX_COMPONENTS)
        return fail(c, LBM_EINVAL, "more components than the static labelling scratch holds (" + std::to_string(nr) +
                                       " > " + std::to_string(LBM_COMPONENTS_STATIC_MAX_COMPONENTS) + ")");
    *n_out = nr;
    if (nr == 0) return LBM_OK;
    if (d2) Launcher<2>::lab_stats(a, lab, slot, st, nr);
    else Launcher<3>::lab_stats(a, lab, slot, st, nr);
    hipLaunchKernelGGL(k_lab_order, dim3((nr + 255) / 256), dim3(256), 0, c->stream, st, nr, sorted);
    HIPCHECK(c, hipGetLastError());
    const int nc = std::min(nr, max_out);
    if (nc > 0)
        HIPCHECK(c, hipMemcpyAsync(out, sorted, sizeof(lbm_component) * nc, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // extern "C"
