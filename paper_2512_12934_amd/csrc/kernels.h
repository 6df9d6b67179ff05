// kernels.h -- device kernels of one lattice step (pull scheme).
//
// Storage.  Each population plane holds, at node x, the post-collision value
// f*_i(x, t) (not yet streamed), over a box padded by one node on every
// lattice axis; the padding holds the populations the open boundaries supply.
// The post-streaming distribution of eq. (2) is obtained by a gather:
//     f_i(x, t+1) = f*_i(x - e_i, t)        (periodic axes wrap)
//     f_i(x, t+1) = f*_ibar(x, t)           if x - e_i is solid (eq. B1)
//     f_i(x, t+1) = padding slot at x - e_i if that lies beyond an open face
// Two arrays alternate between source and destination every step.
//
// One step is four launches:
//   k_main           all fluid nodes: densities of the tile plus a two-node
//                    halo into LDS (mirror ghost layers at open faces,
//                    eqs. 24-25), force (eqs. 10-11), common velocity
//                    (eqs. 7-8), MRT collision (eq. 1); FP64 partial mass
//                    flows at inlet nodes and the x_{N-1} column (eq. 23)
//   k_outlet         chi = Q_in / Q' (eq. 23) and the collision of the outlet
//                    column with the corrected normal velocity (eq. 22)
//   k_inlet          alpha-corrected NEQ extrapolation (eqs. 13-19) into the
//                    padding slots; partial sums of eq. (21)
//   k_outlet_fill    convective outflow (eq. 20) into the padding slots
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.h"
#include "params.h"

namespace lbm {

// ---------------------------------------------------------------------------
// storage codecs: FP32, or binary16 of (f - w_i) with round-to-nearest-even
// ---------------------------------------------------------------------------
template <int STORE> struct Codec;
template <> struct Codec<0> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p, float) { return *p; }
    static __device__ __forceinline__ void st(T *p, float v, float) { *p = v; }
};
template <> struct Codec<1> {
    using T = __half;
    static __device__ __forceinline__ float ld(const T *p, float w) { return __half2float(*p) + w; }
    static __device__ __forceinline__ void st(T *p, float v, float w) { *p = __float2half_rn(v - w); }
};

__device__ __forceinline__ int64_t pidx(const Geometry &g, int x, int y, int z)
{
    return (int64_t)(x + 1) + (int64_t)g.P[0] * ((int64_t)(y + 1) + (int64_t)g.P[1] * (int64_t)(z + 1));
}

template <int DIM>
__device__ __forceinline__ int64_t dir_off(const Geometry &g, int i)
{
    return (int64_t)Lat<DIM>::E[i][0] + (int64_t)g.P[0] * ((int64_t)Lat<DIM>::E[i][1] +
                                                          (int64_t)g.P[1] * (int64_t)Lat<DIM>::E[i][2]);
}

// Padded index of the slot that supplies population i at box node (x,y,z)
// when no bounce-back applies: x - e_i with periodic wrap.
template <int DIM>
__device__ __forceinline__ int64_t src_slot(const Geometry &g, int x, int y, int z, int i)
{
    int s[3] = {x - Lat<DIM>::E[i][0], y - Lat<DIM>::E[i][1], z - Lat<DIM>::E[i][2]};
#pragma unroll
    for (int a = 0; a < DIM; a++) {
        if (g.periodic[a]) {
            if (s[a] < 0) s[a] += g.n[a];
            else if (s[a] >= g.n[a]) s[a] -= g.n[a];
        }
    }
    if (DIM == 2) s[2] = -1;
    return pidx(g, s[0], s[1], s[2]);
}

// Post-streaming populations of one component at one node.
template <int DIM, int STORE>
__device__ __forceinline__ void gather(const typename Codec<STORE>::T *__restrict__ fk, const Geometry &g,
                                       int64_t p, uint32_t tw, int x, int y, int z,
                                       float (&f)[Lat<DIM>::Q])
{
    constexpr int Q = Lat<DIM>::Q;
    if (!(tw & T_EDGE)) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const bool bb = (tw >> i) & 1u;
            const int64_t a = bb ? (int64_t)Lat<DIM>::OPP[i] * g.Ppad + p
                                 : (int64_t)i * g.Ppad + p - dir_off<DIM>(g, i);
            f[i] = Codec<STORE>::ld(fk + a, weight<DIM>(i));
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const bool bb = (tw >> i) & 1u;
            const int64_t a = bb ? (int64_t)Lat<DIM>::OPP[i] * g.Ppad + p
                                 : (int64_t)i * g.Ppad + src_slot<DIM>(g, x, y, z, i);
            f[i] = Codec<STORE>::ld(fk + a, weight<DIM>(i));
        }
    }
}

// Single post-streaming population i of one component.
template <int DIM, int STORE>
__device__ __forceinline__ float gather1(const typename Codec<STORE>::T *__restrict__ fk, const Geometry &g,
                                         int64_t p, uint32_t tw, int x, int y, int z, int i)
{
    const bool bb = (tw >> i) & 1u;
    const int64_t a = bb ? (int64_t)Lat<DIM>::OPP[i] * g.Ppad + p
                         : (int64_t)i * g.Ppad + src_slot<DIM>(g, x, y, z, i);
    return Codec<STORE>::ld(fk + a, weight<DIM>(i));
}

__device__ __forceinline__ void coords_of(const Geometry &g, int64_t b, int &x, int &y, int &z)
{
    x = (int)(b % g.n[0]);
    y = (int)((b / g.n[0]) % g.n[1]);
    z = (int)(b / ((int64_t)g.n[0] * g.n[1]));
}

// Maps a halo coordinate onto the box: periodic axes wrap; beyond a
// non-periodic face the mirror image about that face (ghost layers of
// eqs. 24-25: the first ghost copies the face node, the second its neighbour).
__device__ __forceinline__ int map_axis(int v, int n, int periodic)
{
    if (v < 0) return periodic ? v + n : -1 - v;
    if (v >= n) return periodic ? v - n : 2 * n - 1 - v;
    return v;
}

// Deterministic block-wide sum of two doubles (256 threads, 4 waves).
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red /*[8]*/)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    __syncthreads();
    if (ln == 0) { red[2 * wv] = a; red[2 * wv + 1] = b; }
    __syncthreads();
    a = (red[0] + red[2]) + (red[4] + red[6]);
    b = (red[1] + red[3]) + (red[5] + red[7]);
}

// Deterministic sum of a partials array [n][2] by every block (fixed order).
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int n, double &a, double &b,
                                                double *red)
{
    a = 0.0;
    b = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    block_sum2(a, b, red);
}

enum { MODE_STEP = 0, MODE_MOMENTS = 1 };

// ---------------------------------------------------------------------------
// k_main: the fused per-node update over a TX x TY x TZ tile.
// ---------------------------------------------------------------------------
template <int DIM, int STORE, int MODE, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_main(const typename Codec<STORE>::T *__restrict__ src,
                                              typename Codec<STORE>::T *__restrict__ dst,
                                              const uint32_t *__restrict__ type, Geometry g, Physics ph,
                                              Boundary bd, int tiles_x, int tiles_y,
                                              double *__restrict__ out_rho, double *__restrict__ out_u,
                                              int *__restrict__ flag)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    constexpr int HX = TX + 4, HY = TY + 4, HZ = DIM == 3 ? TZ + 4 : 1;
    constexpr int NH = HX * HY * HZ;
    constexpr int NT = TX * TY * (DIM == 3 ? TZ : 1);
    __shared__ float2 s_psi[NH];
    __shared__ uint8_t s_sol[NH];
    __shared__ double s_red[8];

    const int tile = blockIdx.x;
    const int tx = tile % tiles_x;
    const int ty = (tile / tiles_x) % tiles_y;
    const int tz = tile / (tiles_x * tiles_y);
    const int x0 = tx * TX, y0 = ty * TY, z0 = DIM == 3 ? tz * TZ : 0;
    const T *src1 = src + (int64_t)Q * g.Ppad;

    // ---- stage 1: psi_k = rho_k over the tile and its halo (0 on solids)
    for (int h = threadIdx.x; h < NH; h += 256) {
        const int lx = h % HX, ly = (h / HX) % HY, lz = h / (HX * HY);
        int gx = x0 - 2 + lx, gy = y0 - 2 + ly, gz = DIM == 3 ? z0 - 2 + lz : 0;
        float p1 = 0.0f, p2 = 0.0f;
        uint8_t sol = 1;
        const bool need = gx < g.n[0] + 2 && gy < g.n[1] + 2 && (DIM == 2 || gz < g.n[2] + 2);
        if (need) {
            gx = map_axis(gx, g.n[0], g.periodic[0]);
            gy = map_axis(gy, g.n[1], g.periodic[1]);
            if (DIM == 3) gz = map_axis(gz, g.n[2], g.periodic[2]);
            const int64_t b = (int64_t)gx + (int64_t)g.n[0] * ((int64_t)gy + (int64_t)g.n[1] * gz);
            const uint32_t tw = type[b];
            if (!(tw & T_SOLID)) {
                const int64_t p = pidx(g, gx, gy, DIM == 3 ? gz : -1);
                float f[Q];
                gather<DIM, STORE>(src, g, p, tw, gx, gy, gz, f);
                float r = 0.0f;
#pragma unroll
                for (int i = 0; i < Q; i++) r += f[i];
                p1 = r;
                gather<DIM, STORE>(src1, g, p, tw, gx, gy, gz, f);
                r = 0.0f;
#pragma unroll
                for (int i = 0; i < Q; i++) r += f[i];
                p2 = r;
                sol = 0;
            }
        }
        s_psi[h] = make_float2(p1, p2);
        s_sol[h] = sol;
    }
    __syncthreads();

    double q_in = 0.0, q_out = 0.0;
    for (int q = threadIdx.x; q < NT; q += 256) {
        const int lx = q % TX, ly = (q / TX) % TY, lz = DIM == 3 ? q / (TX * TY) : 0;
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (x >= g.n[0] || y >= g.n[1] || (DIM == 3 && z >= g.n[2])) continue;
        const int64_t b = (int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)g.n[1] * z);
        const uint32_t tw = type[b];
        if (tw & T_SOLID) {
            if (MODE == MODE_MOMENTS) {
                out_rho[b] = 0.0;
                out_rho[g.N + b] = 0.0;
                for (int d = 0; d < 3; d++) out_u[d * g.N + b] = 0.0;
            }
            continue;
        }
        const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
        const int hc = ((DIM == 3 ? lz + 2 : 0) * HY + ly + 2) * HX + lx + 2;
        const float2 ps = s_psi[hc];

        // ---- stage 2: forces (eqs. 10-11) and body force
        float g1[3] = {0.f, 0.f, 0.f}, g2[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f};
        const bool near = ph.adhesion && (tw & T_NEARWALL);
#pragma unroll
        for (int dz = (DIM == 3 ? -2 : 0); dz <= (DIM == 3 ? 2 : 0); dz++)
#pragma unroll
            for (int dy = -2; dy <= 2; dy++)
#pragma unroll
                for (int dx = -2; dx <= 2; dx++) {
                    const int r2 = dx * dx + dy * dy + dz * dz;
                    const float w = stencil_w<DIM>(r2);
                    if (r2 == 0 || w == 0.0f) continue;
                    const int ho = (dz * HY + dy) * HX + dx;
                    const float2 v = s_psi[hc + ho];
                    if (dx) { g1[0] = fmaf(w * dx, v.x, g1[0]); g2[0] = fmaf(w * dx, v.y, g2[0]); }
                    if (dy) { g1[1] = fmaf(w * dy, v.x, g1[1]); g2[1] = fmaf(w * dy, v.y, g2[1]); }
                    if (dz) { g1[2] = fmaf(w * dz, v.x, g1[2]); g2[2] = fmaf(w * dz, v.y, g2[2]); }
                }
        if (near) {
#pragma unroll
            for (int dz = (DIM == 3 ? -2 : 0); dz <= (DIM == 3 ? 2 : 0); dz++)
#pragma unroll
                for (int dy = -2; dy <= 2; dy++)
#pragma unroll
                    for (int dx = -2; dx <= 2; dx++) {
                        const int r2 = dx * dx + dy * dy + dz * dz;
                        const float w = stencil_w<DIM>(r2);
                        if (r2 == 0 || w == 0.0f) continue;
                        const int ho = (dz * HY + dy) * HX + dx;
                        const float sv = (float)s_sol[hc + ho];
                        if (dx) A[0] = fmaf(w * dx, sv, A[0]);
                        if (dy) A[1] = fmaf(w * dy, sv, A[1]);
                        if (dz) A[2] = fmaf(w * dz, sv, A[2]);
                    }
        }
        const float r1 = ps.x, r2 = ps.y, rt = r1 + r2;
        float F1[3], F2[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            F1[d] = -ph.G12 * r1 * g2[d] - ph.Gw[0] * r1 * A[d] + (r1 / rt) * ph.Fb[d];
            F2[d] = -ph.G12 * r2 * g1[d] - ph.Gw[1] * r2 * A[d] + (r2 / rt) * ph.Fb[d];
        }

        // ---- stage 3: common velocity (eqs. 7-8)
        float fa[Q], fb[Q];
        gather<DIM, STORE>(src, g, p, tw, x, y, z, fa);
        gather<DIM, STORE>(src1, g, p, tw, x, y, z, fb);
        float J1[3] = {0.f, 0.f, 0.f}, J2[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < Q; i++) {
#pragma unroll
            for (int d = 0; d < DIM; d++) {
                const int e = Lat<DIM>::E[i][d];
                if (e == 1) { J1[d] += fa[i]; J2[d] += fb[i]; }
                else if (e == -1) { J1[d] -= fa[i]; J2[d] -= fb[i]; }
            }
        }
        float u[3];
        const float irt = 1.0f / rt;
#pragma unroll
        for (int d = 0; d < 3; d++) u[d] = (J1[d] + J2[d] + 0.5f * (F1[d] + F2[d])) * irt;

        if (MODE == MODE_MOMENTS) {
            out_rho[b] = r1;
            out_rho[g.N + b] = r2;
            for (int d = 0; d < 3; d++) out_u[d * g.N + b] = u[d];
            continue;
        }
        if (!(rt > 0.0f) || !isfinite(rt) || !isfinite(u[0] + u[1] + u[2])) *flag = 1;

        if (tw & T_ROLE) {
            const int slot = bd.bslot[b];
            float *fF = bd.faceF + (int64_t)slot * 6;
#pragma unroll
            for (int d = 0; d < 3; d++) { fF[d] = F1[d]; fF[3 + d] = F2[d]; }
            if (tw & T_XPRIME) {
                const float un = bd.out_sign * u[bd.out_axis];
                bd.faceU[slot] = un;
                q_out += (double)rt * (double)un;
            }
            if (tw & T_INLET) {
                const Patch &pt = bd.patch[(tw & T_PATCH_MASK) >> T_PATCH_SHIFT];
                q_in += (double)rt * (double)(pt.sign * u[pt.axis]);
            }
            if ((tw & T_OUTLET) && bd.chi_on) continue;   // collided by k_outlet
        }

        // ---- stage 5: MRT collision of each component, stored at x
        {
            const Rates s1 = {ph.se[0], ph.seps[0], ph.sq, ph.snu[0]};
            collide<DIM>(fa, r1, J1, u, F1, s1);
            T *d1 = dst;
#pragma unroll
            for (int i = 0; i < Q; i++) Codec<STORE>::st(d1 + (int64_t)i * g.Ppad + p, fa[i], weight<DIM>(i));
            const Rates s2 = {ph.se[1], ph.seps[1], ph.sq, ph.snu[1]};
            collide<DIM>(fb, r2, J2, u, F2, s2);
            T *d2 = dst + (int64_t)Q * g.Ppad;
#pragma unroll
            for (int i = 0; i < Q; i++) Codec<STORE>::st(d2 + (int64_t)i * g.Ppad + p, fb[i], weight<DIM>(i));
        }
    }
    if (MODE == MODE_STEP && bd.qpart) {
        block_sum2(q_in, q_out, s_red);
        if (threadIdx.x == 0) {
            bd.qpart[2 * blockIdx.x] = q_in;
            bd.qpart[2 * blockIdx.x + 1] = q_out;
        }
    }
}

// chi of eq. (23); undefined (no outflow through x_{N-1}, or flow against the
// inlets) leaves the outlet uncorrected.
__device__ __forceinline__ double chi_of(double qin, double qout)
{
    return (fabs(qout) < 1e-30 || qin * qout <= 0.0) ? 1.0 : qin / qout;
}

// ---------------------------------------------------------------------------
// k_outlet: eq. (23) and the collision of the outlet column with eq. (22).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_outlet(const typename Codec<STORE>::T *__restrict__ src,
                                                typename Codec<STORE>::T *__restrict__ dst,
                                                const uint32_t *__restrict__ type, Geometry g, Physics ph,
                                                Boundary bd, int *__restrict__ flag)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[8];
    double qin, qout;
    reduce_partials(bd.qpart, bd.n_qpart, qin, qout, s_red);
    const double chi = chi_of(qin, qout);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bd.scal[SC_QIN] = qin;
        bd.scal[SC_QOUT] = qout;
        bd.scal[SC_CHI] = (bd.has_outlet && bd.chi_on) ? chi : 1.0;
    }
    if (!bd.has_outlet || !bd.chi_on) return;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= bd.n_out) return;
    const OutletRec rec = bd.out[r];
    int x, y, z;
    coords_of(g, rec.bN, x, y, z);
    const uint32_t tw = type[rec.bN];
    const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
    float fa[Q], fb[Q];
    gather<DIM, STORE>(src, g, p, tw, x, y, z, fa);
    gather<DIM, STORE>(src + (int64_t)Q * g.Ppad, g, p, tw, x, y, z, fb);
    float r1 = 0.f, r2 = 0.f, J1[3] = {0.f, 0.f, 0.f}, J2[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < Q; i++) {
        r1 += fa[i];
        r2 += fb[i];
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            const int e = Lat<DIM>::E[i][d];
            if (e == 1) { J1[d] += fa[i]; J2[d] += fb[i]; }
            else if (e == -1) { J1[d] -= fa[i]; J2[d] -= fb[i]; }
        }
    }
    const float *fF = bd.faceF + (int64_t)rec.slotN * 6;
    float F1[3], F2[3], u[3];
    const float rt = r1 + r2;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        F1[d] = fF[d];
        F2[d] = fF[3 + d];
        u[d] = (J1[d] + J2[d] + 0.5f * (F1[d] + F2[d])) / rt;
    }
    if (rec.slotP >= 0) u[bd.out_axis] = (float)(chi * (double)(bd.out_sign * bd.faceU[rec.slotP])) * bd.out_sign;
    if (!(rt > 0.0f) || !isfinite(rt) || !isfinite(u[0] + u[1] + u[2])) *flag = 1;
    const Rates s1 = {ph.se[0], ph.seps[0], ph.sq, ph.snu[0]};
    collide<DIM>(fa, r1, J1, u, F1, s1);
    const Rates s2 = {ph.se[1], ph.seps[1], ph.sq, ph.snu[1]};
    collide<DIM>(fb, r2, J2, u, F2, s2);
    T *d2 = dst + (int64_t)Q * g.Ppad;
#pragma unroll
    for (int i = 0; i < Q; i++) {
        Codec<STORE>::st(dst + (int64_t)i * g.Ppad + p, fa[i], weight<DIM>(i));
        Codec<STORE>::st(d2 + (int64_t)i * g.Ppad + p, fb[i], weight<DIM>(i));
    }
}

// ---------------------------------------------------------------------------
// k_inlet: blocks [0, nb_in) rebuild the entering populations of the inlet
// nodes (eqs. 13-19); blocks [nb_in, ...) sum u.n_o over x_{N-1} (eq. 21).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_inlet(typename Codec<STORE>::T *__restrict__ dst,
                                               const uint32_t *__restrict__ type, Geometry g, Boundary bd,
                                               int nb_in)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[8];
    if ((int)blockIdx.x < nb_in) {
        const int r = blockIdx.x * 256 + threadIdx.x;
        if (r >= bd.n_in) return;
        const InletRec rec = bd.in[r];
        const Patch pt = bd.patch[rec.patch];
        int x1, y1, z1, x2, y2, z2;
        coords_of(g, rec.b1, x1, y1, z1);
        coords_of(g, rec.b2, x2, y2, z2);
        const uint32_t tw1 = type[rec.b1], tw2 = type[rec.b2];
        const int64_t p1 = pidx(g, x1, y1, DIM == 3 ? z1 : -1);
        const int64_t p2 = pidx(g, x2, y2, DIM == 3 ? z2 : -1);
        const bool x2_fluid = !(tw2 & T_SOLID);
        float up[3] = {0.f, 0.f, 0.f};
        up[pt.axis] = pt.sign * pt.u_n;
        // rho_k(x2), u(x2) from the streamed f at t+1 with this step's force
        float f2[2][Q], r2[2] = {0.f, 0.f}, u2[3] = {0.f, 0.f, 0.f};
        if (x2_fluid) {
            float J[3] = {0.f, 0.f, 0.f};
            const float *F2 = bd.faceF + (int64_t)rec.slot2 * 6;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                gather<DIM, STORE>(dst + (int64_t)k * Q * g.Ppad, g, p2, tw2, x2, y2, z2, f2[k]);
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    r2[k] += f2[k][i];
#pragma unroll
                    for (int d = 0; d < DIM; d++) J[d] += Lat<DIM>::E[i][d] * f2[k][i];
                }
            }
            const float rt = r2[0] + r2[1];
#pragma unroll
            for (int d = 0; d < 3; d++) u2[d] = (J[d] + 0.5f * (F2[d] + F2[3 + d])) / rt;
        }
        const float *F1 = bd.faceF + (int64_t)rec.slot1 * 6;
        for (int k = 0; k < 2; k++) {
            T *dk = dst + (int64_t)k * Q * g.Ppad;
            float f1[Q];
            gather<DIM, STORE>(dk, g, p1, tw1, x1, y1, z1, f1);
            // eq. (13)/(14) on the populations entering the domain
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if (Lat<DIM>::E[i][pt.axis] * pt.sign <= 0) continue;
                const float neq = x2_fluid ? f2[k][i] - feq<DIM>(i, r2[k], u2) : 0.0f;
                f1[i] = feq<DIM>(i, pt.rho[k], up) + neq;
            }
            if (pt.alpha_on) {
                // eqs. (15)-(19): alpha_i = w_i sum_d e_id dJ_d / D_d over the
                // entering set, dJ = rho_k^p u^p - (sum_i e_i f_i + F^k/2)
                float J[3] = {0.f, 0.f, 0.f}, D[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < Q; i++) {
#pragma unroll
                    for (int d = 0; d < DIM; d++) J[d] += Lat<DIM>::E[i][d] * f1[i];
                    if (Lat<DIM>::E[i][pt.axis] * pt.sign > 0) {
#pragma unroll
                        for (int d = 0; d < DIM; d++)
                            D[d] += weight<DIM>(i) * (float)(Lat<DIM>::E[i][d] * Lat<DIM>::E[i][d]);
                    }
                }
                float dJ[3];
#pragma unroll
                for (int d = 0; d < 3; d++) dJ[d] = pt.rho[k] * up[d] - (J[d] + 0.5f * F1[3 * k + d]);
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    if (Lat<DIM>::E[i][pt.axis] * pt.sign <= 0) continue;
                    float a = 0.0f;
#pragma unroll
                    for (int d = 0; d < DIM; d++)
                        if (Lat<DIM>::E[i][d] != 0) a += weight<DIM>(i) * Lat<DIM>::E[i][d] * dJ[d] / D[d];
                    f1[i] += a;
                }
            }
#pragma unroll
            for (int i = 0; i < Q; i++) {
                if (Lat<DIM>::E[i][pt.axis] * pt.sign <= 0) continue;
                Codec<STORE>::st(dk + (int64_t)i * g.Ppad + src_slot<DIM>(g, x1, y1, z1, i), f1[i], weight<DIM>(i));
            }
        }
        return;
    }
    // eq. (21): partial sums of the outward normal velocity over x_{N-1}
    const int r = (blockIdx.x - nb_in) * 256 + threadIdx.x;
    double su = 0.0, cnt = 0.0;
    if (r < bd.n_out) {
        const OutletRec rec = bd.out[r];
        if (rec.slotP >= 0) {
            int x, y, z;
            coords_of(g, rec.bP, x, y, z);
            const uint32_t tw = type[rec.bP];
            const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
            float rt = 0.f, J = 0.f;
            for (int k = 0; k < 2; k++) {
                float f[Q];
                gather<DIM, STORE>(dst + (int64_t)k * Q * g.Ppad, g, p, tw, x, y, z, f);
#pragma unroll
                for (int i = 0; i < Q; i++) {
                    rt += f[i];
                    J += (float)(Lat<DIM>::E[i][bd.out_axis] * bd.out_sign) * f[i];
                }
            }
            const float *F = bd.faceF + (int64_t)rec.slotP * 6;
            J += 0.5f * bd.out_sign * (F[bd.out_axis] + F[3 + bd.out_axis]);
            su = (double)(J / rt);
            cnt = 1.0;
        }
    }
    block_sum2(su, cnt, s_red);
    if (threadIdx.x == 0) {
        bd.ucpart[2 * (blockIdx.x - nb_in)] = su;
        bd.ucpart[2 * (blockIdx.x - nb_in) + 1] = cnt;
    }
}

// ---------------------------------------------------------------------------
// k_outlet_fill: eq. (20) for the populations entering through the outlet.
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_outlet_fill(const typename Codec<STORE>::T *__restrict__ src,
                                                     typename Codec<STORE>::T *__restrict__ dst,
                                                     const uint32_t *__restrict__ type, Geometry g, Boundary bd)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[8];
    double su, cnt;
    reduce_partials(bd.ucpart, bd.n_ucpart, su, cnt, s_red);
    double Uc = cnt > 0.0 ? su / cnt : 0.0;
    const bool clamped = Uc < 0.0;
    if (clamped) Uc = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bd.scal[SC_UC] = Uc;
        if (clamped) bd.scal[SC_CLAMPS] += 1.0;
    }
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= bd.n_out) return;
    const OutletRec rec = bd.out[r];
    int x, y, z;
    coords_of(g, rec.bN, x, y, z);
    int xp = 0, yp = 0, zp = 0;
    uint32_t twp = 0;
    int64_t pp = 0;
    if (rec.slotP >= 0) {
        coords_of(g, rec.bP, xp, yp, zp);
        twp = type[rec.bP];
        pp = pidx(g, xp, yp, DIM == 3 ? zp : -1);
    }
    const float uc = (float)Uc;
    for (int k = 0; k < 2; k++) {
        const T *sk = src + (int64_t)k * Q * g.Ppad;
        T *dk = dst + (int64_t)k * Q * g.Ppad;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            if (Lat<DIM>::E[i][bd.out_axis] * bd.out_sign >= 0) continue;
            const int64_t a = (int64_t)i * g.Ppad + src_slot<DIM>(g, x, y, z, i);
            const float prev = Codec<STORE>::ld(sk + a, weight<DIM>(i));
            float v = prev;
            if (rec.slotP >= 0) {
                const float fp = gather1<DIM, STORE>(dk, g, pp, twp, xp, yp, zp, i);
                v = (prev + uc * fp) / (1.0f + uc);
            }
            Codec<STORE>::st(dk + a, v, weight<DIM>(i));
        }
    }
}

// ---------------------------------------------------------------------------
// State exchange: canonical f[2][Q][N] (FP64) <-> population slots.
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ void k_scatter(typename Codec<STORE>::T *__restrict__ dst, const uint32_t *__restrict__ type,
                          Geometry g, const double *__restrict__ f)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.N) return;
    const uint32_t tw = type[b];
    if (tw & T_SOLID) return;
    int x, y, z;
    coords_of(g, b, x, y, z);
    const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
    for (int k = 0; k < 2; k++) {
        auto *dk = dst + (int64_t)k * Q * g.Ppad;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const bool bb = (tw >> i) & 1u;
            const int64_t a = bb ? (int64_t)Lat<DIM>::OPP[i] * g.Ppad + p
                                 : (int64_t)i * g.Ppad + src_slot<DIM>(g, x, y, z, i);
            Codec<STORE>::st(dk + a, (float)f[((int64_t)k * Q + i) * g.N + b], weight<DIM>(i));
        }
    }
}

template <int DIM, int STORE>
__global__ void k_gather_state(const typename Codec<STORE>::T *__restrict__ src, const uint32_t *__restrict__ type,
                               Geometry g, double *__restrict__ f)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.N) return;
    const uint32_t tw = type[b];
    for (int k = 0; k < 2; k++) {
        if (tw & T_SOLID) {
            for (int i = 0; i < Q; i++) f[((int64_t)k * Q + i) * g.N + b] = 0.0;
            continue;
        }
        int x, y, z;
        coords_of(g, b, x, y, z);
        const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
        float v[Q];
        gather<DIM, STORE>(src + (int64_t)k * Q * g.Ppad, g, p, tw | T_EDGE, x, y, z, v);
        for (int i = 0; i < Q; i++) f[((int64_t)k * Q + i) * g.N + b] = (double)v[i];
    }
}

// f = feq(rho0, u0) in canonical FP64 layout (initial state).
template <int DIM>
__global__ void k_feq_state(const double *__restrict__ rho0, const double *__restrict__ u0, int64_t N,
                            double *__restrict__ f)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    float u[3] = {0.f, 0.f, 0.f};
    if (u0)
        for (int d = 0; d < 3; d++) u[d] = (float)u0[d * N + b];
    for (int k = 0; k < 2; k++) {
        const float r = (float)rho0[k * N + b];
        for (int i = 0; i < Q; i++) f[((int64_t)k * Q + i) * N + b] = (double)feq<DIM>(i, r, u);
    }
}

// Per-block FP64 partial sums of rho_1 and rho_2 over fluid nodes.
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_mass(const typename Codec<STORE>::T *__restrict__ src,
                                              const uint32_t *__restrict__ type, Geometry g,
                                              double *__restrict__ part)
{
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[8];
    double m1 = 0.0, m2 = 0.0;
    for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < g.N; b += (int64_t)gridDim.x * 256) {
        const uint32_t tw = type[b];
        if (tw & T_SOLID) continue;
        int x, y, z;
        coords_of(g, b, x, y, z);
        const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
        float f[Q];
        gather<DIM, STORE>(src, g, p, tw, x, y, z, f);
        for (int i = 0; i < Q; i++) m1 += (double)f[i];
        gather<DIM, STORE>(src + (int64_t)Q * g.Ppad, g, p, tw, x, y, z, f);
        for (int i = 0; i < Q; i++) m2 += (double)f[i];
    }
    block_sum2(m1, m2, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = m1;
        part[2 * blockIdx.x + 1] = m2;
    }
}

__global__ void k_reduce2(const double *__restrict__ part, int n, double *__restrict__ out)
{
    __shared__ double s_red[8];
    double a, b;
    reduce_partials(part, n, a, b, s_red);
    if (threadIdx.x == 0) { out[0] = a; out[1] = b; }
}

}  // namespace lbm
