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
// One step is four (fused mode) or five (two-pass mode) launches:
//   k_psi            (two-pass mode) psi_k = rho_k of every node into an array
//   k_main           all fluid nodes, swept along the last axis: densities of
//                    each plane plus a two-node lateral halo into an LDS ring
//                    (from the psi array, or recomputed from the populations
//                    in the fused mode; mirror ghost layers at open faces,
//                    eqs. 24-25), force
//                    (eqs. 10-11), common velocity (eqs. 7-8), MRT collision
//                    (eq. 1); the mass flows rho u.n of the inlet nodes and
//                    of the x_{N-1} nodes summed exactly (eq. 23)
//   k_faces          chi = Q_in / Q' (eq. 23) and the collision of the outlet
//                    column with the corrected normal velocity (eq. 22); the
//                    inlet nodes too when none of them pulls from the outlet
//                    column
//   k_inlet          alpha-corrected NEQ extrapolation (eqs. 13-19) into the
//                    padding slots (the inlet nodes k_faces did not take);
//                    partial sums of eq. (21)
//   k_outlet_fill    convective outflow (eq. 20) into the padding slots
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.h"
#include "params.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage codecs.  A population is stored less an offset:
//   FP32:     f_i - w_i                         (the rest state at unit density)
//   binary16: f_i - w_i r, rounded to nearest even, where r is the previous
//             step's density of the component at the node that reads the
//             slot (the reference density, the same at write and at read).
// Near local equilibrium the stored numbers are then small for both the
// majority and the minority phase, so an 11-bit significand keeps the
// relative error of every population small; a fixed offset w_i would leave
// about 1% at a minority density of 0.03.  ld / st take the weight w and the
// reference density r of the reading node (FP32 ignores r).
//   binary16, fixed offset (storage 2): f_i - w_i, the offset as stated for
//             the precision extension, kept as a mode of its own so that its
//             error can be reported beside the reference-density codec.
// ---------------------------------------------------------------------------
template <int STORE> struct Codec;
template <> struct Codec<0> {
    using T = float;
    static constexpr bool REF = false;
    static __device__ __forceinline__ float ld(const T *p, float w, float) { return *p + w; }
    static __device__ __forceinline__ void st(T *p, float v, float w, float) { *p = v - w; }
};
template <> struct Codec<1> {
    using T = __half;
    static constexpr bool REF = true;
    static __device__ __forceinline__ float ld(const T *p, float w, float r) { return __half2float(*p) + w * r; }
    static __device__ __forceinline__ void st(T *p, float v, float w, float r) { *p = __float2half_rn(v - w * r); }
};
template <> struct Codec<2> {
    using T = __half;
    static constexpr bool REF = false;
    static __device__ __forceinline__ float ld(const T *p, float w, float) { return __half2float(*p) + w; }
    static __device__ __forceinline__ void st(T *p, float v, float w, float) { *p = __float2half_rn(v - w); }
};

// Raw buffer access for the node update: one descriptor per component array
// (range-checked by the hardware), a 32-bit per-lane byte offset and a
// wave-uniform byte offset per population plane.
constexpr int BUF_FLAGS = 0x00020000;   // dword 3 of a raw gfx9 buffer descriptor

template <int STORE> struct Buf;
// Cache policy of the buffer accesses (the instruction's aux field): bit 1 is
// the non-temporal hint.  FP32 node-update stores are non-temporal: nothing
// reads them again within the launch, and keeping them out of the way of the
// gathers' neighbour lines was measured faster (binary16 stores, and
// non-temporal loads, were measured slower).
constexpr int CPOL_NT = 2;

// ld = dec(raw(...)): raw issues the load, dec turns the stored bits into the
// population, so a caller can put independent work between the two.
template <> struct Buf<0> {
    static constexpr uint32_t SZ = 4;
    using Raw = uint32_t;
    static __device__ __forceinline__ Raw raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, so, 0);
    }
    static __device__ __forceinline__ float dec(Raw h, float w, float) { return __uint_as_float(h) + w; }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float w, float rr)
    {
        return dec(raw(r, vo, so), w, rr);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float v, float w,
                                              float)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v - w), r, (int)vo, so, CPOL_NT);
    }
};
template <> struct Buf<1> {
    static constexpr uint32_t SZ = 2;
    using Raw = unsigned short;
    static __device__ __forceinline__ Raw raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, so, 0);
    }
    static __device__ __forceinline__ float dec(Raw h, float w, float rr)
    {
        return __half2float(__ushort_as_half(h)) + w * rr;
    }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float w, float rr)
    {
        return dec(raw(r, vo, so), w, rr);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float v, float w,
                                              float rr)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v - w * rr)), r, (int)vo, so, 0);
    }
};

template <> struct Buf<2> {
    static constexpr uint32_t SZ = 2;
    using Raw = unsigned short;
    static __device__ __forceinline__ Raw raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, so, 0);
    }
    static __device__ __forceinline__ float dec(Raw h, float w, float) { return __half2float(__ushort_as_half(h)) + w; }
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float w, float rr)
    {
        return dec(raw(r, vo, so), w, rr);
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, int so, float v, float w, float)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v - w)), r, (int)vo, so, 0);
    }
};

template <int STORE>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t comp_rsrc(const void *base, int comp, int Q, int64_t Ppad)
{
    const char *p = (const char *)base + (int64_t)comp * Q * Ppad * Buf<STORE>::SZ;
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)((int64_t)Q * Ppad * Buf<STORE>::SZ),
                                             BUF_FLAGS);
}

__device__ __forceinline__ float pick3(const float (&v)[3], int a) { return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]); }

template <int DIM>
__device__ __forceinline__ int e_axis(int i, int a)
{
    return a == 0 ? Lat<DIM>::E[i][0] : (a == 1 ? Lat<DIM>::E[i][1] : Lat<DIM>::E[i][2]);
}

// Padded index of box node (x, y, z); x = 0 sits xoff elements into each row
// so that rows start on a 128-byte line (see Geometry).
__device__ __forceinline__ int64_t pidx(const Geometry &g, int x, int y, int z)
{
    return (int64_t)(x + g.xoff) + (int64_t)g.P[0] * ((int64_t)(y + 1) + (int64_t)g.P[1] * (int64_t)(z + 1));
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
    int s0 = x - Lat<DIM>::E[i][0], s1 = y - Lat<DIM>::E[i][1], s2 = z - Lat<DIM>::E[i][2];
    if (g.periodic[0]) s0 = s0 < 0 ? s0 + g.n[0] : (s0 >= g.n[0] ? s0 - g.n[0] : s0);
    if (g.periodic[1]) s1 = s1 < 0 ? s1 + g.n[1] : (s1 >= g.n[1] ? s1 - g.n[1] : s1);
    if (DIM == 3 && g.periodic[2]) s2 = s2 < 0 ? s2 + g.n[2] : (s2 >= g.n[2] ? s2 - g.n[2] : s2);
    if (DIM == 2) s2 = -1;
    return pidx(g, s0, s1, s2);
}

// Slot index (padded, within one component array) supplying population i.
template <int DIM>
__device__ __forceinline__ int64_t slot_of(const Geometry &g, int64_t p, uint32_t tw, int x, int y, int z, int i)
{
    if ((tw >> i) & 1u) return (int64_t)Lat<DIM>::OPP[i] * g.Ppad + p;
    return (int64_t)i * g.Ppad + ((tw & T_EDGE) ? src_slot<DIM>(g, x, y, z, i) : p - dir_off<DIM>(g, i));
}

// Post-streaming populations of one component at one node (pointer access).
// rr: the node's reference density of this component (see Codec).
template <int DIM, int STORE>
__device__ __forceinline__ void gather(const typename Codec<STORE>::T *__restrict__ fk, const Geometry &g,
                                       int64_t p, uint32_t tw, int x, int y, int z,
                                       float (&f)[Lat<DIM>::Q], float rr)
{
    static_for<Lat<DIM>::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        f[i] = Codec<STORE>::ld(fk + slot_of<DIM>(g, p, tw, x, y, z, i), weight<DIM>(i), rr);
    });
}

template <int DIM, int STORE>
__device__ __forceinline__ float gather1(const typename Codec<STORE>::T *__restrict__ fk, const Geometry &g,
                                         int64_t p, uint32_t tw, int x, int y, int z, int i, float rr)
{
    return Codec<STORE>::ld(fk + slot_of<DIM>(g, p, tw, x, y, z, i), weight<DIM>(i), rr);
}

// Byte offset of population plane i within one component array, formed at
// its point of use by one scalar multiply.  The copy through an empty asm
// statement makes the stride opaque, so the compiler cannot hoist the 19
// products out of the node loop: held there, they took 19 scalar registers,
// the kernel ran out of them, and every access then read its offset back
// from a vector-register lane (v_readlane) and waited five cycles before
// the memory instruction could use it.
template <int STORE>
__device__ __forceinline__ int plane_bytes(const Geometry &g, int i)
{
    int s = (int)((uint32_t)g.Ppad * Buf<STORE>::SZ);
    asm volatile("" : "+s"(s));
    return s * i;
}

// Where the populations that stream into node p (pull) are stored, as byte
// offsets within one component: a[i] per lane, plus the wave-uniform offset
// so_i that uniform_plane() gives.  The wave takes the cheapest of three
// address forms that is valid for all its nodes:
// * no bounce-back and no periodic wrap (wave_fast): population i sits at
//   plane_i + p - off_i, so a[i] is the shifted lane offset and the plane is
//   the wave-uniform offset;
// * walls but no wrap: per lane the streamed slot or the node's own slot of
//   the opposite direction (bounce-back), selected without branches, with
//   the plane in a[i];
// * otherwise the slot of every direction from its own rule.
// Only the addresses depend on the form; the loads are then issued in one
// straight run for both components, so no load is pending across a join of
// the three forms (such a join would make the loads wait for earlier ones).
template <int DIM, int STORE>
__device__ __forceinline__ void gather_addr(const Geometry &g, uint32_t p, uint32_t tw, int x, int y, int z,
                                            bool wave_fast, uint32_t (&a)[Lat<DIM>::Q])
{
    constexpr uint32_t SZ = Buf<STORE>::SZ;
    const uint32_t vb = (p - 1u) * SZ;
    const uint32_t sy = (uint32_t)g.P[0] * SZ, sz = (uint32_t)g.P[0] * (uint32_t)g.P[1] * SZ;
    auto shifted = [&](auto ic) -> uint32_t {
        constexpr int i = decltype(ic)::value;
        constexpr int ex = Lat<DIM>::E[i][0], ey = Lat<DIM>::E[i][1], ez = Lat<DIM>::E[i][2];
        uint32_t vo = vb + (uint32_t)(1 - ex) * SZ;
        if constexpr (ey == 1) vo -= sy;
        if constexpr (ey == -1) vo += sy;
        if constexpr (ez == 1) vo -= sz;
        if constexpr (ez == -1) vo += sz;
        return vo;
    };
    if (wave_fast) {
        static_for<Lat<DIM>::Q>([&](auto ic) { a[decltype(ic)::value] = shifted(ic); });
    } else if (__ballot(tw & T_EDGE) == 0) {
        static_for<Lat<DIM>::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const uint32_t own = p * SZ + (uint32_t)plane_bytes<STORE>(g, Lat<DIM>::OPP[i]);
            a[i] = ((tw >> i) & 1u) ? own : shifted(ic) + (uint32_t)plane_bytes<STORE>(g, i);
        });
    } else {
        static_for<Lat<DIM>::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            a[i] = (uint32_t)slot_of<DIM>(g, (int64_t)p, tw, x, y, z, i) * SZ;
        });
    }
}

// The wave-uniform part of the offset of direction i (the plane in the fast form).
template <int STORE>
__device__ __forceinline__ int uniform_plane(const Geometry &g, bool wave_fast, int i)
{
    // formed unconditionally and selected, so the node loop takes no branch here
    const int so = plane_bytes<STORE>(g, i);
    return wave_fast ? so : 0;
}

// The stored bits of the populations that stream into node p, one component.
template <int DIM, int STORE>
__device__ __forceinline__ void bgather_raw(__amdgpu_buffer_rsrc_t rs, const Geometry &g, uint32_t p, uint32_t tw,
                                            int x, int y, int z, bool wave_fast,
                                            typename Buf<STORE>::Raw (&f)[Lat<DIM>::Q])
{
    uint32_t a[Lat<DIM>::Q];
    gather_addr<DIM, STORE>(g, p, tw, x, y, z, wave_fast, a);
    static_for<Lat<DIM>::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        f[i] = Buf<STORE>::raw(rs, a[i], uniform_plane<STORE>(g, wave_fast, i));
    });
}

// The same for both components (same addresses, two buffers).
template <int DIM, int STORE>
__device__ __forceinline__ void bgather2_raw(__amdgpu_buffer_rsrc_t rs0, __amdgpu_buffer_rsrc_t rs1,
                                             const Geometry &g, uint32_t p, uint32_t tw, int x, int y, int z,
                                             bool wave_fast, typename Buf<STORE>::Raw (&f1)[Lat<DIM>::Q],
                                             typename Buf<STORE>::Raw (&f2)[Lat<DIM>::Q])
{
    uint32_t a[Lat<DIM>::Q];
    gather_addr<DIM, STORE>(g, p, tw, x, y, z, wave_fast, a);
    static_for<Lat<DIM>::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        f1[i] = Buf<STORE>::raw(rs0, a[i], uniform_plane<STORE>(g, wave_fast, i));
    });
    static_for<Lat<DIM>::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        f2[i] = Buf<STORE>::raw(rs1, a[i], uniform_plane<STORE>(g, wave_fast, i));
    });
}

// Populations from the stored bits that bgather_raw loaded.
template <int DIM, int STORE>
__device__ __forceinline__ void decode(const typename Buf<STORE>::Raw (&h)[Lat<DIM>::Q], float (&f)[Lat<DIM>::Q],
                                       float rr)
{
    static_for<Lat<DIM>::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        f[i] = Buf<STORE>::dec(h[i], weight<DIM>(i), rr);
    });
}

template <int DIM, int STORE>
__device__ __forceinline__ void bgather(__amdgpu_buffer_rsrc_t rs, const Geometry &g, uint32_t p, uint32_t tw,
                                        int x, int y, int z, bool wave_fast, float (&f)[Lat<DIM>::Q], float rr)
{
    typename Buf<STORE>::Raw h[Lat<DIM>::Q];
    bgather_raw<DIM, STORE>(rs, g, p, tw, x, y, z, wave_fast, h);
    decode<DIM, STORE>(h, f, rr);
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

// Linear index in the caller's frame of the memory-frame node (x, y, z).
__device__ __forceinline__ int64_t caller_index(const Geometry &g, int x, int y, int z)
{
    return (int64_t)x * g.ostride[0] + (int64_t)y * g.ostride[1] + (int64_t)z * g.ostride[2];
}

// Deterministic block-wide sum of two doubles over NT threads (whole waves):
// a butterfly inside each wave, then the wave sums in a fixed pairwise order.
template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red /*[2 * NT / 64]*/)
{
    static_assert(NT % 64 == 0 && NT <= 1024, "whole waves");
    constexpr int NW = NT / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if constexpr (NW > 1) {
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
        __syncthreads();
        if (ln == 0) { red[2 * wv] = a; red[2 * wv + 1] = b; }
        __syncthreads();
        // every thread folds the wave sums in the same fixed pairwise order
        double ta[NW], tb[NW];
#pragma unroll
        for (int j = 0; j < NW; j++) { ta[j] = red[2 * j]; tb[j] = red[2 * j + 1]; }
#pragma unroll
        for (int w = NW / 2; w > 0; w >>= 1) {
#pragma unroll
            for (int j = 0; j < w; j++) { ta[j] += ta[j + w]; tb[j] += tb[j + w]; }
        }
        a = ta[0];
        b = tb[0];
    }
}

// Deterministic sum of a partials array [n][2] by every block (fixed order).
template <int NT>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int n, double &a, double &b,
                                                double *red)
{
    a = 0.0;
    b = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    block_sum2<NT>(a, b, red);
}

// ---------------------------------------------------------------------------
// The sums Q_in and Q' of eq. (23) as integers in units of 2^-40.  Each term
// rho u.n (the FP64 product of two floats) is rounded once to that grid; the
// integer sums are then exact, so they do not depend on which block adds
// which term or in what order (every launch shape and tile configuration
// gives the same bits).  The grid is far below FP32 resolution; the range
// holds |Q| < 2^23.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long flow_fix(double q) { return __double2ll_rn(q * 0x1p40); }
__device__ __forceinline__ double flow_unfix(unsigned long long v) { return (double)(long long)v * 0x1p-40; }

// ---------------------------------------------------------------------------
// k_main: the fused per-node update as a sweep along the last lattice axis
// (y in 2-D, z in 3-D).  A block owns a lateral tile (TX in 2-D, TX x TY in
// 3-D) and a chunk of ZC planes of the sweep axis; it advances W planes per
// iteration and keeps psi of the planes it needs (window plus two on each
// side) in an LDS ring of W + 4 planes, so psi is computed once per plane and
// only the lateral two-node halo is recomputed by neighbouring blocks.
// Work items are ordered lateral-x fastest, then lateral-y, then chunk, and
// each of the eight XCDs takes a contiguous range of them, so the blocks that
// share halo data share an L2.
// ---------------------------------------------------------------------------
//
// PSRC selects where psi comes from: 0 = recomputed here from the gathered
// populations of each plane (one fused kernel), 1 = read from the psi array
// that k_psi wrote for this step (the populations are then read only once).
//
// KEEPB = 1 holds both components' populations in registers between the
// velocity and the collision; KEEPB = 0 gathers component 2 again after
// component 1 is stored (fewer registers, one more pass through the caches).
template <int DIM, int STORE, int PSRC, int TX, int TY, int W, int ZC, int KEEPB>
__device__ __forceinline__ void main_item(const typename Codec<STORE>::T *__restrict__ src,
                                          typename Codec<STORE>::T *__restrict__ dst,
                                          const uint32_t *__restrict__ type, const float2 *__restrict__ psi,
                                          const float2 *__restrict__ ref, const Geometry &g, const Physics &ph,
                                          const Boundary &bd, int tiles_x, int tiles_y, int item,
                                          int *__restrict__ flag, unsigned long long *__restrict__ qacc)
{
    constexpr int Q = Lat<DIM>::Q;
    constexpr int LY = DIM == 3 ? TY : 1;          // lateral y extent of the tile
    constexpr int HX = TX + 4, HY = DIM == 3 ? TY + 4 : 1;
    constexpr int PLANE = HX * HY;                 // lateral halo positions per plane
    constexpr int R = W + 4;                       // ring planes
    constexpr int RP = DIM == 3 ? 1 : 256 / TX;    // 2-D: rows covered by one pass of the block
    constexpr int NPT = DIM == 3 ? W : W / RP;     // nodes per thread per iteration
    constexpr int NOFF = DIM == 3 ? 125 : 25;      // offsets of the 5^DIM stencil box
    static_assert(DIM == 3 ? TX * LY == 256 : (256 % TX == 0 && W % RP == 0), "256 threads per block");
    __shared__ float2 s_psi[R * PLANE];
    __shared__ uint8_t s_sol[R * PLANE];
    // 2-D fused mode, binary16: the stored bits of the populations that
    // stream into each ring node, gathered once for its psi and read back by
    // the node update (the same loads, so the same bits).  FP32 would need
    // 39 KB of LDS per block and lose more occupancy than it saves.
    constexpr bool STAGE = DIM == 2 && PSRC == 0 && STORE != 0;
    __shared__ typename Buf<STORE>::Raw s_fr[STAGE ? R * PLANE * 2 * Q : 1];

    const __amdgpu_buffer_rsrc_t rs0 = comp_rsrc<STORE>(src, 0, Q, g.Ppad);
    const __amdgpu_buffer_rsrc_t rs1 = comp_rsrc<STORE>(src, 1, Q, g.Ppad);
    // the item's share of the eq. (23) sums (fixed point, see flow_fix),
    // gathered by LDS atomics at the face nodes, so that nothing is held in
    // registers across the sweep
    __shared__ unsigned long long s_q[2];
    if (threadIdx.x == 0) s_q[0] = s_q[1] = 0ull;
    __syncthreads();                               // the ring of a previous item is free
    {
        const int ns = g.n[DIM - 1];
        const int tx = item % tiles_x;
        const int ty = (item / tiles_x) % tiles_y;
        const int ch = item / (tiles_x * tiles_y);
        const int x0 = tx * TX, y0 = DIM == 3 ? ty * TY : 0;
        const int s0 = ch * ZC, s1 = min(s0 + ZC, ns);

        // psi of sweep planes [pa, pb) into the ring
        auto load_planes = [&](int pa, int pb) {
            const int cnt = (pb - pa) * PLANE;
            for (int h = threadIdx.x; h < cnt; h += 256) {
                const int pl = pa + h / PLANE, r = h % PLANE;
                const int lx = r % HX, ly = r / HX;
                int gx = x0 - 2 + lx, gy, gz;
                if (DIM == 3) { gy = y0 - 2 + ly; gz = pl; }
                else { gy = pl; gz = 0; }
                const bool need = gx < g.n[0] + 2 && gy < g.n[1] + 2 && (DIM == 2 || gz < g.n[2] + 2);
                const int slot = ((pl + 4 * R) % R) * PLANE + r;
                if constexpr (PSRC == 1) {
                    // psi of this step from k_psi; solids carry -0.0 (zero in
                    // every sum, and the sign marks them for the adhesion stencil)
                    float2 v = make_float2(0.0f, 0.0f);
                    uint8_t sol = 1;
                    if (need) {
                        gx = map_axis(gx, g.n[0], g.periodic[0]);
                        gy = map_axis(gy, g.n[1], g.periodic[1]);
                        if (DIM == 3) gz = map_axis(gz, g.n[2], g.periodic[2]);
                        v = psi[(int64_t)gx + (int64_t)g.n[0] * ((int64_t)gy + (int64_t)g.n[1] * gz)];
                        sol = signbit(v.x) ? 1 : 0;
                    }
                    s_psi[slot] = v;
                    s_sol[slot] = sol;
                    continue;
                }
                uint32_t tw = T_SOLID;
                uint32_t pp = 0;
                if (need) {
                    gx = map_axis(gx, g.n[0], g.periodic[0]);
                    gy = map_axis(gy, g.n[1], g.periodic[1]);
                    if (DIM == 3) gz = map_axis(gz, g.n[2], g.periodic[2]);
                    const int64_t b = (int64_t)gx + (int64_t)g.n[0] * ((int64_t)gy + (int64_t)g.n[1] * gz);
                    tw = type[b];
                    pp = (uint32_t)pidx(g, gx, gy, DIM == 3 ? gz : -1);
                }
                const bool fluid = !(tw & T_SOLID);
                const bool wave_fast = __ballot(fluid && (tw & (T_BBMASK | T_EDGE))) == 0;
                float p1 = 0.0f, p2 = 0.0f;
                if (fluid) {
                    float f[Q];
                    float2 rf = make_float2(0.0f, 0.0f);
                    if constexpr (Codec<STORE>::REF) rf = ref[(int64_t)gx + (int64_t)g.n[0] * ((int64_t)gy + (int64_t)g.n[1] * gz)];
                    typename Buf<STORE>::Raw h1[Q], h2[Q];
                    bgather2_raw<DIM, STORE>(rs0, rs1, g, pp, tw, gx, gy, gz, wave_fast, h1, h2);
                    if constexpr (STAGE) {
                        static_for<Q>([&](auto ic) {
                            constexpr int i = decltype(ic)::value;
                            s_fr[slot * 2 * Q + i] = h1[i];
                            s_fr[slot * 2 * Q + Q + i] = h2[i];
                        });
                    }
                    decode<DIM, STORE>(h1, f, rf.x);
                    static_for<Q>([&](auto ic) { p1 += f[decltype(ic)::value]; });
                    decode<DIM, STORE>(h2, f, rf.y);
                    static_for<Q>([&](auto ic) { p2 += f[decltype(ic)::value]; });
                }
                s_psi[slot] = make_float2(p1, p2);
                s_sol[slot] = fluid ? 0 : 1;
            }
        };

        // node k of this thread in the sweep window starting at plane w0
        const int lx = threadIdx.x % TX, ly = DIM == 3 ? threadIdx.x / TX : 0;
        auto sweep_of = [&](int w0, int k) { return DIM == 3 ? w0 + k : w0 + k * RP + (int)threadIdx.x / TX; };
        auto type_of = [&](int sv) -> uint32_t {
            const int x = x0 + lx, y = DIM == 3 ? y0 + ly : sv, z = DIM == 3 ? sv : 0;
            const bool valid = x < g.n[0] && sv < s1 && (DIM == 2 || y < g.n[1]);
            return valid ? type[(int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)g.n[1] * z)] : T_SOLID;
        };
        load_planes(s0 - 2, s0 + 2);
        for (int w0 = s0; w0 < s1; w0 += W) {
            __syncthreads();                      // ring slots of w0-6..w0-3 are free
            // the type words of the window's nodes are loaded together with
            // the psi planes, whose wait covers them: loaded node by node they
            // would each wait for the previous node's stores to complete (the
            // memory counter also counts stores)
            uint32_t twq[NPT];
            static_for<NPT>([&](auto jc) { twq[decltype(jc)::value] = type_of(sweep_of(w0, decltype(jc)::value)); });
            load_planes(w0 + 2, w0 + W + 2);
            __syncthreads();
            // settle the type loads here, once per window: an empty statement
            // that reads them, so that the wait is not placed at the head of
            // the node loop, where it would run on every node
#pragma unroll
            for (int j = 0; j < NPT; j++) asm volatile("" ::"v"(twq[j]));
#pragma unroll 1
            for (int k = 0; k < NPT; k++) {
                const int sv = sweep_of(w0, k);
                const int x = x0 + lx;
                const int y = DIM == 3 ? y0 + ly : sv;
                const int z = DIM == 3 ? sv : 0;
                const bool valid = x < g.n[0] && sv < s1 && (DIM == 2 || y < g.n[1]);
                const int64_t b = valid ? (int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)g.n[1] * z) : 0;
                const uint32_t tw = twq[0];
                static_for<NPT - 1>([&](auto jc) { twq[decltype(jc)::value] = twq[decltype(jc)::value + 1]; });
                const bool fluid = !(tw & T_SOLID);
                const bool wave_fast = __ballot(fluid && (tw & (T_BBMASK | T_EDGE))) == 0;
                if (!fluid) continue;
                const uint32_t p = (uint32_t)pidx(g, x, y, DIM == 3 ? z : -1);
                // base[d]: ring index of the lateral corner (-2, -2) of the
                // node's neighbourhood in sweep plane sv + d - 2, so every
                // stencil offset below is a non-negative immediate
                const int corner = (DIM == 3 ? ly * HX : 0) + lx;
                int base[5];
                static_for<5>([&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    base[d] = ((sv + d - 2 + 4 * R) % R) * PLANE + corner;
                });
                constexpr int CEN = (DIM == 3 ? 2 * HX : 0) + 2;   // the node itself
                // the populations of the node: loads issued here, before the
                // force stencil, so the LDS work below hides their latency
                typename Buf<STORE>::Raw h1[Q], h2[Q];
                if constexpr (STAGE) {
                    // staged in the ring when psi of this node's plane was formed
                    const int sl = base[2] + CEN;
                    static_for<Q>([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        h1[i] = s_fr[sl * 2 * Q + i];
                        h2[i] = s_fr[sl * 2 * Q + Q + i];
                    });
                } else if constexpr (KEEPB) {
                    bgather2_raw<DIM, STORE>(rs0, rs1, g, p, tw, x, y, z, wave_fast, h1, h2);
                } else {
                    bgather_raw<DIM, STORE>(rs0, g, p, tw, x, y, z, wave_fast, h1);
                }
                const float2 ps = s_psi[base[2] + CEN];
                // psi(t) of the node for the next step's reference densities
                // and the face kernels (the two-pass mode has it from k_psi)
                if constexpr (PSRC == 0) const_cast<float2 *>(psi)[b] = ps;
                float2 rf = make_float2(0.0f, 0.0f);
                if constexpr (Codec<STORE>::REF) rf = ref[b];

                // ---- wall adhesion (eq. 11): only nodes with a solid within the stencil
                float A[3] = {0.f, 0.f, 0.f};
                if (ph.adhesion && (tw & T_NEARWALL)) {
                    static_for<NOFF>([&](auto oc) {
                        constexpr int o = decltype(oc)::value;
                        constexpr int dx = o % 5 - 2, dy = (o / 5) % 5 - 2, dz = DIM == 3 ? o / 25 - 2 : 0;
                        constexpr int r2 = dx * dx + dy * dy + dz * dz;
                        constexpr float w = stencil_w<DIM>(r2);
                        if constexpr (r2 != 0 && w != 0.0f) {
                            constexpr int ddy = DIM == 3 ? dy : 0, ddz = DIM == 3 ? dz : dy;
                            const float sv1 = (float)s_sol[base[2 + ddz] + CEN + ddy * HX + dx];
                            if constexpr (dx != 0) A[0] = fmaf(w * dx, sv1, A[0]);
                            if constexpr (dy != 0) A[1] = fmaf(w * dy, sv1, A[1]);
                            if constexpr (dz != 0) A[2] = fmaf(w * dz, sv1, A[2]);
                        }
                    });
                }
                // ---- forces (eqs. 10-11): the stencil in pairs of opposite
                // offsets, one sweep-plane distance at a time (the loop bounds
                // how many LDS reads are in flight)
                float g1[3] = {0.f, 0.f, 0.f}, g2[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
                for (int sd = 0; sd <= 2; sd++) {
                    const int bp = ((sv + sd + 4 * R) % R) * PLANE + corner + CEN;
                    const int bm = ((sv - sd + 4 * R) % R) * PLANE + corner + CEN;
                    auto plane = [&](auto sdc) {
                        constexpr int SD = decltype(sdc)::value;
                        static_for<25>([&](auto oc) {
                            constexpr int o = decltype(oc)::value;
                            constexpr int a = o % 5 - 2, bq = o / 5 - 2;   // lateral offsets
                            // (dx, dy, dz) of the offset and its lateral / sweep split
                            constexpr int dx = a, dy = DIM == 3 ? bq : SD, dz = DIM == 3 ? SD : 0;
                            constexpr int lat_y = DIM == 3 ? bq : 0;
                            constexpr int r2 = dx * dx + dy * dy + dz * dz;
                            constexpr float w = stencil_w<DIM>(r2);
                            // the half of the stencil with a positive first nonzero of (sweep, lateral-y, x)
                            constexpr bool half = SD > 0 || (lat_y > 0 || (lat_y == 0 && dx > 0));
                            constexpr bool in2d = DIM == 3 || bq == 0;
                            if constexpr (half && in2d && w != 0.0f) {
                                constexpr int ho = lat_y * HX + dx;
                                const float2 vp = s_psi[bp + ho];
                                const float2 vm = s_psi[bm - ho];
                                const float d1 = vp.x - vm.x, d2 = vp.y - vm.y;
                                if constexpr (dx != 0) { g1[0] = fmaf(w * dx, d1, g1[0]); g2[0] = fmaf(w * dx, d2, g2[0]); }
                                if constexpr (dy != 0) { g1[1] = fmaf(w * dy, d1, g1[1]); g2[1] = fmaf(w * dy, d2, g2[1]); }
                                if constexpr (dz != 0) { g1[2] = fmaf(w * dz, d1, g1[2]); g2[2] = fmaf(w * dz, d2, g2[2]); }
                            }
                        });
                    };
                    if (sd == 0) plane(std::integral_constant<int, 0>{});
                    else if (sd == 1) plane(std::integral_constant<int, 1>{});
                    else plane(std::integral_constant<int, 2>{});
                }
                const float r1 = ps.x, r2 = ps.y, rt = r1 + r2;
                const float w1 = r1 / rt, w2 = r2 / rt;
                float F1[3], F2[3];
                static_for<3>([&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    F1[d] = -ph.G12 * r1 * g2[d] - ph.Gw[0] * r1 * A[d] + w1 * ph.Fb[d];
                    F2[d] = -ph.G12 * r2 * g1[d] - ph.Gw[1] * r2 * A[d] + w2 * ph.Fb[d];
                });

                // ---- common velocity (eqs. 7-8)
                PairF<DIM> qa, qb;
                float J1[3], J2[3];
                {
                    float f[Q];
                    decode<DIM, STORE>(h1, f, rf.x);
                    to_pairs<DIM>(f, qa);
                    pair_momentum<DIM>(qa, J1);
                    if constexpr (!KEEPB && !STAGE) bgather_raw<DIM, STORE>(rs1, g, p, tw, x, y, z, wave_fast, h2);
                    decode<DIM, STORE>(h2, f, rf.y);
                    to_pairs<DIM>(f, qb);
                    pair_momentum<DIM>(qb, J2);
                }
                float u[3];
                const float irt = 1.0f / rt;
                static_for<3>([&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    u[d] = (J1[d] + J2[d] + 0.5f * (F1[d] + F2[d])) * irt;
                });

                if (!(rt > 0.0f) || !isfinite(rt) || !isfinite(u[0] + u[1] + u[2])) *flag = 1;

                if (tw & T_ROLE) {
                    const int slot = bd.bslot[b];
                    float *fF = bd.faceF + (int64_t)slot * 6;
                    fF[0] = F1[0]; fF[1] = F1[1]; fF[2] = F1[2];
                    fF[3] = F2[0]; fF[4] = F2[1]; fF[5] = F2[2];
                    if (tw & T_XPRIME) {
                        const float un = bd.out_sign * pick3(u, bd.out_axis);
                        bd.faceU[slot] = un;
                        atomicAdd(&s_q[1], (unsigned long long)flow_fix((double)rt * (double)un));
                    }
                    if (tw & T_INLET) {
                        const Patch pt = bd.patch[(tw & T_PATCH_MASK) >> T_PATCH_SHIFT];
                        atomicAdd(&s_q[0], (unsigned long long)flow_fix((double)rt * (double)(pt.sign * pick3(u, pt.axis))));
                    }
                    if ((tw & T_OUTLET) && bd.chi_on) continue;   // collided by the face launch (k_faces)
                }

                // ---- MRT collision of each component, stored at x
                const __amdgpu_buffer_rsrc_t rd0 = comp_rsrc<STORE>(dst, 0, Q, g.Ppad);
                const __amdgpu_buffer_rsrc_t rd1 = comp_rsrc<STORE>(dst, 1, Q, g.Ppad);
                const uint32_t vo = p * Buf<STORE>::SZ;
                // reference density of the node that reads population i next
                // step: the destination x + e_i, or x itself on bounce-back
                auto dest_psi = [&](auto ic) -> float2 {
                    constexpr int i = decltype(ic)::value;
                    constexpr int ex = Lat<DIM>::E[i][0], ey = Lat<DIM>::E[i][1], ez = Lat<DIM>::E[i][2];
                    if ((tw >> Lat<DIM>::OPP[i]) & 1u) return ps;
                    if constexpr (DIM == 3) return s_psi[base[2 + ez] + CEN + ey * HX + ex];
                    else return s_psi[base[2 + ey] + CEN + ex];
                };
                float fo[Q];
                // a moving wall: the populations that bounce back from it take
                // its momentum, -2 w_j rho_k (e_j . u_w) / cs^2, stored with
                // them (only this node reads them)
                const float *cw = (tw & T_MOVWALL) ? bd.wallc + (int64_t)bd.bslot[b] * Q : nullptr;
                const Rates ra = {ph.se[0], ph.seps[0], ph.sq, ph.snu[0]};
                collide_pairs<DIM, STORE == 0>(qa, r1, J1, u, F1, ra, fo);
                if (cw) static_for<Q>([&](auto ic) { fo[decltype(ic)::value] = fmaf(cw[decltype(ic)::value], r1, fo[decltype(ic)::value]); });
                static_for<Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    float rd = 0.0f;
                    if constexpr (Codec<STORE>::REF) rd = dest_psi(ic).x;
                    Buf<STORE>::st(rd0, vo, plane_bytes<STORE>(g, i), fo[i], weight<DIM>(i), rd);
                });
                if constexpr (!KEEPB) {
                    float f[Q];
                    bgather<DIM, STORE>(rs1, g, p, tw, x, y, z, wave_fast, f, rf.y);
                    to_pairs<DIM>(f, qb);
                }
                const Rates rb = {ph.se[1], ph.seps[1], ph.sq, ph.snu[1]};
                collide_pairs<DIM, STORE == 0>(qb, r2, J2, u, F2, rb, fo);
                if (cw) static_for<Q>([&](auto ic) { fo[decltype(ic)::value] = fmaf(cw[decltype(ic)::value], r2, fo[decltype(ic)::value]); });
                static_for<Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    float rd = 0.0f;
                    if constexpr (Codec<STORE>::REF) rd = dest_psi(ic).y;
                    Buf<STORE>::st(rd1, vo, plane_bytes<STORE>(g, i), fo[i], weight<DIM>(i), rd);
                });
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_q[0]) atomicAdd(qacc, s_q[0]);
        if (s_q[1]) atomicAdd(qacc + 1, s_q[1]);
    }
}

// One context: one block per work item (tiles that hold fluid, in tile
// order).
// Binary16 storage asks for four waves per SIMD (128 VGPRs): its 64x4 tile
// then runs at occupancy 4 instead of 3 without spilling, 2.4% faster; FP32
// gains nothing from the request and takes what it needs.
template <int DIM, int STORE, int PSRC, int TX, int TY, int W, int ZC, int KEEPB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STORE != 0 ? 4 : 1)))
void k_main(const typename Codec<STORE>::T *__restrict__ src,
                                              typename Codec<STORE>::T *__restrict__ dst,
                                              const uint32_t *__restrict__ type,
                                              const float2 *__restrict__ psi, const float2 *__restrict__ ref,
                                              Geometry g, Physics ph, Boundary bd, int tiles_x, int tiles_y,
                                              int n_items, const int *__restrict__ item_list,
                                              int *__restrict__ flag, unsigned long long *__restrict__ qacc)
{
    // blocks go round-robin to the 8 XCDs (blockIdx % 8); each XCD takes
    // groups of MAIN_XCD_GROUP consecutive work items, so that all XCDs sweep
    // nearby addresses at the same time while x-neighbour tiles still share
    // an L2 (measured faster than both one item per XCD turn and contiguous
    // ranges per XCD); the grid is a multiple of 8 * MAIN_XCD_GROUP blocks
    const int S = (int)blockIdx.x / 8, r = (int)blockIdx.x % 8;
    const int k = ((S / MAIN_XCD_GROUP) * 8 + r) * MAIN_XCD_GROUP + S % MAIN_XCD_GROUP;
    if (k < n_items)
        main_item<DIM, STORE, PSRC, TX, TY, W, ZC, KEEPB>(src, dst, type, psi, ref, g, ph, bd, tiles_x, tiles_y,
                                                          item_list[k], flag, qacc);
}

// ---------------------------------------------------------------------------
// k_psi: psi_k = rho_k = sum_i f_i^k of every node (eq. 8 with psi_k = rho_k)
// from the post-streaming populations, as float2 per box node; solid nodes
// get (-0.0, -0.0).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__device__ __forceinline__ void psi_body(int blk, const typename Codec<STORE>::T *__restrict__ src,
                                             const uint32_t *__restrict__ type, Geometry g,
                                             float2 *__restrict__ psi, const float2 *__restrict__ ref)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blk * 256 + threadIdx.x;
    const bool valid = b < g.N;
    const uint32_t tw = valid ? type[b] : T_SOLID;
    const bool fluid = !(tw & T_SOLID);
    const bool wave_fast = __ballot(fluid && (tw & (T_BBMASK | T_EDGE))) == 0;
    if (!valid) return;
    if (!fluid) {
        psi[b] = make_float2(-0.0f, -0.0f);
        return;
    }
    int x, y, z;
    coords_of(g, b, x, y, z);
    const uint32_t p = (uint32_t)pidx(g, x, y, DIM == 3 ? z : -1);
    float f[Q], r1 = 0.0f, r2 = 0.0f;
    float2 rf = make_float2(0.0f, 0.0f);
    if constexpr (Codec<STORE>::REF) rf = ref[b];
    typename Buf<STORE>::Raw h1[Q], h2[Q];
    bgather2_raw<DIM, STORE>(comp_rsrc<STORE>(src, 0, Q, g.Ppad), comp_rsrc<STORE>(src, 1, Q, g.Ppad), g, p, tw, x,
                             y, z, wave_fast, h1, h2);
    decode<DIM, STORE>(h1, f, rf.x);
    static_for<Q>([&](auto ic) { r1 += f[decltype(ic)::value]; });
    decode<DIM, STORE>(h2, f, rf.y);
    static_for<Q>([&](auto ic) { r2 += f[decltype(ic)::value]; });
    psi[b] = make_float2(r1, r2);
}

template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_psi(const typename Codec<STORE>::T *__restrict__ src,
                                             const uint32_t *__restrict__ type, Geometry g,
                                             float2 *__restrict__ psi, const float2 *__restrict__ ref)
{
    psi_body<DIM, STORE>((int)blockIdx.x, src, type, g, psi, ref);
}

// Density and momentum of the populations of one component.  The momentum is
// summed over opposite pairs, f_i - f_opp(i) first: the two are close, so
// their difference is exact and the small differences add with little
// rounding (the velocity is a small difference of large populations).
template <int DIM>
__device__ __forceinline__ void moments_of(const float (&f)[Lat<DIM>::Q], float &rho, float (&J)[3])
{
    rho = 0.0f;
    static_for<Lat<DIM>::Q>([&](auto ic) { rho += f[decltype(ic)::value]; });
    static_for<3>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        float acc = 0.0f;
        static_for<Pairs<DIM>::P>([&](auto pc) {
            constexpr int i = Pairs<DIM>::first(decltype(pc)::value);
            constexpr int e = Lat<DIM>::E[i][d];
            if constexpr (e == 1) acc += f[i] - f[Lat<DIM>::OPP[i]];
            else if constexpr (e == -1) acc -= f[i] - f[Lat<DIM>::OPP[i]];
        });
        J[d] = acc;
    });
}

// ---------------------------------------------------------------------------
// k_moments: rho_k and the common velocity of eqs. (7)-(8) (with this
// state's force, before any outlet override) of every node, one thread per
// node, with psi of the neighbours read from the array k_psi wrote.
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_moments(const typename Codec<STORE>::T *__restrict__ src,
                                                 const uint32_t *__restrict__ type,
                                                 const float2 *__restrict__ psi, const float2 *__restrict__ ref,
                                                 Geometry g, Physics ph, double *__restrict__ out_rho,
                                                 double *__restrict__ out_u)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= g.N) return;
    const uint32_t tw = type[b];
    int x, y, z;
    coords_of(g, b, x, y, z);
    const int64_t bo = caller_index(g, x, y, z);
    if (tw & T_SOLID) {
        out_rho[bo] = 0.0;
        out_rho[g.N + bo] = 0.0;
        out_u[bo] = out_u[g.N + bo] = out_u[2 * g.N + bo] = 0.0;
        return;
    }
    auto psi_at = [&](int dx, int dy, int dz) {
        const int qx = map_axis(x + dx, g.n[0], g.periodic[0]);
        const int qy = map_axis(y + dy, g.n[1], g.periodic[1]);
        const int qz = DIM == 3 ? map_axis(z + dz, g.n[2], g.periodic[2]) : 0;
        return psi[(int64_t)qx + (int64_t)g.n[0] * ((int64_t)qy + (int64_t)g.n[1] * qz)];
    };
    // the stencil in pairs of opposite offsets, in the node update's order
    // (sweep distance, then lateral offsets), so u matches the step's
    float g1[3] = {0.f, 0.f, 0.f}, g2[3] = {0.f, 0.f, 0.f}, A[3] = {0.f, 0.f, 0.f};
    static_for<3>([&](auto sdc) {
        constexpr int SD = decltype(sdc)::value;
        static_for<25>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            constexpr int a = o % 5 - 2, bq = o / 5 - 2;
            constexpr int dx = a, dy = DIM == 3 ? bq : SD, dz = DIM == 3 ? SD : 0;
            constexpr int lat_y = DIM == 3 ? bq : 0;
            constexpr int r2 = dx * dx + dy * dy + dz * dz;
            constexpr float w = stencil_w<DIM>(r2);
            constexpr bool half = SD > 0 || (lat_y > 0 || (lat_y == 0 && dx > 0));
            constexpr bool in2d = DIM == 3 || bq == 0;
            if constexpr (half && in2d && w != 0.0f) {
                const float2 vp = psi_at(dx, dy, dz), vm = psi_at(-dx, -dy, -dz);
                const float d1 = vp.x - vm.x, d2 = vp.y - vm.y;
                const float ds = (signbit(vp.x) ? 1.0f : 0.0f) - (signbit(vm.x) ? 1.0f : 0.0f);
                const int e3[3] = {dx, dy, dz};
                static_for<3>([&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    if (e3[d] != 0) {
                        g1[d] = fmaf(w * e3[d], d1, g1[d]);
                        g2[d] = fmaf(w * e3[d], d2, g2[d]);
                        A[d] = fmaf(w * e3[d], ds, A[d]);
                    }
                });
            }
        });
    });
    if (!ph.adhesion) A[0] = A[1] = A[2] = 0.0f;
    const float2 ps = psi[b];
    const float r1 = ps.x, r2 = ps.y, rt = r1 + r2;
    const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
    float f[Q], ra, rb, Ja[3], Jb[3];
    const float2 rf = ref[b];
    gather<DIM, STORE>(src, g, p, tw | T_EDGE, x, y, z, f, rf.x);
    moments_of<DIM>(f, ra, Ja);
    gather<DIM, STORE>(src + (int64_t)Q * g.Ppad, g, p, tw | T_EDGE, x, y, z, f, rf.y);
    moments_of<DIM>(f, rb, Jb);
    out_rho[bo] = r1;
    out_rho[g.N + bo] = r2;
    static_for<3>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        const float F1 = -ph.G12 * r1 * g2[d] - ph.Gw[0] * r1 * A[d] + (r1 / rt) * ph.Fb[d];
        const float F2 = -ph.G12 * r2 * g1[d] - ph.Gw[1] * r2 * A[d] + (r2 / rt) * ph.Fb[d];
        if (d < DIM) out_u[g.ax[d] * g.N + bo] = (Ja[d] + Jb[d] + 0.5f * (F1 + F2)) / rt;
    });
}

// chi of eq. (23); undefined (no outflow through x_{N-1}, or flow against the
// inlets) leaves the outlet uncorrected.
__device__ __forceinline__ double chi_of(double qin, double qout)
{
    return (fabs(qout) < 1e-30 || qin * qout <= 0.0) ? 1.0 : qin / qout;
}

// ---------------------------------------------------------------------------
// eq. (23) from the sums the node update left in acc (this step's parity):
// every thread of the first face launch forms chi itself; one thread records
// Q_in, Q' and chi and clears the sums of the other parity for the next step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double chi_from(const Boundary &bd, const unsigned long long *acc,
                                           unsigned long long *next, bool record)
{
    const double qin = flow_unfix(acc[0]), qout = flow_unfix(acc[1]);
    const double chi = (bd.has_outlet && bd.chi_on) ? chi_of(qin, qout) : 1.0;
    if (record) {
        bd.scal[SC_QIN] = qin;
        bd.scal[SC_QOUT] = qout;
        bd.scal[SC_CHI] = chi;
        next[0] = 0ull;
        next[1] = 0ull;
    }
    return chi;
}

// ---------------------------------------------------------------------------
// The collision of the outlet column with eq. (22) for a given chi (eq. 23).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__device__ __forceinline__ void outlet_body(int blk, const typename Codec<STORE>::T *__restrict__ src,
                                                    typename Codec<STORE>::T *__restrict__ dst,
                                                    const uint32_t *__restrict__ type,
                                                    const float2 *__restrict__ psi, const float2 *__restrict__ ref,
                                                    Geometry g, Physics ph, Boundary bd, int *__restrict__ flag,
                                                    double chi)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    const int r = blk * FACE_NT + threadIdx.x;
    if (r >= bd.n_out) return;
    const OutletRec rec = bd.out[r];
    int x, y, z;
    coords_of(g, rec.bN, x, y, z);
    const uint32_t tw = type[rec.bN];
    const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
    float fa[Q], fb[Q];
    const float2 rf = ref[rec.bN];
    gather<DIM, STORE>(src, g, p, tw, x, y, z, fa, rf.x);
    gather<DIM, STORE>(src + (int64_t)Q * g.Ppad, g, p, tw, x, y, z, fb, rf.y);
    float r1, r2, J1[3], J2[3];
    moments_of<DIM>(fa, r1, J1);
    moments_of<DIM>(fb, r2, J2);
    const float *fF = bd.faceF + (int64_t)rec.slotN * 6;
    float F1[3] = {fF[0], fF[1], fF[2]}, F2[3] = {fF[3], fF[4], fF[5]}, u[3];
    const float rt = r1 + r2;
    static_for<3>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        u[d] = (J1[d] + J2[d] + 0.5f * (F1[d] + F2[d])) / rt;
    });
    if (rec.slotP >= 0) {
        // eq. (22): the outward velocity is chi times that of x_{N-1}
        const float un = (float)(chi * (double)bd.faceU[rec.slotP]) * bd.out_sign;
        if (bd.out_axis == 0) u[0] = un;
        else if (bd.out_axis == 1) u[1] = un;
        else u[2] = un;
    }
    if (!(rt > 0.0f) || !isfinite(rt) || !isfinite(u[0] + u[1] + u[2])) *flag = 1;
    // reference density of the node that reads population i next step
    auto dest_psi = [&](auto ic) -> float2 {
        constexpr int i = decltype(ic)::value;
        if constexpr (!Codec<STORE>::REF) return make_float2(0.0f, 0.0f);
        if ((tw >> Lat<DIM>::OPP[i]) & 1u) return psi[rec.bN];
        const int qx = map_axis(x + Lat<DIM>::E[i][0], g.n[0], g.periodic[0]);
        const int qy = map_axis(y + Lat<DIM>::E[i][1], g.n[1], g.periodic[1]);
        const int qz = DIM == 3 ? map_axis(z + Lat<DIM>::E[i][2], g.n[2], g.periodic[2]) : 0;
        return psi[(int64_t)qx + (int64_t)g.n[0] * ((int64_t)qy + (int64_t)g.n[1] * qz)];
    };
    float fo[Q];
    PairF<DIM> q;
    to_pairs<DIM>(fa, q);
    const Rates s1 = {ph.se[0], ph.seps[0], ph.sq, ph.snu[0]};
    collide_pairs<DIM, STORE == 0>(q, r1, J1, u, F1, s1, fo);
    static_for<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        Codec<STORE>::st(dst + (int64_t)i * g.Ppad + p, fo[i], weight<DIM>(i), dest_psi(ic).x);
    });
    to_pairs<DIM>(fb, q);
    const Rates s2 = {ph.se[1], ph.seps[1], ph.sq, ph.snu[1]};
    collide_pairs<DIM, STORE == 0>(q, r2, J2, u, F2, s2, fo);
    T *d2 = dst + (int64_t)Q * g.Ppad;
    static_for<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        Codec<STORE>::st(d2 + (int64_t)i * g.Ppad + p, fo[i], weight<DIM>(i), dest_psi(ic).y);
    });
}

// ---------------------------------------------------------------------------
// k_inlet: blocks [0, nb_in) rebuild the entering populations of the inlet
// nodes (eqs. 13-19); blocks [nb_in, ...) sum u.n_o over x_{N-1} (eq. 21).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__device__ __forceinline__ void inlet_body(int blk, typename Codec<STORE>::T *__restrict__ dst,
                                                   const uint32_t *__restrict__ type,
                                                   const float2 *__restrict__ psi, Geometry g, Boundary bd,
                                                   int nb_in)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[2 * FACE_NT / 64];
    if ((int)blk < nb_in) {
        const int r = blk * FACE_NT + threadIdx.x;
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
        const float un = pt.sign * pt.u_n;
        const float up[3] = {pt.axis == 0 ? un : 0.0f, pt.axis == 1 ? un : 0.0f, pt.axis == 2 ? un : 0.0f};
        // rho_k(x2), u(x2) from the streamed f at t+1 with this step's force
        float fa2[Q], fb2[Q], ra2 = 0.f, rb2 = 0.f, u2[3] = {0.f, 0.f, 0.f};
        if (x2_fluid) {
            float Ja[3], Jb[3];
            // f(t+1) is read with psi(t) as the reference density
            const float2 r2f = psi[rec.b2];
            gather<DIM, STORE>(dst, g, p2, tw2, x2, y2, z2, fa2, r2f.x);
            gather<DIM, STORE>(dst + (int64_t)Q * g.Ppad, g, p2, tw2, x2, y2, z2, fb2, r2f.y);
            moments_of<DIM>(fa2, ra2, Ja);
            moments_of<DIM>(fb2, rb2, Jb);
            const float *F2 = bd.faceF + (int64_t)rec.slot2 * 6;
            const float rt = ra2 + rb2;
            static_for<3>([&](auto dc) {
                constexpr int d = decltype(dc)::value;
                u2[d] = (Ja[d] + Jb[d] + 0.5f * (F2[d] + F2[3 + d])) / rt;
            });
        } else {
            static_for<Q>([&](auto ic) { fa2[decltype(ic)::value] = 0.0f; fb2[decltype(ic)::value] = 0.0f; });
        }
        const float *F1 = bd.faceF + (int64_t)rec.slot1 * 6;
        static_for<2>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            T *dk = dst + (int64_t)k * Q * g.Ppad;
            const float rho_p = pt.rho[k];
            const float rho2 = k == 0 ? ra2 : rb2;
            const float(&f2)[Q] = k == 0 ? fa2 : fb2;
            float f1[Q];
            const float2 r1f = psi[rec.b1];
            const float rref1 = k == 0 ? r1f.x : r1f.y;
            // the populations that leave x1: the entering ones are replaced
            // below, so their ghost slots (a line of their own when the face
            // is normal to the fastest memory axis) are not read
            static_for<Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                f1[i] = e_axis<DIM>(i, pt.axis) * pt.sign > 0
                            ? 0.0f
                            : gather1<DIM, STORE>(dk, g, p1, tw1, x1, y1, z1, i, rref1);
            });
            // eq. (13)/(14) on the populations entering the domain
            static_for<Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if (e_axis<DIM>(i, pt.axis) * pt.sign > 0) {
                    const float neq = x2_fluid ? f2[i] - feq<DIM>(i, rho2, u2) : 0.0f;
                    f1[i] = feq<DIM>(i, rho_p, up) + neq;
                }
            });
            if (pt.alpha_on) {
                // eqs. (15)-(19): alpha_i = w_i sum_d e_id dJ_d / D_d over the
                // entering set, dJ = rho_k^p u^p - (sum_i e_i f_i + F^k/2)
                float rr, J[3], D[3] = {0.f, 0.f, 0.f};
                moments_of<DIM>(f1, rr, J);
                static_for<Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    if (e_axis<DIM>(i, pt.axis) * pt.sign > 0) {
                        static_for<3>([&](auto dc) {
                            constexpr int d = decltype(dc)::value;
                            constexpr int e = Lat<DIM>::E[i][d];
                            if constexpr (e != 0) D[d] += weight<DIM>(i);
                        });
                    }
                });
                float dJ[3];
                static_for<3>([&](auto dc) {
                    constexpr int d = decltype(dc)::value;
                    dJ[d] = rho_p * up[d] - (J[d] + 0.5f * F1[3 * k + d]);
                });
                static_for<Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    if (e_axis<DIM>(i, pt.axis) * pt.sign > 0) {
                        float a = 0.0f;
                        static_for<3>([&](auto dc) {
                            constexpr int d = decltype(dc)::value;
                            constexpr int e = Lat<DIM>::E[i][d];
                            if constexpr (e != 0) a += weight<DIM>(i) * (float)e * dJ[d] / D[d];
                        });
                        f1[i] += a;
                    }
                });
            }
            static_for<Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if (e_axis<DIM>(i, pt.axis) * pt.sign > 0)
                    Codec<STORE>::st(dk + (int64_t)i * g.Ppad + src_slot<DIM>(g, x1, y1, z1, i), f1[i],
                                     weight<DIM>(i), rref1);
            });
        });
        return;
    }
    // eq. (21): partial sums of the outward normal velocity over x_{N-1}
    const int r = (blk - nb_in) * FACE_NT + threadIdx.x;
    double su = 0.0, cnt = 0.0;
    if (r < bd.n_out) {
        const OutletRec rec = bd.out[r];
        if (rec.slotP >= 0) {
            int x, y, z;
            coords_of(g, rec.bP, x, y, z);
            const uint32_t tw = type[rec.bP];
            const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
            float rt = 0.f, J = 0.f;
            static_for<2>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                float f[Q], rk, Jk[3];
                const float2 rpf = psi[rec.bP];
                gather<DIM, STORE>(dst + (int64_t)k * Q * g.Ppad, g, p, tw, x, y, z, f, k == 0 ? rpf.x : rpf.y);
                moments_of<DIM>(f, rk, Jk);
                rt += rk;
                J += bd.out_sign * pick3(Jk, bd.out_axis);
            });
            const float *F = bd.faceF + (int64_t)rec.slotP * 6;
            const float Fa[3] = {F[0], F[1], F[2]}, Fb[3] = {F[3], F[4], F[5]};
            J += 0.5f * bd.out_sign * (pick3(Fa, bd.out_axis) + pick3(Fb, bd.out_axis));
            su = (double)(J / rt);
            cnt = 1.0;
        }
    }
    block_sum2<FACE_NT>(su, cnt, s_red);
    if (threadIdx.x == 0) {
        bd.ucpart[2 * (blk - nb_in)] = su;
        bd.ucpart[2 * (blk - nb_in) + 1] = cnt;
    }
}

template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_inlet(typename Codec<STORE>::T *__restrict__ dst,
                                                   const uint32_t *__restrict__ type,
                                                   const float2 *__restrict__ psi, Geometry g, Boundary bd,
                                                   int nb_in)
{
    inlet_body<DIM, STORE>((int)blockIdx.x, dst, type, psi, g, bd, nb_in);
}

// ---------------------------------------------------------------------------
// k_faces: the first launch after the node update.  chi from this step's
// sums; blocks [0, nb_out) collide the outlet column, blocks [nb_out,
// nb_out + nb_in) rebuild inlet nodes (only when no inlet node pulls from the
// outlet column, checked at creation, so the two sets are independent).
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_faces(const typename Codec<STORE>::T *__restrict__ src,
                                                   typename Codec<STORE>::T *__restrict__ dst,
                                                   const uint32_t *__restrict__ type,
                                                   const float2 *__restrict__ psi, const float2 *__restrict__ ref,
                                                   Geometry g, Physics ph, Boundary bd, int *__restrict__ flag,
                                                   const unsigned long long *__restrict__ acc,
                                                   unsigned long long *__restrict__ next, int nb_out, int nb_in)
{
    const int blk = (int)blockIdx.x;
    const double chi = chi_from(bd, acc, next, blk == 0 && threadIdx.x == 0);
    if (blk < nb_out) outlet_body<DIM, STORE>(blk, src, dst, type, psi, ref, g, ph, bd, flag, chi);
    else if (blk - nb_out < nb_in) inlet_body<DIM, STORE>(blk - nb_out, dst, type, psi, g, bd, nb_in);
}

// ---------------------------------------------------------------------------
// k_outlet_fill: eq. (20) for the populations entering through the outlet.
// ---------------------------------------------------------------------------
template <int DIM, int STORE>
__device__ __forceinline__ void outlet_fill_body(int blk, const typename Codec<STORE>::T *__restrict__ src,
                                                         typename Codec<STORE>::T *__restrict__ dst,
                                                         const uint32_t *__restrict__ type,
                                                         const float2 *__restrict__ psi,
                                                         const float2 *__restrict__ ref, Geometry g, Boundary bd)
{
    using T = typename Codec<STORE>::T;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ double s_red[2 * FACE_NT / 64];
    double su, cnt;
    reduce_partials<FACE_NT>(bd.ucpart, bd.n_ucpart, su, cnt, s_red);
    double Uc = cnt > 0.0 ? su / cnt : 0.0;
    const bool clamped = Uc < 0.0;
    if (clamped) Uc = 0.0;
    if (blk == 0 && threadIdx.x == 0) {
        bd.scal[SC_UC] = Uc;
        if (clamped) bd.scal[SC_CLAMPS] += 1.0;
    }
    const int r = blk * FACE_NT + threadIdx.x;
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
    // f(t) of x_N from the FP32 history; f(t+1) is stored for x_N with
    // psi(t) as its reference density, and x' is read at t+1 with psi(t)
    const float2 rt1 = psi[rec.bN];
    const float2 rp = rec.slotP >= 0 ? psi[rec.bP] : make_float2(0.0f, 0.0f);
    static_for<2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        T *dk = dst + (int64_t)k * Q * g.Ppad;
        const float r1 = k == 0 ? rt1.x : rt1.y, rpk = k == 0 ? rp.x : rp.y;
        static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (e_axis<DIM>(i, bd.out_axis) * bd.out_sign < 0) {
                const int64_t a = (int64_t)i * g.Ppad + src_slot<DIM>(g, x, y, z, i);
                float *h = bd.hist + ((int64_t)k * Q + i) * bd.n_slots + rec.slotN;
                const float prev = *h;
                float v = prev;
                if (rec.slotP >= 0) {
                    const float fp = gather1<DIM, STORE>(dk, g, pp, twp, xp, yp, zp, i, rpk);
                    v = (prev + uc * fp) / (1.0f + uc);
                }
                *h = v;
                Codec<STORE>::st(dk + a, v, weight<DIM>(i), r1);
            }
        });
    });
}

template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_outlet_fill(const typename Codec<STORE>::T *__restrict__ src,
                                                         typename Codec<STORE>::T *__restrict__ dst,
                                                         const uint32_t *__restrict__ type,
                                                         const float2 *__restrict__ psi,
                                                         const float2 *__restrict__ ref, Geometry g, Boundary bd)
{
    outlet_fill_body<DIM, STORE>((int)blockIdx.x, src, dst, type, psi, ref, g, bd);
}

// ---------------------------------------------------------------------------
// State exchange: canonical f[2][Q][N] (FP64) <-> population slots.
// ---------------------------------------------------------------------------
// The state's own densities become the reference densities of its slots
// (every slot of the node is read by the node itself), written to ref.
template <int DIM, int STORE>
__global__ void k_scatter(typename Codec<STORE>::T *__restrict__ dst, const uint32_t *__restrict__ type,
                          Geometry g, Boundary bd, const double *__restrict__ f, float2 *__restrict__ ref)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.N) return;
    const uint32_t tw = type[b];
    if (tw & T_SOLID) {
        ref[b] = make_float2(-0.0f, -0.0f);
        return;
    }
    int x, y, z;
    coords_of(g, b, x, y, z);
    const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
    const int64_t bo = caller_index(g, x, y, z);
    float rr[2];
    for (int k = 0; k < 2; k++) {
        double r = 0.0;
        for (int i = 0; i < Q; i++) r += f[((int64_t)k * Q + i) * g.N + bo];
        rr[k] = (float)r;
    }
    ref[b] = make_float2(rr[0], rr[1]);
    for (int k = 0; k < 2; k++) {
        auto *dk = dst + (int64_t)k * Q * g.Ppad;
        static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const float v = (float)f[((int64_t)k * Q + g.dmap[i]) * g.N + bo];
            Codec<STORE>::st(dk + slot_of<DIM>(g, p, tw | T_EDGE, x, y, z, i), v, weight<DIM>(i), rr[k]);
            // the outlet history of eq. (20) starts from the state itself
            if ((tw & T_OUTLET) && e_axis<DIM>(i, bd.out_axis) * bd.out_sign < 0)
                bd.hist[((int64_t)k * Q + i) * bd.n_slots + bd.bslot[b]] = v;
        });
    }
}

template <int DIM, int STORE>
__global__ void k_gather_state(const typename Codec<STORE>::T *__restrict__ src, const uint32_t *__restrict__ type,
                               const float2 *__restrict__ ref, Geometry g, Boundary bd, double *__restrict__ f)
{
    constexpr int Q = Lat<DIM>::Q;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= g.N) return;
    const uint32_t tw = type[b];
    int x, y, z;
    coords_of(g, b, x, y, z);
    const int64_t bo = caller_index(g, x, y, z);
    for (int k = 0; k < 2; k++) {
        if (tw & T_SOLID) {
            for (int i = 0; i < Q; i++) f[((int64_t)k * Q + i) * g.N + bo] = 0.0;
            continue;
        }
        const int64_t p = pidx(g, x, y, DIM == 3 ? z : -1);
        float v[Q];
        const float2 rf = ref[b];
        gather<DIM, STORE>(src + (int64_t)k * Q * g.Ppad, g, p, tw | T_EDGE, x, y, z, v, k == 0 ? rf.x : rf.y);
        static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            // populations entering through the outlet: the FP32 history (the
            // stored copy is its rounding)
            if ((tw & T_OUTLET) && e_axis<DIM>(i, bd.out_axis) * bd.out_sign < 0)
                v[i] = bd.hist[((int64_t)k * Q + i) * bd.n_slots + bd.bslot[b]];
            f[((int64_t)k * Q + g.dmap[i]) * g.N + bo] = (double)v[i];
        });
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
    if (u0) {
        u[0] = (float)u0[b];
        u[1] = (float)u0[N + b];
        u[2] = (float)u0[2 * N + b];
    }
    for (int k = 0; k < 2; k++) {
        const float r = (float)rho0[k * N + b];
        static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            f[((int64_t)k * Q + i) * N + b] = (double)feq<DIM>(i, r, u);
        });
    }
}

// Per-block FP64 partial sums of rho_1 and rho_2 over fluid nodes.
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_mass(const typename Codec<STORE>::T *__restrict__ src,
                                              const uint32_t *__restrict__ type,
                                              const float2 *__restrict__ ref, Geometry g,
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
        const float2 rf = ref[b];
        gather<DIM, STORE>(src, g, p, tw | T_EDGE, x, y, z, f, rf.x);
        static_for<Q>([&](auto ic) { m1 += (double)f[decltype(ic)::value]; });
        gather<DIM, STORE>(src + (int64_t)Q * g.Ppad, g, p, tw | T_EDGE, x, y, z, f, rf.y);
        static_for<Q>([&](auto ic) { m2 += (double)f[decltype(ic)::value]; });
    }
    block_sum2<256>(m1, m2, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = m1;
        part[2 * blockIdx.x + 1] = m2;
    }
}

static __global__ void k_reduce2(const double *__restrict__ part, int n, double *__restrict__ out)
{
    __shared__ double s_red[8];
    double a, b;
    reduce_partials<256>(part, n, a, b, s_red);
    if (threadIdx.x == 0) { out[0] = a; out[1] = b; }
}

// ---------------------------------------------------------------------------
// Batched step: every member of a batch advanced by one launch per stage.
// Members share the lattice, the storage and the node-update configuration
// and differ in everything else (size, geometry, physics, faces).  The A/B
// parity `cur` is common to all members.
// ---------------------------------------------------------------------------

// A member's descriptor is read-only for the whole launch: the batch kernels
// read it through the constant address space, so its fields come in by
// scalar loads into uniform registers, as kernel arguments do (through a
// generic pointer they were vector loads, and the node update held the
// descriptor in some twenty vector registers).
using CMember = const __attribute__((address_space(4))) Member;

// A copy of a structure held in the constant address space, word by word so
// that it compiles to scalar loads.
template <class S>
__device__ __forceinline__ S const_copy(const __attribute__((address_space(4))) S *p)
{
    static_assert(sizeof(S) % 4 == 0, "whole words");
    S v;
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t *d = (uint32_t *)&v;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / 4); k++) d[k] = q[k];
    return v;
}

// Largest i in [0, n) with start[i] <= v (start is nondecreasing, start[0] = 0).
__device__ __forceinline__ int member_of(const int *__restrict__ start, int n, int v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);   // uniform over the block
}

template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_psi_batch(BatchTab t, int cur)
{
    using T = typename Codec<STORE>::T;
    const int i = member_of(t.psi0, t.n, (int)blockIdx.x);
    CMember *m = (CMember *)(t.m + i);
    psi_body<DIM, STORE>((int)blockIdx.x - t.psi0[i], (const T *)m->f[cur], m->type, const_copy(&m->g),
                         (float2 *)m->psi[cur], (const float2 *)m->psi[cur ^ 1]);
}

// Persistent node update over the concatenated work items of all members.
// The blocks (a multiple of 8) step through virtual block indices v; v % 8 is
// the XCD of the block, and the items are dealt to the XCDs as in k_main, in
// groups of MAIN_XCD_GROUP consecutive items per turn.
template <int DIM, int STORE, int PSRC, int TX, int TY, int W, int ZC, int KEEPB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STORE != 0 ? 4 : 1)))
void k_main_batch(BatchTab t, int cur)
{
    using T = typename Codec<STORE>::T;
    const int total = t.item0[t.n];
    const int span = (total + 8 * MAIN_XCD_GROUP - 1) / (8 * MAIN_XCD_GROUP) * (8 * MAIN_XCD_GROUP);
    for (int v = (int)blockIdx.x; v < span; v += (int)gridDim.x) {
        const int S = v / 8, r = v % 8;
        const int w = ((S / MAIN_XCD_GROUP) * 8 + r) * MAIN_XCD_GROUP + S % MAIN_XCD_GROUP;
        if (w >= total) continue;
        const int i = __builtin_amdgcn_readfirstlane(t.item_mem[w]);
        CMember *m = (CMember *)(t.m + i);
        const Geometry g = const_copy(&m->g);
        const Physics ph = const_copy(&m->ph);
        const Boundary bd = const_copy(&m->bd);
        main_item<DIM, STORE, PSRC, TX, TY, W, ZC, KEEPB>((const T *)m->f[cur], (T *)m->f[cur ^ 1], m->type,
                                                          (const float2 *)m->psi[cur],
                                                          (const float2 *)m->psi[cur ^ 1], g, ph, bd,
                                                          m->tiles_x, m->tiles_y, m->item_list[w - t.item0[i]],
                                                          m->flag, bd.qacc + 2 * cur);
    }
}

// eq. (23) from the sums of each member, one thread per member
static __global__ __launch_bounds__(64) void k_chi_batch(BatchTab t, int cur)
{
    const int i = (int)(blockIdx.x * 64 + threadIdx.x);
    if (i >= t.n) return;
    const Boundary bd = const_copy(&((CMember *)(t.m + i))->bd);
    (void)chi_from(bd, bd.qacc + 2 * cur, bd.qacc + 2 * (cur ^ 1), true);
}

template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_outlet_batch(BatchTab t, int cur)
{
    using T = typename Codec<STORE>::T;
    const int i = member_of(t.out0, t.n, (int)blockIdx.x);
    CMember *m = (CMember *)(t.m + i);
    const Boundary bd = const_copy(&m->bd);
    outlet_body<DIM, STORE>((int)blockIdx.x - t.out0[i], (const T *)m->f[cur], (T *)m->f[cur ^ 1], m->type,
                            (const float2 *)m->psi[cur], (const float2 *)m->psi[cur ^ 1], const_copy(&m->g),
                            const_copy(&m->ph), bd, m->flag, bd.scal[SC_CHI]);
}

template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_inlet_batch(BatchTab t, int cur)
{
    using T = typename Codec<STORE>::T;
    const int i = member_of(t.inl0, t.n, (int)blockIdx.x);
    CMember *m = (CMember *)(t.m + i);
    inlet_body<DIM, STORE>((int)blockIdx.x - t.inl0[i], (T *)m->f[cur ^ 1], m->type, (const float2 *)m->psi[cur],
                           const_copy(&m->g), const_copy(&m->bd), m->nb_in);
}

template <int DIM, int STORE>
__global__ __launch_bounds__(FACE_NT) void k_outlet_fill_batch(BatchTab t, int cur)
{
    using T = typename Codec<STORE>::T;
    const int i = member_of(t.fill0, t.n, (int)blockIdx.x);
    CMember *m = (CMember *)(t.m + i);
    outlet_fill_body<DIM, STORE>((int)blockIdx.x - t.fill0[i], (const T *)m->f[cur], (T *)m->f[cur ^ 1], m->type,
                                 (const float2 *)m->psi[cur], (const float2 *)m->psi[cur ^ 1],
                                 const_copy(&m->g), const_copy(&m->bd));
}

// ---------------------------------------------------------------------------
// Droplet labels.  The dispersed phase is the set of fluid nodes of a box
// whose component-k density (summed from the current populations) exceeds a
// threshold; droplets are its face-connected components.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool in_box(const Box3 &bx, int x, int y, int z)
{
    return x >= bx.lo[0] && x < bx.hi[0] && y >= bx.lo[1] && y < bx.hi[1] && z >= bx.lo[2] && z < bx.hi[2];
}

// rho_k of a fluid node from its post-streaming populations
template <int DIM, int STORE>
__device__ __forceinline__ float node_rho(const typename Codec<STORE>::T *__restrict__ src, const Geometry &g,
                                          uint32_t tw, int x, int y, int z, int k, float rr)
{
    constexpr int Q = Lat<DIM>::Q;
    float f[Q];
    gather<DIM, STORE>(src + (int64_t)k * Q * g.Ppad, g, pidx(g, x, y, DIM == 3 ? z : -1), tw, x, y, z, f, rr);
    float r = 0.0f;
    static_for<Q>([&](auto ic) { r += f[decltype(ic)::value]; });
    return r;
}

// count of dispersed nodes in the box, added to *out (zeroed by k_zero64)
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_probe(const typename Codec<STORE>::T *__restrict__ src,
                                               const uint32_t *__restrict__ type, const float2 *__restrict__ ref,
                                               Geometry g, int k, Box3 bx, float thr,
                                               unsigned long long *__restrict__ out)
{
    const int ex = bx.hi[0] - bx.lo[0], ey = bx.hi[1] - bx.lo[1], ez = bx.hi[2] - bx.lo[2];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int hit = 0;
    if (v < (int64_t)ex * ey * ez) {
        const int x = bx.lo[0] + (int)(v % ex), y = bx.lo[1] + (int)((v / ex) % ey),
                  z = bx.lo[2] + (int)(v / ((int64_t)ex * ey));
        const int64_t b = (int64_t)x + (int64_t)g.n[0] * ((int64_t)y + (int64_t)g.n[1] * z);
        const uint32_t tw = type[b];
        if (!(tw & T_SOLID)) {
            const float2 rf = ref[b];
            hit = node_rho<DIM, STORE>(src, g, tw | T_EDGE, x, y, z, k, k == 0 ? rf.x : rf.y) > thr;
        }
    }
    const unsigned long long c = __popcll(__ballot(hit));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

static __global__ void k_zero64(unsigned long long *p) { *p = 0ull; }

// label = own box index on dispersed nodes of the box, -1 elsewhere
template <int DIM, int STORE>
__global__ __launch_bounds__(256) void k_lab_init(const typename Codec<STORE>::T *__restrict__ src,
                                                  const uint32_t *__restrict__ type,
                                                  const float2 *__restrict__ ref, Geometry g, int k, Box3 bx,
                                                  float thr, int *__restrict__ lab)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= g.N) return;
    int x, y, z;
    coords_of(g, b, x, y, z);
    const uint32_t tw = type[b];
    bool in = !(tw & T_SOLID) && in_box(bx, x, y, z);
    if (in) {
        const float2 rf = ref[b];
        in = node_rho<DIM, STORE>(src, g, tw | T_EDGE, x, y, z, k, k == 0 ? rf.x : rf.y) > thr;
    }
    lab[b] = in ? (int)b : -1;
}

// One pass of minimum-label propagation over face neighbours plus pointer
// jumping (lab[lab[b]] <= lab[b]).  Labels only decrease, so passes may run
// concurrently and in any order; the fixed point is the smallest box index
// of each component.
static __global__ __launch_bounds__(256) void k_lab_prop(Geometry g, int dim, int *lab, int *changed)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= g.N) return;
    const int l = lab[b];
    if (l < 0) return;
    int x, y, z;
    coords_of(g, b, x, y, z);
    int m = l;
    auto take = [&](int64_t nb) {
        const int v = lab[nb];
        if (v >= 0 && v < m) m = v;
    };
    if (x > 0) take(b - 1);
    if (x + 1 < g.n[0]) take(b + 1);
    if (y > 0) take(b - g.n[0]);
    if (y + 1 < g.n[1]) take(b + g.n[0]);
    if (dim == 3) {
        const int64_t pl = (int64_t)g.n[0] * g.n[1];
        if (z > 0) take(b - pl);
        if (z + 1 < g.n[2]) take(b + pl);
    }
    const int j = lab[m];
    if (j >= 0 && j < m) m = j;
    if (m < l) {
        lab[b] = m;
        *changed = 1;
    }
}

// roots (lab[b] == b) get consecutive slots in an arbitrary order; the host
// orders the components afterwards
static __global__ __launch_bounds__(256) void k_lab_roots(Geometry g, const int *__restrict__ lab,
                                                          int *__restrict__ slot, int *__restrict__ n_roots)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= g.N) return;
    if (lab[b] == (int)b) slot[b] = atomicAdd(n_roots, 1);
}

// per component: size, smallest caller-frame index, caller-frame bounding box
// (integer atomics: the result does not depend on the order)
static __global__ __launch_bounds__(256) void k_lab_stats_init(CompStat *st, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    st[i].size = 0ull;
    st[i].first = ~0ull;
    for (int a = 0; a < 3; a++) {
        st[i].lo[a] = 0x7fffffff;
        st[i].hi[a] = -1;
    }
}

static __global__ __launch_bounds__(256) void k_lab_stats(Geometry g, const int *__restrict__ lab,
                                                          const int *__restrict__ slot, CompStat *st)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= g.N) return;
    const int l = lab[b];
    if (l < 0) return;
    CompStat *c = st + slot[l];
    int x, y, z;
    coords_of(g, b, x, y, z);
    const int mc[3] = {x, y, z};
    atomicAdd(&c->size, 1ull);
    atomicMin(&c->first, (unsigned long long)caller_index(g, x, y, z));
    for (int a = 0; a < 3; a++) {
        atomicMin(&c->lo[g.ax[a]], mc[a]);
        atomicMax(&c->hi[g.ax[a]], mc[a] + 1);
    }
}

}  // namespace lbm
