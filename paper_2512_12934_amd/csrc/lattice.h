// lattice.h -- compile-time lattice constants and the per-node MRT collision
// of the HIP solver (device side).
//
// D2Q9 (Sec. II A): velocities in the order fixed by the unknown sets of
// Sec. II B; moment basis rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy whose
// first three rows are those printed in eq. (3) and whose order matches S of
// eq. (4).  D3Q19 (not in the paper): 19-velocity lattice with the orthogonal
// polynomial moment basis rho, e, eps, j, q per axis, 3p_xx, 3pi_xx, p_ww,
// pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z.
//
// The collision works in moment space with closed-form equilibrium moments
// (eq. 6) and forcing moments (eq. 9):
//     f* = f - T^-1 [ S (m - m_eq) - (I - S/2) F_m ],   m = T f   (eq. 1)
// where T^-1 = T^T diag(1/|row|^2) because the rows are orthogonal.
//
// Every loop over directions, moment rows and stencil offsets is expanded at
// compile time (static_for), so all matrix entries and weights are literals
// in the generated code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace lbm {

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1.
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int DIM> struct Lat;

template <> struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int E[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

template <> struct Lat<3> {
    static constexpr int Q = 19;
    static constexpr int E[19][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

template <int DIM>
__host__ __device__ constexpr int e2_of(int i)
{
    return Lat<DIM>::E[i][0] * Lat<DIM>::E[i][0] + Lat<DIM>::E[i][1] * Lat<DIM>::E[i][1] +
           Lat<DIM>::E[i][2] * Lat<DIM>::E[i][2];
}

// Lattice weights: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36.
template <int DIM>
__host__ __device__ constexpr float weight(int i)
{
    return DIM == 2 ? (e2_of<DIM>(i) == 0 ? 4.0f / 9.0f : (e2_of<DIM>(i) == 1 ? 1.0f / 9.0f : 1.0f / 36.0f))
                    : (e2_of<DIM>(i) == 0 ? 1.0f / 3.0f : (e2_of<DIM>(i) == 1 ? 1.0f / 18.0f : 1.0f / 36.0f));
}

// Integer entry T[r][i] of the moment matrix.
template <int DIM>
__host__ __device__ constexpr int trow(int r, int i)
{
    const int x = Lat<DIM>::E[i][0], y = Lat<DIM>::E[i][1], z = Lat<DIM>::E[i][2];
    const int s = x * x + y * y + z * z;
    if (DIM == 2) {
        switch (r) {
        case 0: return 1;
        case 1: return 3 * s - 4;
        case 2: return (9 * s * s - 21 * s + 8) / 2;  // 4 - 21 s/2 + 9 s^2/2
        case 3: return x;
        case 4: return (3 * s - 5) * x;
        case 5: return y;
        case 6: return (3 * s - 5) * y;
        case 7: return x * x - y * y;
        default: return x * y;
        }
    }
    switch (r) {
    case 0: return 1;
    case 1: return 19 * s - 30;
    case 2: return (21 * s * s - 53 * s + 24) / 2;
    case 3: return x;
    case 4: return (5 * s - 9) * x;
    case 5: return y;
    case 6: return (5 * s - 9) * y;
    case 7: return z;
    case 8: return (5 * s - 9) * z;
    case 9: return 3 * x * x - s;
    case 10: return (3 * s - 5) * (3 * x * x - s);
    case 11: return y * y - z * z;
    case 12: return (3 * s - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

template <int DIM>
__host__ __device__ constexpr int tnorm(int r)
{
    int acc = 0;
    for (int i = 0; i < Lat<DIM>::Q; i++) acc += trow<DIM>(r, i) * trow<DIM>(r, i);
    return acc;
}

// Row parity under e -> -e.
template <int DIM>
__host__ __device__ constexpr bool row_odd(int r)
{
    for (int i = 1; i < Lat<DIM>::Q; i++)
        if (trow<DIM>(r, i) != 0) return trow<DIM>(r, Lat<DIM>::OPP[i]) == -trow<DIM>(r, i);
    return false;
}

// Opposite pairs: the member listed first in the velocity order.
template <int DIM> struct Pairs {
    static constexpr int P = (Lat<DIM>::Q - 1) / 2;
    static constexpr int first(int p)
    {
        int n = 0;
        for (int i = 1; i < Lat<DIM>::Q; i++)
            if (i < Lat<DIM>::OPP[i]) {
                if (n == p) return i;
                n++;
            }
        return 0;
    }
};

// Relaxation rates of one component (eq. 4): s_rho = s_j = 1.
struct Rates {
    float se, seps, sq, snu;
};

// Populations of one node and component in pair form: s_p = f_i + f_ibar,
// d_p = f_i - f_ibar.  Even moment rows use only s_p and the rest
// population, odd rows only d_p, which halves both transforms.
template <int DIM> struct PairF {
    float f0;
    float s[Pairs<DIM>::P];
    float d[Pairs<DIM>::P];
};

template <int DIM>
__device__ __forceinline__ void to_pairs(const float (&f)[Lat<DIM>::Q], PairF<DIM> &q)
{
    q.f0 = f[0];
    static_for<Pairs<DIM>::P>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = Pairs<DIM>::first(p), o = Lat<DIM>::OPP[i];
        q.s[p] = f[i] + f[o];
        q.d[p] = f[i] - f[o];
    });
}

template <int DIM>
__device__ __forceinline__ void pair_momentum(const PairF<DIM> &q, float (&J)[3])
{
    static_for<3>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        float acc = 0.0f;
        static_for<Pairs<DIM>::P>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int e = Lat<DIM>::E[Pairs<DIM>::first(p)][d];
            if constexpr (e == 1) acc += q.d[p];
            else if constexpr (e == -1) acc -= q.d[p];
        });
        J[d] = acc;
    });
}

// Relaxed non-equilibrium part of moment row R divided by |row R|^2:
//   a_R = [ s_R (m_R - m_eq,R) - (1 - s_R/2) F_m,R ] / |T_R|^2
// with the closed-form equilibrium moments of eq. (6) and forcing moments of
// eq. (9).  Momentum rows (s_j = 1) use J - rho u - F/2 directly.
template <int DIM, int R>
__device__ __forceinline__ float relax_row(float m, float rho, const float (&J)[3], const float (&u)[3],
                                           const float (&F)[3], const Rates &s, float uu, float uF)
{
    const float ux = u[0], uy = u[1], uz = u[2];
    const float Fx = F[0], Fy = F[1], Fz = F[2];
    constexpr float inv = 1.0f / (float)tnorm<DIM>(R);
    float a = 0.0f;
    if constexpr (DIM == 2) {
        if constexpr (R == 1) a = s.se * (m - rho * (-2.0f + 3.0f * uu)) - (1.0f - 0.5f * s.se) * (6.0f * uF);
        else if constexpr (R == 2) a = s.seps * (m - rho * (1.0f - 3.0f * uu)) + (1.0f - 0.5f * s.seps) * (6.0f * uF);
        else if constexpr (R == 3) a = (J[0] - rho * ux) - 0.5f * Fx;
        else if constexpr (R == 4) a = s.sq * (m + rho * ux) + (1.0f - 0.5f * s.sq) * Fx;
        else if constexpr (R == 5) a = (J[1] - rho * uy) - 0.5f * Fy;
        else if constexpr (R == 6) a = s.sq * (m + rho * uy) + (1.0f - 0.5f * s.sq) * Fy;
        else if constexpr (R == 7)
            a = s.snu * (m - rho * (ux * ux - uy * uy)) - (1.0f - 0.5f * s.snu) * (2.0f * (ux * Fx - uy * Fy));
        else if constexpr (R == 8) a = s.snu * (m - rho * ux * uy) - (1.0f - 0.5f * s.snu) * (ux * Fy + uy * Fx);
    } else {
        constexpr float c23 = 2.0f / 3.0f;
        if constexpr (R == 1) a = s.se * (m - rho * (-11.0f + 19.0f * uu)) - (1.0f - 0.5f * s.se) * (38.0f * uF);
        else if constexpr (R == 2) a = s.seps * (m - rho * (3.0f - 5.5f * uu)) + (1.0f - 0.5f * s.seps) * (11.0f * uF);
        else if constexpr (R == 3) a = (J[0] - rho * ux) - 0.5f * Fx;
        else if constexpr (R == 4) a = s.sq * (m + c23 * rho * ux) + (1.0f - 0.5f * s.sq) * (c23 * Fx);
        else if constexpr (R == 5) a = (J[1] - rho * uy) - 0.5f * Fy;
        else if constexpr (R == 6) a = s.sq * (m + c23 * rho * uy) + (1.0f - 0.5f * s.sq) * (c23 * Fy);
        else if constexpr (R == 7) a = (J[2] - rho * uz) - 0.5f * Fz;
        else if constexpr (R == 8) a = s.sq * (m + c23 * rho * uz) + (1.0f - 0.5f * s.sq) * (c23 * Fz);
        else if constexpr (R == 9)
            a = s.snu * (m - rho * (3.0f * ux * ux - uu)) - (1.0f - 0.5f * s.snu) * (2.0f * (3.0f * ux * Fx - uF));
        else if constexpr (R == 10)
            a = s.snu * (m + 0.5f * rho * (3.0f * ux * ux - uu)) + (1.0f - 0.5f * s.snu) * (3.0f * ux * Fx - uF);
        else if constexpr (R == 11)
            a = s.snu * (m - rho * (uy * uy - uz * uz)) - (1.0f - 0.5f * s.snu) * (2.0f * (uy * Fy - uz * Fz));
        else if constexpr (R == 12)
            a = s.snu * (m + 0.5f * rho * (uy * uy - uz * uz)) + (1.0f - 0.5f * s.snu) * (uy * Fy - uz * Fz);
        else if constexpr (R == 13) a = s.snu * (m - rho * ux * uy) - (1.0f - 0.5f * s.snu) * (ux * Fy + uy * Fx);
        else if constexpr (R == 14) a = s.snu * (m - rho * uy * uz) - (1.0f - 0.5f * s.snu) * (uy * Fz + uz * Fy);
        else if constexpr (R == 15) a = s.snu * (m - rho * ux * uz) - (1.0f - 0.5f * s.snu) * (ux * Fz + uz * Fx);
        else a = s.sq * m;   // m_x, m_y, m_z: no equilibrium or forcing part
    }
    return a * inv;
}

// eq. (1) in moment space on a node in pair form; writes f* into out[Q].
// Rows are streamed: each moment is formed, relaxed and scattered back into
// the even / odd parts of the pairs before the next one.  rho must be the
// node's density, the sum of the populations in q.
template <int DIM, bool RESID>
__device__ __forceinline__ void collide_pairs(const PairF<DIM> &q, float rho, const float (&J)[3],
                                              const float (&u)[3], const float (&F)[3], const Rates &s,
                                              float (&out)[Lat<DIM>::Q])
{
    constexpr int Q = Lat<DIM>::Q;
    constexpr int P = Pairs<DIM>::P;
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    float ev[P], od[P], rest = 0.0f;
    static_for<P>([&](auto pc) {
        ev[decltype(pc)::value] = 0.0f;
        od[decltype(pc)::value] = 0.0f;
    });
    static_for<Q - 1>([&](auto rc) {
        constexpr int R = decltype(rc)::value + 1;
        constexpr bool odd = row_odd<DIM>(R);
        constexpr bool mom = DIM == 2 ? (R == 3 || R == 5) : (R == 3 || R == 5 || R == 7);
        float m = 0.0f;
        if constexpr (!mom) {
            constexpr int t0 = trow<DIM>(R, 0);
            if constexpr (t0 != 0) m = (float)t0 * q.f0;
            static_for<P>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                constexpr int t = trow<DIM>(R, Pairs<DIM>::first(p));
                const float v = odd ? q.d[p] : q.s[p];
                if constexpr (t == 1) m += v;
                else if constexpr (t == -1) m -= v;
                else if constexpr (t != 0) m = fmaf((float)t, v, m);
            });
        }
        const float a = relax_row<DIM, R>(m, rho, J, u, F, s, uu, uF);
        if constexpr (!RESID) {
            constexpr int t0 = trow<DIM>(R, 0);
            if constexpr (t0 != 0) rest = fmaf((float)t0, a, rest);
        }
        static_for<P>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int t = trow<DIM>(R, Pairs<DIM>::first(p));
            if constexpr (t != 0) {
                float &acc = odd ? od[p] : ev[p];
                if constexpr (t == 1) acc += a;
                else if constexpr (t == -1) acc -= a;
                else acc = fmaf((float)t, a, acc);
            }
        });
    });
    float moving = 0.0f;
    static_for<P>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = Pairs<DIM>::first(p), o = Lat<DIM>::OPP[i];
        const float fi = 0.5f * (q.s[p] + q.d[p]), fo = 0.5f * (q.s[p] - q.d[p]);
        out[i] = fi - ev[p] - od[p];
        out[o] = fo - ev[p] + od[p];
        if constexpr (RESID) moving += out[i] + out[o];
    });
    // RESID: the rest population is the residual of the node's density.  In
    // exact arithmetic the relaxed rows change no mass (every row but the
    // first sums to zero over the velocities); in FP32 their rounded scatter
    // into the rest population left a systematic mass drift (2e-4 of a
    // component over 20k steps of a 3-D droplet, ten times what the residual
    // leaves).  Binary16 storage rounds far more than that, and the residual
    // costs a VALU-bound binary16 node update 4%, so it scatters as well.
    if constexpr (RESID) out[0] = rho - moving;
    else out[0] = q.f0 - rest;
}

// Equilibrium of eq. (6) (second-order term over 2 cs^4), cs^2 = 1/3.
template <int DIM>
__device__ __forceinline__ float feq(int i, float rho, const float (&u)[3])
{
    const float eu = Lat<DIM>::E[i][0] * u[0] + Lat<DIM>::E[i][1] * u[1] + Lat<DIM>::E[i][2] * u[2];
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return rho * weight<DIM>(i) * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * uu);
}

// ---------------------------------------------------------------------------
// 8th-order interaction stencil (eqs. 10-11).  2-D weights as printed in
// Sec. II A over the 24 nonzero offsets of the 5x5 square; 3-D weights are the
// unique positive solution of the same isotropy conditions on the shells
// |e|^2 = 1,2,3,4,5,6,8 of the 5x5x5 cube (92 offsets).
// ---------------------------------------------------------------------------
template <int DIM>
__host__ __device__ constexpr float stencil_w(int r2)
{
    if (DIM == 2) {
        return r2 == 1 ? 4.0f / 21.0f : r2 == 2 ? 4.0f / 45.0f : r2 == 4 ? 1.0f / 60.0f
             : r2 == 5 ? 2.0f / 315.0f : r2 == 8 ? 1.0f / 5040.0f : 0.0f;
    }
    return r2 == 1 ? 4.0f / 45.0f : r2 == 2 ? 1.0f / 21.0f : r2 == 3 ? 2.0f / 105.0f
         : r2 == 4 ? 5.0f / 504.0f : r2 == 5 ? 1.0f / 315.0f : r2 == 6 ? 1.0f / 630.0f
         : r2 == 8 ? 1.0f / 5040.0f : 0.0f;
}

}  // namespace lbm
