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
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

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

// Relaxation rates of one component (eq. 4): s_rho = s_j = 1.
struct Rates {
    float se, seps, sq, snu;
};

// Post-collision populations of one node and one component, in place.
//   f    : populations f_i^k (post-streaming)
//   rho  : rho_k ; J : sum_i e_i f_i^k
//   u    : common velocity used by feq and the forcing term
//   F    : total force on component k
template <int DIM>
__device__ __forceinline__ void collide(float (&f)[Lat<DIM>::Q], float rho, const float (&J)[3],
                                        const float (&u)[3], const float (&F)[3], const Rates &s)
{
    constexpr int Q = Lat<DIM>::Q;
    float m[Q];
#pragma unroll
    for (int r = 0; r < Q; r++) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const int t = trow<DIM>(r, i);
            if (t == 1) acc += f[i];
            else if (t == -1) acc -= f[i];
            else if (t != 0) acc = fmaf((float)t, f[i], acc);
        }
        m[r] = acc;
    }
    const float ux = u[0], uy = u[1], uz = u[2];
    const float Fx = F[0], Fy = F[1], Fz = F[2];
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
    // d[r] = s_r (m_r - meq_r) - (1 - s_r/2) Fm_r
    float d[Q];
    const float he = 1.0f - 0.5f * s.se, hps = 1.0f - 0.5f * s.seps;
    const float hq = 1.0f - 0.5f * s.sq, hn = 1.0f - 0.5f * s.snu;
    d[0] = 0.0f;
    if constexpr (DIM == 2) {
        d[1] = s.se * (m[1] - rho * (-2.0f + 3.0f * uu)) - he * (6.0f * uF);
        d[2] = s.seps * (m[2] - rho * (1.0f - 3.0f * uu)) - hps * (-6.0f * uF);
        d[3] = (J[0] - rho * ux) - 0.5f * Fx;
        d[4] = s.sq * (m[4] + rho * ux) - hq * (-Fx);
        d[5] = (J[1] - rho * uy) - 0.5f * Fy;
        d[6] = s.sq * (m[6] + rho * uy) - hq * (-Fy);
        d[7] = s.snu * (m[7] - rho * (ux * ux - uy * uy)) - hn * (2.0f * (ux * Fx - uy * Fy));
        d[8] = s.snu * (m[8] - rho * ux * uy) - hn * (ux * Fy + uy * Fx);
    } else {
        const float c23 = 2.0f / 3.0f;
        const float pxx = 3.0f * ux * ux - uu, pww = uy * uy - uz * uz;
        const float fxx = 3.0f * ux * Fx - uF, fww = uy * Fy - uz * Fz;
        d[1] = s.se * (m[1] - rho * (-11.0f + 19.0f * uu)) - he * (38.0f * uF);
        d[2] = s.seps * (m[2] - rho * (3.0f - 5.5f * uu)) - hps * (-11.0f * uF);
        d[3] = (J[0] - rho * ux) - 0.5f * Fx;
        d[4] = s.sq * (m[4] + c23 * rho * ux) - hq * (-c23 * Fx);
        d[5] = (J[1] - rho * uy) - 0.5f * Fy;
        d[6] = s.sq * (m[6] + c23 * rho * uy) - hq * (-c23 * Fy);
        d[7] = (J[2] - rho * uz) - 0.5f * Fz;
        d[8] = s.sq * (m[8] + c23 * rho * uz) - hq * (-c23 * Fz);
        d[9] = s.snu * (m[9] - rho * pxx) - hn * (2.0f * fxx);
        d[10] = s.snu * (m[10] + 0.5f * rho * pxx) - hn * (-fxx);
        d[11] = s.snu * (m[11] - rho * pww) - hn * (2.0f * fww);
        d[12] = s.snu * (m[12] + 0.5f * rho * pww) - hn * (-fww);
        d[13] = s.snu * (m[13] - rho * ux * uy) - hn * (ux * Fy + uy * Fx);
        d[14] = s.snu * (m[14] - rho * uy * uz) - hn * (uy * Fz + uz * Fy);
        d[15] = s.snu * (m[15] - rho * ux * uz) - hn * (ux * Fz + uz * Fx);
        d[16] = s.sq * m[16];
        d[17] = s.sq * m[17];
        d[18] = s.sq * m[18];
    }
#pragma unroll
    for (int r = 1; r < Q; r++) d[r] *= 1.0f / (float)tnorm<DIM>(r);
#pragma unroll
    for (int i = 0; i < Q; i++) {
        float acc = f[i];
#pragma unroll
        for (int r = 1; r < Q; r++) {
            const int t = trow<DIM>(r, i);
            if (t == 1) acc -= d[r];
            else if (t == -1) acc += d[r];
            else if (t != 0) acc = fmaf(-(float)t, d[r], acc);
        }
        f[i] = acc;
    }
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
