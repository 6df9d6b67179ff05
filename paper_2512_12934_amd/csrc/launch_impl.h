// launch_impl.h -- definitions of Launcher<DIM>; included by exactly one
// translation unit per lattice.
#pragma once

#include <algorithm>
#include <utility>

#include "kernels.h"
#include "launch.h"

namespace lbm {

namespace detail {

template <int DIM> constexpr const TileCfg &cfg_at(int i) { return DIM == 2 ? CFG2[i] : CFG3[i]; }
template <int DIM> constexpr int cfg_count() { return DIM == 2 ? NCFG2 : NCFG3; }

template <int DIM, int STORE, int I>
void launch_cfg(const StepArgs &a)
{
    constexpr TileCfg c = cfg_at<DIM>(I);
    using T = typename Codec<STORE>::T;
    hipLaunchKernelGGL((k_main<DIM, STORE, c.psrc, c.tx, c.ty, c.w, c.zc, c.keepb>), dim3(a.grid), dim3(256), 0,
                       a.stream, (const T *)a.src, (T *)a.dst, a.type, (const float2 *)a.psi, a.ref, a.g, a.ph,
                       a.bd, a.tiles_x, a.tiles_y, a.items, a.item_list, a.flag, a.qacc);
}

template <int DIM, int STORE, int... I>
void launch_step_cfg(int cfg, const StepArgs &a, std::integer_sequence<int, I...>)
{
    ((cfg == I ? launch_cfg<DIM, STORE, I>(a) : void()), ...);
}

template <int DIM, int STORE, int I>
void launch_batch_cfg(const BatchArgs &b)
{
    constexpr TileCfg c = cfg_at<DIM>(I);
    if (c.psrc && b.g_psi)
        hipLaunchKernelGGL((k_psi_batch<DIM, STORE>), dim3(b.g_psi), dim3(256), 0, b.stream, b.t, b.cur);
    if (b.g_main)
        hipLaunchKernelGGL((k_main_batch<DIM, STORE, c.psrc, c.tx, c.ty, c.w, c.zc, c.keepb>), dim3(b.g_main),
                           dim3(256), 0, b.stream, b.t, b.cur);
    if (b.g_chi) hipLaunchKernelGGL(k_chi_batch, dim3(b.g_chi), dim3(64), 0, b.stream, b.t, b.cur);
    if (b.g_out)
        hipLaunchKernelGGL((k_outlet_batch<DIM, STORE>), dim3(b.g_out), dim3(FACE_NT), 0, b.stream, b.t, b.cur);
    if (b.g_inl)
        hipLaunchKernelGGL((k_inlet_batch<DIM, STORE>), dim3(b.g_inl), dim3(FACE_NT), 0, b.stream, b.t, b.cur);
    if (b.g_fill)
        hipLaunchKernelGGL((k_outlet_fill_batch<DIM, STORE>), dim3(b.g_fill), dim3(FACE_NT), 0, b.stream, b.t,
                           b.cur);
}

template <int DIM, int STORE, int... I>
void launch_batch(int cfg, const BatchArgs &b, std::integer_sequence<int, I...>)
{
    ((cfg == I ? launch_batch_cfg<DIM, STORE, I>(b) : void()), ...);
}

}  // namespace detail

// The storage mode as a compile-time constant: 0 FP32, 1 binary16 with the
// reference density, 2 binary16 with the fixed offset (see Codec).
template <typename F> void with_store(int storage, F &&f)
{
    if (storage == 0) f(std::integral_constant<int, 0>{});
    else if (storage == 1) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{});
}

#define LBM_STORE_T(sc) typename Codec<decltype(sc)::value>::T

template <int DIM>
void Launcher<DIM>::psi(int storage, const StepArgs &a)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_psi<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream, (const T *)a.src,
                           a.type, a.g, a.psi, a.ref);
    });
}

template <int DIM>
void Launcher<DIM>::moments(int storage, const StepArgs &a)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_moments<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream,
                           (const T *)a.src, a.type, (const float2 *)a.psi, a.ref, a.g, a.ph, a.orho, a.ou);
    });
}

template <int DIM>
void Launcher<DIM>::main(int storage, int cfg, const StepArgs &a)
{
    constexpr int N = detail::cfg_count<DIM>();
    with_store(storage, [&](auto sc) {
        detail::launch_step_cfg<DIM, decltype(sc)::value>(cfg, a, std::make_integer_sequence<int, N>{});
    });
}

template <int DIM>
void Launcher<DIM>::faces(int storage, const StepArgs &a, int nb_out, int nb_in)
{
    // at least one block: it records chi and the sums and clears the next ones
    const unsigned nb = (unsigned)std::max(1, nb_out + nb_in);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_faces<DIM, decltype(sc)::value>), dim3(nb), dim3(FACE_NT), 0, a.stream,
                           (const T *)a.src, (T *)a.dst, a.type, (const float2 *)a.psi, a.ref, a.g, a.ph, a.bd,
                           a.flag, a.qacc, a.qnext, nb_out, nb_in);
    });
}

template <int DIM>
void Launcher<DIM>::inlet(int storage, const StepArgs &a, unsigned nb, int nb_in)
{
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_inlet<DIM, decltype(sc)::value>), dim3(nb), dim3(FACE_NT), 0, a.stream, (T *)a.dst,
                           a.type, (const float2 *)a.psi, a.g, a.bd, nb_in);
    });
}

template <int DIM>
void Launcher<DIM>::outlet_fill(int storage, const StepArgs &a, unsigned nb)
{
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_outlet_fill<DIM, decltype(sc)::value>), dim3(nb), dim3(FACE_NT), 0, a.stream,
                           (const T *)a.src, (T *)a.dst, a.type, (const float2 *)a.psi, a.ref, a.g, a.bd);
    });
}

template <int DIM>
void Launcher<DIM>::scatter(int storage, const StepArgs &a, const double *f, float2 *ref_out)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    // writes the source array (the state f(t)) and its reference densities
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_scatter<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream, (T *)a.src,
                           a.type, a.g, a.bd, f, ref_out);
    });
}

template <int DIM>
void Launcher<DIM>::gather_state(int storage, const StepArgs &a, double *f)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_gather_state<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream,
                           (const T *)a.src, a.type, a.ref, a.g, a.bd, f);
    });
}

template <int DIM>
void Launcher<DIM>::feq_state(const double *rho0, const double *u0, int64_t N, double *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_feq_state<DIM>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rho0, u0, N, f);
}

template <int DIM>
void Launcher<DIM>::mass(int storage, const StepArgs &a, double *part, int nb, double *out)
{
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_mass<DIM, decltype(sc)::value>), dim3((unsigned)nb), dim3(256), 0, a.stream,
                           (const T *)a.src, a.type, a.ref, a.g, part);
    });
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, a.stream, (const double *)part, nb, out);
}

template <int DIM>
void Launcher<DIM>::probe(int storage, const StepArgs &a, int k, const Box3 &bx, float thr, unsigned long long *out)
{
    const int64_t vol = (int64_t)(bx.hi[0] - bx.lo[0]) * (bx.hi[1] - bx.lo[1]) * (bx.hi[2] - bx.lo[2]);
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(1), 0, a.stream, out);
    if (vol <= 0) return;
    const unsigned nb = (unsigned)((vol + 255) / 256);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_probe<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream, (const T *)a.src,
                           a.type, a.ref, a.g, k, bx, thr, out);
    });
}

template <int DIM>
void Launcher<DIM>::lab_init(int storage, const StepArgs &a, int k, const Box3 &bx, float thr, int *lab)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    with_store(storage, [&](auto sc) {
        using T = LBM_STORE_T(sc);
        hipLaunchKernelGGL((k_lab_init<DIM, decltype(sc)::value>), dim3(nb), dim3(256), 0, a.stream,
                           (const T *)a.src, a.type, a.ref, a.g, k, bx, thr, lab);
    });
}

template <int DIM>
void Launcher<DIM>::lab_prop(const StepArgs &a, int *lab, int *changed, int passes)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    for (int p = 0; p < passes; p++) hipLaunchKernelGGL(k_lab_prop, dim3(nb), dim3(256), 0, a.stream, a.g, DIM, lab, changed);
}

template <int DIM>
void Launcher<DIM>::lab_roots(const StepArgs &a, const int *lab, int *slot, int *n_roots)
{
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    hipLaunchKernelGGL(k_lab_roots, dim3(nb), dim3(256), 0, a.stream, a.g, lab, slot, n_roots);
}

template <int DIM>
void Launcher<DIM>::lab_stats(const StepArgs &a, const int *lab, const int *slot, CompStat *st, int n)
{
    if (n > 0) hipLaunchKernelGGL(k_lab_stats_init, dim3((n + 255) / 256), dim3(256), 0, a.stream, st, n);
    const unsigned nb = (unsigned)((a.g.N + 255) / 256);
    hipLaunchKernelGGL(k_lab_stats, dim3(nb), dim3(256), 0, a.stream, a.g, lab, slot, st);
}

template <int DIM>
void Launcher<DIM>::batch_step(int storage, int cfg, const BatchArgs &b)
{
    constexpr int N = detail::cfg_count<DIM>();
    with_store(storage, [&](auto sc) {
        detail::launch_batch<DIM, decltype(sc)::value>(cfg, b, std::make_integer_sequence<int, N>{});
    });
}

#undef LBM_STORE_T

}  // namespace lbm
