// probe.hip -- plain streaming kernels that measure the HBM rate a kernel of
// a given access width can reach on this device: the practical ceiling next
// to the published peak for the rooflines of the step kernels.
#include <hip/hip_runtime.h>

#include "../../include/lbm_probe.h"
#include "lattice.h"

namespace {

// one 4-byte element per thread
__global__ __launch_bounds__(256) void k_copy_b32(const uint32_t *__restrict__ a, uint32_t *__restrict__ b,
                                                  size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// eight 4-byte elements per thread, each load coalesced over the block
__global__ __launch_bounds__(256) void k_copy_b32x8(const uint32_t *__restrict__ a, uint32_t *__restrict__ b,
                                                    size_t n)
{
    const size_t i0 = (size_t)blockIdx.x * 2048 + threadIdx.x;
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = i0 + 256 * k < n ? a[i0 + 256 * k] : 0u;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (i0 + 256 * k < n) b[i0 + 256 * k] = v[k];
}

// one 16-byte element per thread
__global__ __launch_bounds__(256) void k_copy_b128(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// reads one 16-byte element per thread; the sum is stored only in the
// impossible case that it equals a NaN payload, which keeps the loads
__global__ __launch_bounds__(256) void k_read_b128(const uint4 *__restrict__ a, uint32_t *__restrict__ out,
                                                   size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const uint4 v = a[i];
        const uint32_t s = v.x ^ v.y ^ v.z ^ v.w;
        if (s == 0x7fc0dead) out[0] = s;
    }
}

// The access pattern of the 3-D node update without its arithmetic: each
// node loads the 19 populations of two components from its neighbours'
// slots (38 planes of M nodes, the slot of direction i shifted by -e_i in a
// 128 x 128 x nz box) and stores 38 values at its own slots, non-temporal
// like the FP32 node update.  A thread takes PULL_NZ nodes along the slowest
// axis; nodes lie in planes [2, nz - 2) with nz - 4 a multiple of PULL_NZ,
// so every shifted slot is inside its plane.  PIPE = 0 issues a node's loads
// after the previous node's stores (the order of the node update); PIPE = 1
// issues them before those stores (two register sets in turn, no copies).
constexpr int PULL_PX = 128, PULL_PY = 128, PULL_NZ = 16;

template <int PIPE>
__global__ __launch_bounds__(256) void k_pull_d3q19(const void *src, void *dst, uint32_t bytes, uint32_t M)
{
    constexpr int Q = lbm::Lat<3>::Q;
    constexpr int flags = 0x00020000;   // dword 3 of a raw gfx9 buffer descriptor
    const __amdgpu_buffer_rsrc_t a = __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)bytes, flags);
    const __amdgpu_buffer_rsrc_t b = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)bytes, flags);
    const uint32_t xy = blockIdx.x * 256 + threadIdx.x;
    const int z0 = 2 + (int)blockIdx.y * PULL_NZ;
    auto load = [&](int z, uint32_t (&v)[2 * Q]) {
        const uint32_t j = xy + (uint32_t)z * PULL_PX * PULL_PY;
        lbm::static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int off = lbm::Lat<3>::E[i][0] + PULL_PX * (lbm::Lat<3>::E[i][1] + PULL_PY * lbm::Lat<3>::E[i][2]);
            v[i] = __builtin_amdgcn_raw_buffer_load_b32(a, (int)((j - off) * 4u), (int)(i * M * 4u), 0);
            v[Q + i] = __builtin_amdgcn_raw_buffer_load_b32(a, (int)((j - off) * 4u), (int)((Q + i) * M * 4u), 0);
        });
    };
    auto store = [&](int z, const uint32_t (&v)[2 * Q]) {
        const uint32_t j = xy + (uint32_t)z * PULL_PX * PULL_PY;
        lbm::static_for<2 * Q>([&](auto ic) {
            constexpr int c = decltype(ic)::value;
            __builtin_amdgcn_raw_buffer_store_b32(v[c], b, (int)(j * 4u), (int)(c * M * 4u), 2);
        });
    };
    if constexpr (PIPE == 0) {
#pragma unroll 1
        for (int z = z0; z < z0 + PULL_NZ; z++) {
            uint32_t v[2 * Q];
            load(z, v);
            store(z, v);
        }
    } else {
        uint32_t A[2 * Q], B[2 * Q];
        load(z0, A);
#pragma unroll 1
        for (int z = z0; z < z0 + PULL_NZ - 2; z += 2) {
            load(z + 1, B);
            store(z, A);
            load(z + 2, A);
            store(z + 1, B);
        }
        load(z0 + PULL_NZ - 1, B);
        store(z0 + PULL_NZ - 2, A);
        store(z0 + PULL_NZ - 1, B);
    }
}

// The same pattern with both components of a population side by side in one
// 8-byte slot: 19 loads and 19 stores of 8 bytes per node (the same bytes,
// half the memory instructions), a node's loads after the previous node's
// stores.
__global__ __launch_bounds__(256) void k_pull_d3q19_pairs(const void *src, void *dst, uint32_t bytes, uint32_t M)
{
    constexpr int Q = lbm::Lat<3>::Q;
    constexpr int flags = 0x00020000;   // dword 3 of a raw gfx9 buffer descriptor
    const __amdgpu_buffer_rsrc_t a = __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)bytes, flags);
    const __amdgpu_buffer_rsrc_t b = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)bytes, flags);
    const uint32_t xy = blockIdx.x * 256 + threadIdx.x;
    const int z0 = 2 + (int)blockIdx.y * PULL_NZ;
#pragma unroll 1
    for (int z = z0; z < z0 + PULL_NZ; z++) {
        const uint32_t j = xy + (uint32_t)z * PULL_PX * PULL_PY;
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        u32x2 v[Q];
        lbm::static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int off = lbm::Lat<3>::E[i][0] + PULL_PX * (lbm::Lat<3>::E[i][1] + PULL_PY * lbm::Lat<3>::E[i][2]);
            v[i] = __builtin_amdgcn_raw_buffer_load_b64(a, (int)((j - off) * 8u), (int)(i * M * 8u), 0);
        });
        lbm::static_for<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            __builtin_amdgcn_raw_buffer_store_b64(v[i], b, (int)(j * 8u), (int)(i * M * 8u), 2);
        });
    }
}

}  // namespace

extern "C" lbm_status lbm_stream_probe(const void *src, void *dst, size_t bytes, int kind, int reps,
                                       void *hip_stream, double *gbs)
{
    if (!src || !dst || !gbs || bytes < 16 || bytes % 16 || kind < 0 || kind > 6 || reps < 1) return LBM_EINVAL;
    if (kind >= 4 && bytes > 0x7fffffffu) return LBM_EINVAL;   // 32-bit buffer offsets
    const size_t n = (kind == 0 || kind == 3) ? bytes / 4 : bytes / 16;
    const size_t per_block = kind == 3 ? 2048 : 256;
    if ((n + per_block - 1) / per_block > 0x7fffffffu) return LBM_EINVAL;
    dim3 grid((unsigned)((n + per_block - 1) / per_block));
    // pull pattern: 38 planes of M = 128 * 128 * nz nodes within the buffers,
    // nz - 4 a multiple of the planes per thread
    const int nz_fit = (int)(bytes / (38ull * 4 * PULL_PX * PULL_PY));
    const int pull_nz = 4 + (nz_fit - 4) / PULL_NZ * PULL_NZ;
    const uint32_t pull_M = (uint32_t)pull_nz * PULL_PX * PULL_PY;
    double moved_per_launch = 0.0;
    if (kind >= 4) {
        if (nz_fit < 4 + PULL_NZ) return LBM_EINVAL;
        grid = dim3(PULL_PX * PULL_PY / 256, (unsigned)((pull_nz - 4) / PULL_NZ));
        moved_per_launch = 2.0 * 38.0 * 4.0 * (double)PULL_PX * PULL_PY * (pull_nz - 4);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBM_EDEVICE;
    auto launch = [&]() {
        if (kind == 0) hipLaunchKernelGGL(k_copy_b32, grid, dim3(256), 0, s, (const uint32_t *)src, (uint32_t *)dst, n);
        else if (kind == 1) hipLaunchKernelGGL(k_copy_b128, grid, dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n);
        else if (kind == 2) hipLaunchKernelGGL(k_read_b128, grid, dim3(256), 0, s, (const uint4 *)src, (uint32_t *)dst, n);
        else if (kind == 3) hipLaunchKernelGGL(k_copy_b32x8, grid, dim3(256), 0, s, (const uint32_t *)src, (uint32_t *)dst, n);
        else if (kind == 4) hipLaunchKernelGGL(k_pull_d3q19<0>, grid, dim3(256), 0, s, src, dst, (uint32_t)bytes, pull_M);
        else if (kind == 5) hipLaunchKernelGGL(k_pull_d3q19<1>, grid, dim3(256), 0, s, src, dst, (uint32_t)bytes, pull_M);
        else hipLaunchKernelGGL(k_pull_d3q19_pairs, grid, dim3(256), 0, s, src, dst, (uint32_t)bytes, pull_M);
    };
    launch();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++) launch();
    (void)hipEventRecord(e1, s);
    float ms = 0.0f;
    const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                    hipGetLastError() == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || ms <= 0.0f) return LBM_EDEVICE;
    const double moved = kind >= 4 ? moved_per_launch * reps : (kind == 2 ? 1.0 : 2.0) * (double)bytes * reps;
    *gbs = moved / (ms * 1e-3) / 1e9;
    return LBM_OK;
}
