// surrogate.hip -- ensemble of small MLPs (4 -> H -> H -> 2, tanh) that maps
// the parameters of a channel run (capillary number, flow-rate ratio,
// viscosity ratio, width) to its droplet labels, trained on the GPU and
// queried with BF16 matrix-core inference.  Members whose predictions spread
// by more than a threshold send the query back to the lattice Boltzmann
// solver (the fallback mask).
//
// Training is full-batch Adam on the mean squared error:
//   k_fwd_bwd  one block per (64-sample tile, member): forward, backward and
//              the tile's partial gradient of every parameter (FP32, VALU)
//   k_adam     per parameter: the tile partials summed in tile order (so the
//              result does not depend on scheduling), then the Adam update
// Inference:
//   k_predict  one block per 64 queries, every member in turn: layer 1 on
//              VALU, layer 2 as 16x16x16 BF16 MFMA tiles with FP32
//              accumulation, layer 3 on VALU; ensemble mean, standard
//              deviation and the fallback flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"

namespace {

constexpr int H = 128;                       // hidden width
constexpr int NIN = 4, NOUT = 2;
constexpr int TS = 64;                       // samples per block
// parameter vector of one member
constexpr int O_W1 = 0;                      // [H][NIN]
constexpr int O_B1 = O_W1 + H * NIN;         // [H]
constexpr int O_W2 = O_B1 + H;               // [H][H], row i = output unit i
constexpr int O_B2 = O_W2 + H * H;           // [H]
constexpr int O_W3 = O_B2 + H;               // [NOUT][H]
constexpr int O_B3 = O_W3 + NOUT * H;        // [NOUT]
constexpr int P = O_B3 + NOUT;               // 17410 for H = 128

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// counter-based uniform in [-1, 1): splitmix64 of (seed, member, index)
__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t m, uint64_t i)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (m * 0x100000001B3ull + i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0f - 1.0f;
}

// weights uniform in +-1/sqrt(fan_in), biases zero; Adam moments zero
__global__ void k_init(float *__restrict__ params, float *__restrict__ am, float *__restrict__ av, int members,
                       uint64_t seed)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)members * P) return;
    const int m = (int)(t / P), p = (int)(t % P);
    float v = 0.0f;
    if (p < O_B1) v = hash_uniform(seed, m, p) * 0.5f;                      // fan-in 4
    else if (p >= O_W2 && p < O_B2) v = hash_uniform(seed, m, p) * 0.08838834764831845f;   // 1/sqrt(128)
    else if (p >= O_W3 && p < O_B3) v = hash_uniform(seed, m, p) * 0.08838834764831845f;
    params[t] = v;
    am[t] = 0.0f;
    av[t] = 0.0f;
}

// Forward and backward pass of one 64-sample tile through one member.
// loss = sum over samples and outputs of (y - Y)^2 / (n * NOUT); the tile's
// part of every gradient goes to gpart[member][tile][P], its loss to
// lpart[member][tile].
__global__ __launch_bounds__(256) void k_fwd_bwd(const float *__restrict__ params, const float *__restrict__ X,
                                                 const float *__restrict__ Y, int n, float *__restrict__ gpart,
                                                 float *__restrict__ lpart)
{
    const int tile = blockIdx.x, m = blockIdx.y, ntile = gridDim.x;
    const float *w = params + (int64_t)m * P;
    float *g = gpart + ((int64_t)m * ntile + tile) * P;
    __shared__ float s_w2t[H * H];           // W2 transposed: s_w2t[j * H + i] = W2[i][j]
    __shared__ float s_h1[TS * H];           // tanh(layer 1), then dz1
    __shared__ float s_h2[TS * H];           // tanh(layer 2), then dz2
    __shared__ float s_x[TS * NIN];
    __shared__ float s_dy[TS * NOUT];
    __shared__ float s_red[256];
    const int tid = threadIdx.x;
    const int s0 = tile * TS;
    const int ns = min(TS, n - s0);          // valid samples of this tile

    for (int e = tid; e < H * H; e += 256) {
        const int i = e / H, j = e % H;
        s_w2t[j * H + i] = w[O_W2 + e];
    }
    for (int e = tid; e < TS * NIN; e += 256) s_x[e] = e / NIN < ns ? X[(int64_t)s0 * NIN + e] : 0.0f;
    __syncthreads();

    // layer 1: h1[s][i] = tanh(b1[i] + sum_c W1[i][c] x[s][c])
    for (int e = tid; e < TS * H; e += 256) {
        const int s = e / H, i = e % H;
        float a = w[O_B1 + i];
        for (int c = 0; c < NIN; c++) a = fmaf(w[O_W1 + i * NIN + c], s_x[s * NIN + c], a);
        s_h1[e] = tanhf(a);
    }
    __syncthreads();

    // layer 2: thread owns unit i and samples sb, sb + 2, ...
    const int i = tid % H, sb = tid / H;
    {
        float acc[TS / 2];
        for (int k = 0; k < TS / 2; k++) acc[k] = w[O_B2 + i];
        for (int j = 0; j < H; j++) {
            const float wij = s_w2t[j * H + i];
#pragma unroll
            for (int k = 0; k < TS / 2; k++) acc[k] = fmaf(s_h1[(sb + 2 * k) * H + j], wij, acc[k]);
        }
#pragma unroll
        for (int k = 0; k < TS / 2; k++) s_h2[(sb + 2 * k) * H + i] = tanhf(acc[k]);
    }
    __syncthreads();

    // layer 3 and the loss: one thread per (sample, output)
    float lsum = 0.0f;
    if (tid < TS * NOUT) {
        const int s = tid / NOUT, o = tid % NOUT;
        float y = w[O_B3 + o];
        for (int j = 0; j < H; j++) y = fmaf(w[O_W3 + o * H + j], s_h2[s * H + j], y);
        float d = 0.0f;
        if (s < ns) {
            const float r = y - Y[(int64_t)(s0 + s) * NOUT + o];
            lsum = r * r / (float)(n * NOUT);
            d = 2.0f * r / (float)(n * NOUT);
        }
        s_dy[tid] = d;
    }
    s_red[tid] = lsum;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) s_red[tid] += s_red[tid + st];
        __syncthreads();
    }
    if (tid == 0) lpart[(int64_t)m * ntile + tile] = s_red[0];

    // layer 3 gradients: dW3[o][j] = sum_s dy[s][o] h2[s][j]; db3[o] = sum_s dy[s][o]
    for (int e = tid; e < NOUT * H; e += 256) {
        const int o = e / H, j = e % H;
        float a = 0.0f;
        for (int s = 0; s < TS; s++) a = fmaf(s_dy[s * NOUT + o], s_h2[s * H + j], a);
        g[O_W3 + e] = a;
    }
    if (tid < NOUT) {
        float a = 0.0f;
        for (int s = 0; s < TS; s++) a += s_dy[s * NOUT + tid];
        g[O_B3 + tid] = a;
    }
    __syncthreads();
    // dz2[s][i] = (sum_o dy[s][o] W3[o][i]) (1 - h2^2), in place of h2
    for (int e = tid; e < TS * H; e += 256) {
        const int s = e / H, u = e % H;
        float d = 0.0f;
        for (int o = 0; o < NOUT; o++) d = fmaf(s_dy[s * NOUT + o], w[O_W3 + o * H + u], d);
        const float h = s_h2[e];
        s_h2[e] = d * (1.0f - h * h);
    }
    __syncthreads();
    // dW2[i][j] = sum_s dz2[s][i] h1[s][j]: thread owns unit i and 64 of the j
    {
        const int jb = (tid / H) * (H / 2);
        float acc[H / 2];
        for (int k = 0; k < H / 2; k++) acc[k] = 0.0f;
        float db = 0.0f;
        for (int s = 0; s < TS; s++) {
            const float dz = s_h2[s * H + i];
            db += dz;
#pragma unroll
            for (int k = 0; k < H / 2; k++) acc[k] = fmaf(dz, s_h1[s * H + jb + k], acc[k]);
        }
        for (int k = 0; k < H / 2; k++) g[O_W2 + i * H + jb + k] = acc[k];
        if (jb == 0) g[O_B2 + i] = db;
    }
    __syncthreads();
    // dz1[s][j] = (sum_i dz2[s][i] W2[i][j]) (1 - h1^2): thread owns j and samples sb, sb + 2, ...
    {
        const int j = tid % H;
        float acc[TS / 2];
        for (int k = 0; k < TS / 2; k++) acc[k] = 0.0f;
        for (int u = 0; u < H; u++) {
            const float wuj = w[O_W2 + u * H + j];
#pragma unroll
            for (int k = 0; k < TS / 2; k++) acc[k] = fmaf(s_h2[(sb + 2 * k) * H + u], wuj, acc[k]);
        }
        __syncthreads();                     // every read of h1 by the dW2 pass is done
#pragma unroll
        for (int k = 0; k < TS / 2; k++) {
            const float h = s_h1[(sb + 2 * k) * H + j];
            s_h1[(sb + 2 * k) * H + j] = acc[k] * (1.0f - h * h);
        }
    }
    __syncthreads();
    // dW1[j][c] = sum_s dz1[s][j] x[s][c]; db1[j] = sum_s dz1[s][j]
    for (int e = tid; e < H * (NIN + 1); e += 256) {
        const int j = e / (NIN + 1), c = e % (NIN + 1);
        float a = 0.0f;
        for (int s = 0; s < TS; s++) a = fmaf(s_h1[s * H + j], c < NIN ? s_x[s * NIN + c] : 1.0f, a);
        if (c < NIN) g[O_W1 + j * NIN + c] = a;
        else g[O_B1 + j] = a;
    }
}

// gradient = tile partials summed in tile order; optional copy out; Adam step
__global__ void k_adam(float *__restrict__ params, float *__restrict__ am, float *__restrict__ av,
                       const float *__restrict__ gpart, int members, int ntile, float lr, float b1, float b2,
                       float eps, float c1, float c2, int update, float *__restrict__ gout)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)members * P) return;
    const int m = (int)(t / P), p = (int)(t % P);
    float gsum = 0.0f;
    for (int k = 0; k < ntile; k++) gsum += gpart[((int64_t)m * ntile + k) * P + p];
    if (gout) gout[t] = gsum;
    if (!update) return;
    const float mm = b1 * am[t] + (1.0f - b1) * gsum;
    const float vv = b2 * av[t] + (1.0f - b2) * gsum * gsum;
    am[t] = mm;
    av[t] = vv;
    params[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// loss per member: tile partials in tile order
__global__ void k_loss(const float *__restrict__ lpart, int members, int ntile, float *__restrict__ out)
{
    const int m = threadIdx.x;
    if (m >= members) return;
    float a = 0.0f;
    for (int k = 0; k < ntile; k++) a += lpart[m * ntile + k];
    out[m] = a;
}

// W2 of every member as BF16 (round to nearest even) for inference
__global__ void k_w2_bf16(const float *__restrict__ params, int members, uint16_t *__restrict__ w2)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)members * H * H) return;
    const int m = (int)(t / (H * H)), e = (int)(t % (H * H));
    w2[t] = to_bf16(params[(int64_t)m * P + O_W2 + e]);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One block of 256 threads (4 waves) answers 64 queries with every member.
__global__ __launch_bounds__(256) void k_predict(const float *__restrict__ params, const uint16_t *__restrict__ w2,
                                                 int members, const float *__restrict__ X, int n,
                                                 float *__restrict__ mean, float *__restrict__ sd,
                                                 uint8_t *__restrict__ fallback, float thresh, float2 oscale,
                                                 float2 oshift)
{
    __shared__ uint16_t s_h1[TS * H];        // layer-1 activations, BF16
    __shared__ float s_h2[TS * H];           // layer-2 activations
    __shared__ float s_y[TS * NOUT];
    __shared__ float s_sum[TS * NOUT], s_sq[TS * NOUT];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int s0 = blockIdx.x * TS;
    const int ns = min(TS, n - s0);
    if (tid < TS * NOUT) {
        s_sum[tid] = 0.0f;
        s_sq[tid] = 0.0f;
    }
    for (int m = 0; m < members; m++) {
        const float *w = params + (int64_t)m * P;
        const uint16_t *w2m = w2 + (int64_t)m * H * H;
        __syncthreads();
        for (int e = tid; e < TS * H; e += 256) {
            const int s = e / H, i = e % H;
            float a = w[O_B1 + i];
            if (s < ns)
                for (int c = 0; c < NIN; c++) a = fmaf(w[O_W1 + i * NIN + c], X[(int64_t)(s0 + s) * NIN + c], a);
            s_h1[e] = to_bf16(tanhf(a));
        }
        __syncthreads();
        // z2 = h1 W2^T: wave w owns sample rows 16w .. 16w + 15 and all 8
        // column tiles.  16x16x16 operands: lane l holds row (A) / column (B)
        // l % 16 and k = 4 (l / 16) .. +3 of the 16-wide k chunk; the result
        // holds column l % 16 and rows 4 (l / 16) .. +3.
        const int r = lane % 16, kq = 4 * (lane / 16);
        for (int ct = 0; ct < H / 16; ct++) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kc = 0; kc < H; kc += 16) {
                bf16x4 a, b;
                const uint16_t *pa = s_h1 + (16 * wave + r) * H + kc + kq;
                const uint16_t *pb = w2m + (int64_t)(16 * ct + r) * H + kc + kq;
                for (int q = 0; q < 4; q++) {
                    a[q] = (short)pa[q];
                    b[q] = (short)pb[q];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
            }
            const int col = 16 * ct + r;
            for (int q = 0; q < 4; q++) {
                const int row = 16 * wave + kq + q;
                s_h2[row * H + col] = tanhf(acc[q] + w[O_B2 + col]);
            }
        }
        __syncthreads();
        if (tid < TS * NOUT) {
            const int s = tid / NOUT, o = tid % NOUT;
            float y = w[O_B3 + o];
            for (int j = 0; j < H; j++) y = fmaf(w[O_W3 + o * H + j], s_h2[s * H + j], y);
            // the caller's units (the statistics and the fallback test use them)
            y = o == 0 ? fmaf(y, oscale.x, oshift.x) : fmaf(y, oscale.y, oshift.y);
            s_sum[tid] += y;
            s_sq[tid] += y * y;
        }
    }
    __syncthreads();
    if (tid < TS * NOUT) {
        const int s = tid / NOUT;
        const float mu = s_sum[tid] / (float)members;
        const float var = fmaxf(s_sq[tid] / (float)members - mu * mu, 0.0f);
        s_y[tid] = mu;
        if (s < ns) {
            mean[(int64_t)s0 * NOUT + tid] = mu;
            sd[(int64_t)s0 * NOUT + tid] = sqrtf(var);
        }
        s_sum[tid] = sqrtf(var) > thresh * fabsf(mu) ? 1.0f : 0.0f;
    }
    __syncthreads();
    if (tid < TS && tid < ns) {
        bool fb = false;
        for (int o = 0; o < NOUT; o++) fb = fb || s_sum[tid * NOUT + o] != 0.0f;
        fallback[s0 + tid] = fb ? 1 : 0;
    }
}

}  // namespace

struct surr_ctx {
    int members = 0, max_n = 0, ntile_max = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    float *params = nullptr, *am = nullptr, *av = nullptr, *gpart = nullptr, *lpart = nullptr, *loss = nullptr;
    uint16_t *w2 = nullptr;
    int64_t adam_t = 0;
    bool w2_fresh = false;
    std::string err;
};

namespace {

thread_local std::string g_surr_error;

constexpr size_t SALIGN = 256;
size_t salign(size_t v) { return (v + SALIGN - 1) / SALIGN * SALIGN; }

struct SLayout {
    size_t params, am, av, gpart, lpart, loss, w2, total;
};

SLayout surr_layout(int members, int max_n)
{
    const int nt = (max_n + TS - 1) / TS;
    SLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t at = o; o += salign(std::max<size_t>(b, 1)); return at; };
    L.params = take((size_t)members * P * 4);
    L.am = take((size_t)members * P * 4);
    L.av = take((size_t)members * P * 4);
    L.gpart = take((size_t)members * nt * P * 4);
    L.lpart = take((size_t)members * nt * 4);
    L.loss = take((size_t)members * 4);
    L.w2 = take((size_t)members * H * H * 2);
    L.total = o;
    return L;
}

lbm_status sfail(surr_ctx *c, lbm_status st, const std::string &msg)
{
    if (c) c->err = msg;
    else g_surr_error = msg;
    return st;
}

#define SHIPCHECK(c, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return sfail(c, LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

bool args_ok(int members, int hidden, int max_n)
{
    return members >= 1 && members <= 64 && hidden == H && max_n >= 1 && max_n <= (1 << 22);
}

// forward + backward over n samples; gradients summed (and copied to gout if
// given), Adam step if update
lbm_status pass(surr_ctx *c, const float *X, const float *Y, int n, float lr, bool update, float *gout)
{
    const int nt = (n + TS - 1) / TS;
    hipLaunchKernelGGL(k_fwd_bwd, dim3(nt, c->members), dim3(256), 0, c->stream, c->params, X, Y, n, c->gpart,
                       c->lpart);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    if (update) c->adam_t++;
    const float c1 = update ? 1.0f - std::pow(b1, (float)c->adam_t) : 1.0f;
    const float c2 = update ? 1.0f - std::pow(b2, (float)c->adam_t) : 1.0f;
    const int64_t np = (int64_t)c->members * P;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, c->stream, c->params, c->am, c->av,
                       c->gpart, c->members, nt, lr, b1, b2, eps, c1, c2, update ? 1 : 0, gout);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, c->stream, c->lpart, c->members, nt, c->loss);
    if (update) c->w2_fresh = false;
    SHIPCHECK(c, hipGetLastError());
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t surr_workspace_bytes(int members, int hidden, int max_n)
{
    if (!args_ok(members, hidden, max_n)) return 0;
    return surr_layout(members, max_n).total;
}

int surr_param_count(int hidden) { return hidden == H ? P : 0; }

lbm_status surr_create(int members, int hidden, int max_n, uint64_t seed, void *dev_ws, size_t ws_bytes,
                       void *hip_stream, surr_ctx **out)
{
    if (!out) return sfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!args_ok(members, hidden, max_n))
        return sfail(nullptr, LBM_EINVAL, "members must be 1..64, hidden 128, max_n 1..4194304");
    const SLayout L = surr_layout(members, max_n);
    if (!dev_ws || ((uintptr_t)dev_ws) % SALIGN) return sfail(nullptr, LBM_EINVAL, "workspace NULL or misaligned");
    if (ws_bytes < L.total) return sfail(nullptr, LBM_ENOMEM, "workspace too small");
    surr_ctx *c = new surr_ctx();
    c->members = members;
    c->max_n = max_n;
    c->ntile_max = (max_n + TS - 1) / TS;
    c->ws = (char *)dev_ws;
    c->stream = (hipStream_t)hip_stream;
    c->params = (float *)(c->ws + L.params);
    c->am = (float *)(c->ws + L.am);
    c->av = (float *)(c->ws + L.av);
    c->gpart = (float *)(c->ws + L.gpart);
    c->lpart = (float *)(c->ws + L.lpart);
    c->loss = (float *)(c->ws + L.loss);
    c->w2 = (uint16_t *)(c->ws + L.w2);
    const int64_t np = (int64_t)members * P;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, c->stream, c->params, c->am, c->av,
                       members, seed);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        delete c;
        return sfail(nullptr, LBM_EDEVICE, "initialisation failed");
    }
    *out = c;
    return LBM_OK;
}

lbm_status surr_train(surr_ctx *c, const float *X, const float *Y, int n, int epochs, float lr, float *loss_host)
{
    if (!c || !X || !Y || n < 1 || n > c->max_n || epochs < 0 || !(lr > 0.0f))
        return sfail(c, LBM_EINVAL, "bad arguments to surr_train");
    for (int e = 0; e < epochs; e++) {
        const lbm_status st = pass(c, X, Y, n, lr, true, nullptr);
        if (st != LBM_OK) return st;
    }
    if (loss_host) {
        SHIPCHECK(c, hipMemcpyAsync(loss_host, c->loss, (size_t)c->members * 4, hipMemcpyDeviceToHost, c->stream));
        SHIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

lbm_status surr_forward_backward(surr_ctx *c, const float *X, const float *Y, int n, float *grads, float *loss)
{
    if (!c || !X || !Y || !grads || n < 1 || n > c->max_n)
        return sfail(c, LBM_EINVAL, "bad arguments to surr_forward_backward");
    const lbm_status st = pass(c, X, Y, n, 0.0f, false, grads);
    if (st != LBM_OK) return st;
    if (loss) SHIPCHECK(c, hipMemcpyAsync(loss, c->loss, (size_t)c->members * 4, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

lbm_status surr_predict(surr_ctx *c, const float *X, int n, float *mean, float *sd, uint8_t *fallback, float thresh,
                        const float *out_scale, const float *out_shift)
{
    if (!c || !X || !mean || !sd || !fallback || n < 1 || !(thresh >= 0.0f))
        return sfail(c, LBM_EINVAL, "bad arguments to surr_predict");
    const float2 osc = out_scale ? make_float2(out_scale[0], out_scale[1]) : make_float2(1.0f, 1.0f);
    const float2 osh = out_shift ? make_float2(out_shift[0], out_shift[1]) : make_float2(0.0f, 0.0f);
    if (!std::isfinite(osc.x) || !std::isfinite(osc.y) || !std::isfinite(osh.x) || !std::isfinite(osh.y))
        return sfail(c, LBM_EINVAL, "non-finite output scale or shift");
    if (!c->w2_fresh) {
        const int64_t ne = (int64_t)c->members * H * H;
        hipLaunchKernelGGL(k_w2_bf16, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, c->stream, c->params,
                           c->members, c->w2);
        c->w2_fresh = true;
    }
    hipLaunchKernelGGL(k_predict, dim3((unsigned)((n + TS - 1) / TS)), dim3(256), 0, c->stream, c->params, c->w2,
                       c->members, X, n, mean, sd, fallback, thresh, osc, osh);
    SHIPCHECK(c, hipGetLastError());
    return LBM_OK;
}

lbm_status surr_get_params(surr_ctx *c, float *host, size_t bytes)
{
    if (!c || !host || bytes != (size_t)c->members * P * 4) return sfail(c, LBM_EINVAL, "bad arguments to surr_get_params");
    SHIPCHECK(c, hipMemcpyAsync(host, c->params, bytes, hipMemcpyDeviceToHost, c->stream));
    SHIPCHECK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status surr_set_params(surr_ctx *c, const float *host, size_t bytes)
{
    if (!c || !host || bytes != (size_t)c->members * P * 4) return sfail(c, LBM_EINVAL, "bad arguments to surr_set_params");
    SHIPCHECK(c, hipMemcpyAsync(c->params, host, bytes, hipMemcpyHostToDevice, c->stream));
    SHIPCHECK(c, hipStreamSynchronize(c->stream));
    c->w2_fresh = false;
    return LBM_OK;
}

void surr_destroy(surr_ctx *c) { delete c; }

const char *surr_last_error(const surr_ctx *c) { return c ? c->err.c_str() : g_surr_error.c_str(); }

}  // extern "C"
