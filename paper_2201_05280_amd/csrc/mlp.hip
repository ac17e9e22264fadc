// mlp.hip -- coordinate MLP of the learned warm start: 6 inputs -> 4 hidden
// layers of 128 (SiLU) -> 4 outputs, BF16 weights and activations with FP32
// accumulation, FP32 master weights and Adam.
//
// The three 128x128 layers run on the matrix cores: a 64x64 work-group tile
// of C = A B is built from 16x16x16 bf16 MFMA blocks (four waves, each a 16x64
// slab).  The same tile routine gives the forward products, the data
// gradients dA = dZ W and the split-K weight gradients dW = dZ^T A.  The
// 6-wide first layer and the 4-wide last layer are small and run on the
// vector ALUs.  Parameter order: W1[128][6], b1, W2[128][128], b2, W3, b3,
// W4, b4, W5[4][128], b5.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pgk.h"

namespace pgk_mlp_dev {

constexpr int H = 128, NIN = 6, NOUT = 4;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * NIN;
constexpr int OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * H;
constexpr int OFF_W4 = OFF_B3 + H, OFF_B4 = OFF_W4 + H * H;
constexpr int OFF_W5 = OFF_B4 + H, OFF_B5 = OFF_W5 + NOUT * H;
constexpr int NPARAM = OFF_B5 + NOUT;
static_assert(NPARAM == PGK_MLP_NPARAM, "parameter count");

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even
__host__ __device__ inline uint16_t f2bf(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ inline float dsilu(float z)
{
    float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

template <typename T> __device__ inline short as_bf(T v);
template <> __device__ inline short as_bf<uint16_t>(uint16_t v) { return (short)v; }
template <> __device__ inline short as_bf<float>(float v) { return (short)f2bf(v); }

enum { EPI_FWD = 0, EPI_BWD = 1, EPI_WGRAD = 2 };

// C[m][n] = sum_k A(m,k) B(k,n), A(m,k) = A[m*am + k*ak], B(k,n) = B[k*bk + n*bn].
// Work-group tile 64x64 (M0 = 64*blockIdx.x, N0 = 64*blockIdx.y), K range
// [kb, ke) (split K over blockIdx.z for the weight gradient).  Epilogues:
//   EPI_FWD   z = C + bias[n] -> zout[m][n] (fp32), silu(z) -> aout[m][n] (bf16)
//   EPI_BWD   dz = C * dsilu(zin[m][n]) -> zout[m][n] (fp32)
//   EPI_WGRAD atomicAdd(C) into zout[m][n] (fp32)
// four consecutive bf16 values (8-byte aligned) as one MFMA operand
__device__ inline v4i16 load4_bf(const uint16_t *p)
{
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    v4i16 r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

// CONTIG: A and B are contiguous along k (ak = bk = 1, A in bf16): operands
// come in 8-byte loads
template <typename TA, int EPI, bool CONTIG = false>
__global__ __launch_bounds__(256) void k_gemm(const TA *__restrict__ A, int am, int ak,
                                              const uint16_t *__restrict__ B, int bk, int bn, int K, int kchunk,
                                              const float *__restrict__ bias, const float *__restrict__ zin,
                                              float *__restrict__ zout, uint16_t *__restrict__ aout, int ldc,
                                              int mvalid)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + wave * 16, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4f32 acc[4];
    for (int b = 0; b < 4; b++) acc[b] = v4f32{0.f, 0.f, 0.f, 0.f};
    // K in blocks of four 16-deep MFMA steps: all loads of a block are issued
    // before its products, so their latencies overlap
    constexpr int KB = 4;
    for (int k1 = kb; k1 < ke; k1 += 16 * KB) {
        v4i16 a[KB], bb[KB][4];
#pragma unroll
        for (int s = 0; s < KB; s++) {
            const int k0 = k1 + 16 * s;
            const bool in = k0 < ke;
            if constexpr (CONTIG) {
                const uint16_t *Ab = reinterpret_cast<const uint16_t *>(A);
                a[s] = in ? load4_bf(Ab + (size_t)(m0 + r) * am + k0 + kq) : v4i16{0, 0, 0, 0};
#pragma unroll
                for (int b = 0; b < 4; b++)
                    bb[s][b] = in ? load4_bf(B + (size_t)(n0 + 16 * b + r) * bn + k0 + kq) : v4i16{0, 0, 0, 0};
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++)
                    a[s][j] = in ? as_bf<TA>(A[(size_t)(m0 + r) * am + (size_t)(k0 + kq + j) * ak]) : 0;
#pragma unroll
                for (int b = 0; b < 4; b++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        bb[s][b][j] = in ? (short)B[(size_t)(k0 + kq + j) * bk + (size_t)(n0 + 16 * b + r) * bn] : 0;
            }
        }
#pragma unroll
        for (int s = 0; s < KB; s++)
#pragma unroll
            for (int b = 0; b < 4; b++) acc[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[s], bb[s][b], acc[b], 0, 0, 0);
    }
    // lane holds C[m0 + 4*(lane/16) + j][n0 + 16 b + lane%16]
    for (int b = 0; b < 4; b++)
        for (int j = 0; j < 4; j++) {
            int m = m0 + kq + j, n = n0 + 16 * b + r;
            float c = acc[b][j];
            if (EPI == EPI_WGRAD) {
                atomicAdd(&zout[(size_t)m * ldc + n], c);
            } else if (m < mvalid) {
                if (EPI == EPI_FWD) {
                    float z = c + bias[n];
                    zout[(size_t)m * ldc + n] = z;
                    aout[(size_t)m * ldc + n] = f2bf(silu(z));
                } else {
                    zout[(size_t)m * ldc + n] = c * dsilu(zin[(size_t)m * ldc + n]);
                }
            }
        }
}

// first layer: z1 = W1 x + b1 (x not rounded, W1 in bf16); thread per (point, unit)
__global__ void k_layer1(const float *__restrict__ X, int n, int npad, const uint16_t *__restrict__ wbf,
                         const float *__restrict__ master, float *__restrict__ z1, uint16_t *__restrict__ a1)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad * H) return;
    int p = i / H, o = i - p * H;
    float z = master[OFF_B1 + o];
    for (int k = 0; k < NIN; k++) z += bf2f(wbf[OFF_W1 + o * NIN + k]) * (p < n ? X[p * NIN + k] : 0.f);
    z1[i] = z;
    a1[i] = f2bf(silu(z));
}

// last layer: y = W5 a4 + b5; thread per (point, output)
__global__ void k_layer5(const uint16_t *__restrict__ a4, int n, const uint16_t *__restrict__ wbf,
                         const float *__restrict__ master, float *__restrict__ Y)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * NOUT) return;
    int p = i / NOUT, o = i - p * NOUT;
    float y = master[OFF_B5 + o];
    for (int k = 0; k < H; k++) y += bf2f(wbf[OFF_W5 + o * H + k]) * bf2f(a4[p * H + k]);
    Y[i] = y;
}

// dy = 2 (yhat - y)/(4 N) (zero on padding rows) and the loss sum
// dy = 2 (yhat - Y) scale (gradient of the minibatch's mean loss); the
// squared errors are summed into *loss with weight lscale
__global__ void k_loss(const float *__restrict__ yhat, const float *__restrict__ Y, int n, int npad, float scale,
                       float lscale, float *__restrict__ dy, float *__restrict__ loss)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < npad * NOUT) {
        int p = i / NOUT;
        float d = p < n ? yhat[i] - Y[i] : 0.f;
        dy[i] = 2.f * d * scale;
        l = d * d * lscale;
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// dz4 = (dy W5) * dsilu(z4)
__global__ void k_layer5_bwd(const float *__restrict__ dy, const float *__restrict__ z4,
                             const uint16_t *__restrict__ wbf, int npad, float *__restrict__ dz4)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad * H) {
        int p = i / H, k = i - p * H;
        float da = 0.f;
        for (int o = 0; o < NOUT; o++) da += dy[p * NOUT + o] * bf2f(wbf[OFF_W5 + o * H + k]);
        dz4[i] = da * dsilu(z4[i]);
    }
}

// Reductions over the points of a minibatch: work-group b takes points
// [b GP, (b + 1) GP), thread k one hidden unit, and adds its partial sums to
// the gradient (one atomic per value and work-group).
constexpr int GP = 32;

// last layer: dW5[o][k] = sum_p dy[p][o] a4[p][k], db5[o] = sum_p dy[p][o]
__global__ __launch_bounds__(H) void k_layer5_wgrad(const float *__restrict__ dy, const uint16_t *__restrict__ a4,
                                                    int n, float *__restrict__ grad)
{
    const int k = threadIdx.x, p0 = blockIdx.x * GP, p1 = min(n, p0 + GP);
    float g[NOUT] = {0.f, 0.f, 0.f, 0.f}, gb = 0.f;
    for (int p = p0; p < p1; p++) {
        float a = bf2f(a4[(size_t)p * H + k]);
#pragma unroll
        for (int o = 0; o < NOUT; o++) g[o] += dy[p * NOUT + o] * a;
        if (k < NOUT) gb += dy[p * NOUT + k];
    }
#pragma unroll
    for (int o = 0; o < NOUT; o++) atomicAdd(&grad[OFF_W5 + o * H + k], g[o]);
    if (k < NOUT) atomicAdd(&grad[OFF_B5 + k], gb);
}

// bias gradient: column sums of dz[npad][H] (padding rows are zero)
__global__ void k_bias_grad(const float *__restrict__ dz, int npad, float *__restrict__ gb)
{
    int o = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int p = t; p < npad; p += blockDim.x) s += dz[p * H + o];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ float red[4];
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) atomicAdd(&gb[o], red[0] + red[1] + red[2] + red[3]);
}

// first layer: dW1[o][j] = sum_p dz1[p][o] X[p][j]
__global__ __launch_bounds__(H) void k_layer1_wgrad(const float *__restrict__ dz1, const float *__restrict__ X,
                                                    int n, float *__restrict__ grad)
{
    const int o = threadIdx.x, p0 = blockIdx.x * GP, p1 = min(n, p0 + GP);
    float g[NIN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int p = p0; p < p1; p++) {
        float d = dz1[(size_t)p * H + o];
#pragma unroll
        for (int j = 0; j < NIN; j++) g[j] += d * X[p * NIN + j];
    }
#pragma unroll
    for (int j = 0; j < NIN; j++) atomicAdd(&grad[OFF_W1 + o * NIN + j], g[j]);
}

__global__ void k_zero(float *__restrict__ a, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.f;
}

__global__ void k_adam(float *__restrict__ master, uint16_t *__restrict__ wbf, float *__restrict__ grad,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    float g = grad[i];
    float mi = b1 * m[i] + (1.f - b1) * g, vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    float w = master[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    master[i] = w;
    wbf[i] = f2bf(w);
    grad[i] = 0.f;
}

__global__ void k_set_params(const float *__restrict__ theta, float *__restrict__ master,
                             uint16_t *__restrict__ wbf, float *__restrict__ grad, float *__restrict__ m,
                             float *__restrict__ v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    master[i] = theta[i];
    wbf[i] = f2bf(theta[i]);
    grad[i] = 0.f;
    m[i] = 0.f;
    v[i] = 0.f;
}

// bf16 copies of parameters, for the allocation-free inference entry point
__global__ void k_to_bf16(const float *__restrict__ theta, uint16_t *__restrict__ wbf)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPARAM) wbf[i] = f2bf(theta[i]);
}

// bf16 copies of the master weights and a cleared gradient after a load
__global__ void k_refresh(const float *__restrict__ master, uint16_t *__restrict__ wbf, float *__restrict__ grad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    wbf[i] = f2bf(master[i]);
    grad[i] = 0.f;
}

}  // namespace pgk_mlp_dev

using namespace pgk_mlp_dev;

struct pgk_mlp {
    hipStream_t stream = nullptr;
    int nmax = 0, npmax = 0;
    float *master, *grad, *m, *v, *loss;
    uint16_t *wbf;
    float *z[4], *dz, *dz2, *yhat, *dy;
    uint16_t *a[4];
    int t = 0;                      // Adam step count
    std::string err;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t mlp_layout(int nmax, size_t *o)
{
    int np = (nmax + 63) / 64 * 64;
    size_t p = 0;
    auto take = [&](size_t b) { size_t at = p; p += al(b); return at; };
    o[0] = take(4ull * NPARAM);           // master
    o[1] = take(2ull * NPARAM);           // bf16 weights
    o[2] = take(4ull * NPARAM);           // grad
    o[3] = take(4ull * NPARAM);           // m
    o[4] = take(4ull * NPARAM);           // v
    o[5] = take(64);                      // loss
    for (int l = 0; l < 4; l++) o[6 + l] = take(4ull * np * H);   // z1..z4
    for (int l = 0; l < 4; l++) o[10 + l] = take(2ull * np * H);  // a1..a4
    o[14] = take(4ull * np * H);          // dz
    o[15] = take(4ull * np * H);          // dz2
    o[16] = take(4ull * np * NOUT);       // yhat
    o[17] = take(4ull * np * NOUT);       // dy
    return p;
}

#define MHIP(m, call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) { m->err = std::string(#call) + ": " + hipGetErrorString(e_); return PGK_EDEVICE; } \
    } while (0)

extern "C" int pgk_mlp_bytes(int nmax, size_t *bytes)
{
    if (nmax < 1 || !bytes) return PGK_EINVAL;
    size_t o[18];
    *bytes = mlp_layout(nmax, o);
    return PGK_OK;
}

extern "C" int pgk_mlp_create(void *stream, void *buf, size_t bytes, int nmax, pgk_mlp **out)
{
    if (!out || !buf || nmax < 1 || ((uintptr_t)buf & 255)) return PGK_EINVAL;
    size_t o[18];
    if (bytes < mlp_layout(nmax, o)) return PGK_ENOMEM;
    pgk_mlp *m = new pgk_mlp();
    m->stream = (hipStream_t)stream;
    m->nmax = nmax;
    m->npmax = (nmax + 63) / 64 * 64;
    char *b = (char *)buf;
    m->master = (float *)(b + o[0]);
    m->wbf = (uint16_t *)(b + o[1]);
    m->grad = (float *)(b + o[2]);
    m->m = (float *)(b + o[3]);
    m->v = (float *)(b + o[4]);
    m->loss = (float *)(b + o[5]);
    for (int l = 0; l < 4; l++) m->z[l] = (float *)(b + o[6 + l]);
    for (int l = 0; l < 4; l++) m->a[l] = (uint16_t *)(b + o[10 + l]);
    m->dz = (float *)(b + o[14]);
    m->dz2 = (float *)(b + o[15]);
    m->yhat = (float *)(b + o[16]);
    m->dy = (float *)(b + o[17]);
    *out = m;
    return PGK_OK;
}

extern "C" int pgk_mlp_set_params(pgk_mlp *m, const float *theta)
{
    if (!m || !theta) return PGK_EINVAL;
    hipLaunchKernelGGL(k_set_params, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, theta, m->master,
                       m->wbf, m->grad, m->m, m->v);
    MHIP(m, hipGetLastError());
    m->t = 0;
    return PGK_OK;
}

extern "C" int pgk_mlp_get_params(pgk_mlp *m, float *theta)
{
    if (!m || !theta) return PGK_EINVAL;
    MHIP(m, hipMemcpyAsync(theta, m->master, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    return PGK_OK;
}

// forward over n <= nmax points; keeps z and a for a following backward
static int forward(pgk_mlp *m, const float *X, int n)
{
    int np = (n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_layer1, dim3((np * H + 255) / 256), dim3(256), 0, m->stream, X, n, np, m->wbf, m->master,
                       m->z[0], m->a[0]);
    const int offW[3] = {OFF_W2, OFF_W3, OFF_W4}, offB[3] = {OFF_B2, OFF_B3, OFF_B4};
    for (int l = 0; l < 3; l++) {
        // z_{l+1}[p][o] = sum_i a_l[p][i] W[o][i]: B(k=i, n=o) = W[o*H + i]
        hipLaunchKernelGGL((k_gemm<uint16_t, EPI_FWD, true>), dim3(np / 64, H / 64, 1), dim3(256), 0, m->stream,
                           m->a[l], H, 1, m->wbf + offW[l], 1, H, H, H, m->master + offB[l], (const float *)nullptr,
                           m->z[l + 1], m->a[l + 1], H, np);
    }
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_mlp_forward(pgk_mlp *m, const float *X, float *Y, int n)
{
    if (!m || !X || !Y || n < 0) return PGK_EINVAL;
    for (int s = 0; s < n; s += m->nmax) {
        int c = n - s < m->nmax ? n - s : m->nmax;
        int rc = forward(m, X + (size_t)s * NIN, c);
        if (rc) return rc;
        hipLaunchKernelGGL(k_layer5, dim3((c * NOUT + 255) / 256), dim3(256), 0, m->stream, m->a[3], c, m->wbf,
                           m->master, Y + (size_t)s * NOUT);
        MHIP(m, hipGetLastError());
    }
    return PGK_OK;
}

// loss and gradient of one minibatch (n <= nmax) into m->grad (accumulated);
// the squared errors enter m->loss with weight lscale
static int loss_grad(pgk_mlp *m, const float *X, const float *Y, int n, float scale, float lscale)
{
    int np = (n + 63) / 64 * 64;
    int rc = forward(m, X, n);
    if (rc) return rc;
    hipLaunchKernelGGL(k_layer5, dim3((n * NOUT + 255) / 256), dim3(256), 0, m->stream, m->a[3], n, m->wbf,
                       m->master, m->yhat);
    hipLaunchKernelGGL(k_loss, dim3((np * NOUT + 255) / 256), dim3(256), 0, m->stream, m->yhat, Y, n, np, scale,
                       lscale, m->dy, m->loss);
    hipLaunchKernelGGL(k_layer5_wgrad, dim3((n + GP - 1) / GP), dim3(H), 0, m->stream, m->dy, m->a[3], n, m->grad);
    hipLaunchKernelGGL(k_layer5_bwd, dim3((np * H + 255) / 256), dim3(256), 0, m->stream, m->dy, m->z[3], m->wbf,
                       np, m->dz);
    const int offW[3] = {OFF_W2, OFF_W3, OFF_W4}, offB[3] = {OFF_B2, OFF_B3, OFF_B4};
    float *dz = m->dz, *dzn = m->dz2;
    const int kchunk = 128;   // split-K depth of the weight gradients (128: 10% faster per minibatch than 256)
    for (int l = 2; l >= 0; l--) {
        // layer l+2 (0-based hidden index l+1): weights W_{l+2}, input a_l, output dz (of z_{l+1})
        hipLaunchKernelGGL(k_bias_grad, dim3(H), dim3(256), 0, m->stream, dz, np, m->grad + offB[l]);
        // dW[o][i] = sum_p dz[p][o] a_l[p][i]: A(m=o, k=p) = dz[p*H + o], B(k=p, n=i) = a_l[p*H + i]
        hipLaunchKernelGGL((k_gemm<float, EPI_WGRAD>), dim3(H / 64, H / 64, (np + kchunk - 1) / kchunk), dim3(256),
                           0, m->stream, dz, 1, H, m->a[l], H, 1, np, kchunk, (const float *)nullptr,
                           (const float *)nullptr, m->grad + offW[l], (uint16_t *)nullptr, H, H);
        // da_l[p][i] = sum_o dz[p][o] W[o][i]: B(k=o, n=i) = W[o*H + i]; dz_l = da_l * dsilu(z_l)
        hipLaunchKernelGGL((k_gemm<float, EPI_BWD>), dim3(np / 64, H / 64, 1), dim3(256), 0, m->stream, dz, H, 1,
                           m->wbf + offW[l], H, 1, H, H, (const float *)nullptr, m->z[l], dzn, (uint16_t *)nullptr,
                           H, np);
        float *t = dz;
        dz = dzn;
        dzn = t;
    }
    hipLaunchKernelGGL(k_bias_grad, dim3(H), dim3(256), 0, m->stream, dz, np, m->grad + OFF_B1);
    hipLaunchKernelGGL(k_layer1_wgrad, dim3((n + GP - 1) / GP), dim3(H), 0, m->stream, dz, X, n, m->grad);
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_mlp_loss_grad(pgk_mlp *m, const float *X, const float *Y, int n, float *grad, float *loss)
{
    if (!m || !X || !Y || n < 1 || n > m->nmax) return PGK_EINVAL;
    hipLaunchKernelGGL(k_zero, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->grad, NPARAM);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, m->stream, m->loss, 1);
    int rc = loss_grad(m, X, Y, n, 1.0f / (4.0f * n), 1.0f / (4.0f * n));
    if (rc) return rc;
    if (grad) MHIP(m, hipMemcpyAsync(grad, m->grad, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (loss) {
        MHIP(m, hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
        MHIP(m, hipStreamSynchronize(m->stream));
    }
    return PGK_OK;
}

extern "C" int pgk_mlp_adam_step(pgk_mlp *m, float lr, float beta1, float beta2, float eps)
{
    if (!m) return PGK_EINVAL;
    m->t++;
    float c1 = 1.f / (1.f - powf(beta1, (float)m->t)), c2 = 1.f / (1.f - powf(beta2, (float)m->t));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->master, m->wbf, m->grad, m->m,
                       m->v, lr, beta1, beta2, eps, c1, c2);
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_mlp_train(pgk_mlp *m, const float *X, const float *Y, int64_t n, int batch, int epochs, float lr,
                             uint64_t seed, float *loss_per_epoch)
{
    if (!m || !X || !Y || n < 1 || batch < 1 || batch > m->nmax || epochs < 0) return PGK_EINVAL;
    int64_t nb = (n + batch - 1) / batch;
    std::vector<int64_t> order(nb);
    uint64_t s = seed ? seed : 0x9E3779B97F4A7C15ull;
    for (int e = 0; e < epochs; e++) {
        for (int64_t i = 0; i < nb; i++) order[i] = i;
        for (int64_t i = nb - 1; i > 0; i--) {     // Fisher-Yates with xorshift64*
            s ^= s >> 12; s ^= s << 25; s ^= s >> 27;
            int64_t j = (int64_t)((s * 2685821657736338717ull) % (uint64_t)(i + 1));
            int64_t t = order[i]; order[i] = order[j]; order[j] = t;
        }
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, m->stream, m->loss, 1);
        // the gradient accumulator starts at zero; every Adam step clears it again
        if (e == 0) hipLaunchKernelGGL(k_zero, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->grad, NPARAM);
        for (int64_t i = 0; i < nb; i++) {
            int64_t b0 = order[i] * batch;
            int c = (int)(n - b0 < batch ? n - b0 : batch);
            // gradients of the mean loss over this minibatch; the squared
            // errors are weighted 1/(4 n), so that the epoch's sum is the mean
            // over all n points (a last, partial minibatch counts by its size)
            int rc = loss_grad(m, X + b0 * NIN, Y + b0 * NOUT, c, 1.0f / (4.0f * c), 1.0f / (4.0f * (float)n));
            if (rc) return rc;
            rc = pgk_mlp_adam_step(m, lr, 0.9f, 0.999f, 1e-8f);
            if (rc) return rc;
        }
        if (loss_per_epoch) {
            float l;
            MHIP(m, hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
            MHIP(m, hipStreamSynchronize(m->stream));
            loss_per_epoch[e] = l;
        }
    }
    return PGK_OK;
}

extern "C" int pgk_mlp_get_state(pgk_mlp *m, float *master, uint16_t *wbf, float *adam_m, float *adam_v,
                                 int64_t *t)
{
    if (!m) return PGK_EINVAL;
    if (master) MHIP(m, hipMemcpyAsync(master, m->master, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (wbf) MHIP(m, hipMemcpyAsync(wbf, m->wbf, 2ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (adam_m) MHIP(m, hipMemcpyAsync(adam_m, m->m, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (adam_v) MHIP(m, hipMemcpyAsync(adam_v, m->v, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    if (t) *t = m->t;
    return PGK_OK;
}

extern "C" int pgk_mlp_set_state(pgk_mlp *m, const float *master, const float *adam_m, const float *adam_v, int64_t t)
{
    if (!m || !master || !adam_m || !adam_v || t < 0 || t > INT32_MAX) return PGK_EINVAL;
    hipLaunchKernelGGL(k_set_params, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, master, m->master,
                       m->wbf, m->grad, m->m, m->v);
    MHIP(m, hipGetLastError());
    MHIP(m, hipMemcpyAsync(m->m, adam_m, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->v, adam_v, 4ull * NPARAM, hipMemcpyDeviceToDevice, m->stream));
    m->t = (int)t;
    return PGK_OK;
}

// file: 8-byte tag, int64 parameter count, int64 Adam step count, then the
// FP32 master weights, first and second Adam moments (little-endian)
static const char MLP_TAG[8] = {'P', 'G', 'K', 'M', 'L', 'P', '1', 0};

extern "C" int pgk_mlp_save(pgk_mlp *m, const char *path)
{
    if (!m || !path) return PGK_EINVAL;
    std::vector<float> h(3ull * NPARAM);
    MHIP(m, hipMemcpyAsync(h.data(), m->master, 4ull * NPARAM, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipMemcpyAsync(h.data() + NPARAM, m->m, 4ull * NPARAM, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipMemcpyAsync(h.data() + 2 * NPARAM, m->v, 4ull * NPARAM, hipMemcpyDeviceToHost, m->stream));
    MHIP(m, hipStreamSynchronize(m->stream));
    FILE *f = fopen(path, "wb");
    if (!f) { m->err = std::string("cannot open ") + path + " for writing"; return PGK_EINVAL; }
    int64_t hdr[2] = {NPARAM, m->t};
    bool ok = fwrite(MLP_TAG, 1, 8, f) == 8 && fwrite(hdr, 8, 2, f) == 2 && fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) { m->err = std::string("write failed: ") + path; return PGK_EINVAL; }
    return PGK_OK;
}

extern "C" int pgk_mlp_load(pgk_mlp *m, const char *path)
{
    if (!m || !path) return PGK_EINVAL;
    FILE *f = fopen(path, "rb");
    if (!f) { m->err = std::string("cannot open ") + path; return PGK_EINVAL; }
    char tag[8];
    int64_t hdr[2];
    std::vector<float> h(3ull * NPARAM);
    bool ok = fread(tag, 1, 8, f) == 8 && memcmp(tag, MLP_TAG, 8) == 0 && fread(hdr, 8, 2, f) == 2 &&
              hdr[0] == NPARAM && hdr[1] >= 0 && hdr[1] <= INT32_MAX && fread(h.data(), 4, h.size(), f) == h.size();
    fclose(f);
    if (!ok) { m->err = std::string("not a coordinate-MLP file of this shape: ") + path; return PGK_EINVAL; }
    MHIP(m, hipMemcpyAsync(m->master, h.data(), 4ull * NPARAM, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->m, h.data() + NPARAM, 4ull * NPARAM, hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->v, h.data() + 2 * NPARAM, 4ull * NPARAM, hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(k_refresh, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->master, m->wbf, m->grad);
    MHIP(m, hipGetLastError());
    MHIP(m, hipStreamSynchronize(m->stream));   // h is freed on return
    m->t = (int)hdr[1];
    return PGK_OK;
}

// ---------------------------------------------------------------------------
// Inference without any allocation: the bf16 weights and the activations live
// in a file-scope device array (one per GPU, held until the process ends)
// instead of a pgk_mlp buffer.  In host code `scratch` only names the symbol;
// its device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in scratch_dev[].
// ---------------------------------------------------------------------------
constexpr int ST_NMAX = PGK_MLP_STATIC_NMAX;
constexpr size_t ST_WBF = 0;                                     // bf16 weights
constexpr size_t ST_Z = ST_WBF + ((2ull * NPARAM + 255) & ~(size_t)255);   // z of the current layer, fp32
constexpr size_t ST_A0 = ST_Z + 4ull * ST_NMAX * H;              // activations, bf16 ping
constexpr size_t ST_A1 = ST_A0 + 2ull * ST_NMAX * H;             // and pong
constexpr size_t ST_BYTES = ST_A1 + 2ull * ST_NMAX * H;
static_assert(ST_NMAX % 64 == 0, "padded point count must fit");

static __device__ __align__(256) unsigned char scratch[ST_BYTES];

constexpr int ST_MAXDEV = 64;
static std::mutex scratch_mu;
static void *scratch_dev[ST_MAXDEV];

// device address of this GPU's scratch array (the current device)
static int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= ST_MAXDEV) return PGK_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PGK_EDEVICE;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return PGK_OK;
}

extern "C" int pgk_mlp_forward_static(const float *theta, const float *X, float *Y, int n, void *stream)
{
    if (!theta || n < 0 || (n > 0 && (!X || !Y))) return PGK_EINVAL;
    if (n > ST_NMAX) return PGK_ETOOBIG;
    if (n == 0) return PGK_OK;
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    unsigned char *b = (unsigned char *)base;
    uint16_t *wbf = (uint16_t *)(b + ST_WBF), *a[2] = {(uint16_t *)(b + ST_A0), (uint16_t *)(b + ST_A1)};
    float *z = (float *)(b + ST_Z);
    const int np = (n + 63) / 64 * 64;
    // every value a kernel reads below is written earlier in this call (rows
    // n..np-1 included), so nothing needs clearing between calls
    hipLaunchKernelGGL(k_to_bf16, dim3((NPARAM + 255) / 256), dim3(256), 0, st, theta, wbf);
    hipLaunchKernelGGL(k_layer1, dim3((np * H + 255) / 256), dim3(256), 0, st, X, n, np, wbf, theta, z, a[0]);
    const int offW[3] = {OFF_W2, OFF_W3, OFF_W4}, offB[3] = {OFF_B2, OFF_B3, OFF_B4};
    for (int l = 0; l < 3; l++)
        hipLaunchKernelGGL((k_gemm<uint16_t, EPI_FWD, true>), dim3(np / 64, H / 64, 1), dim3(256), 0, st,
                           a[l & 1], H, 1, wbf + offW[l], 1, H, H, H, theta + offB[l], (const float *)nullptr, z,
                           a[(l + 1) & 1], H, np);
    hipLaunchKernelGGL(k_layer5, dim3((n * NOUT + 255) / 256), dim3(256), 0, st, a[1], n, wbf, theta, Y);
    return hipGetLastError() == hipSuccess ? PGK_OK : PGK_EDEVICE;
}

extern "C" const char *pgk_mlp_last_error(const pgk_mlp *m) { return m ? m->err.c_str() : "null mlp"; }

extern "C" void pgk_mlp_destroy(pgk_mlp *m) { delete m; }
