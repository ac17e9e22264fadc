// mlp.hip -- coordinate MLP of the learned warm start: 6 inputs -> 4 hidden
// layers of 128 (SiLU) -> 4 outputs, BF16 weights and activations with FP32
// accumulation, FP32 master weights and Adam.
//
// Inference: the three 128x128 layers run on the matrix cores as 64x64
// work-group tiles of 16x16x16 bf16 MFMA blocks (four waves, each a 16x64
// slab), the 6-wide first layer and the 4-wide last layer on the vector ALUs.
// Training: one fused kernel per minibatch runs the forward and backward
// passes of 16 points per work-group with the activations in LDS and the
// 128x128 products on 16x16x32 bf16 MFMA blocks; a second kernel contracts the
// bf16 factors of the weight gradients over the whole minibatch on MFMA, sums
// the small-gradient slots and applies Adam.  Parameter order: W1[128][6], b1, W2[128][128], b2, W3, b3,
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

// One 128x128 layer of the forward pass as a product on the matrix cores:
// C[m][n] = sum_k A[m][k] B[n][k] with A (activations, bf16 [m][lda]) and B
// (weights W[n][k], bf16) contiguous along k; work-group tile 64x64 (M0 =
// 64 blockIdx.x, N0 = 64 blockIdx.y), four waves each a 16x64 slab of
// 16x16x16 bf16 blocks.  Epilogue: z = C + bias[n] -> zout[m][n] (fp32),
// silu(z) -> aout[m][n] (bf16), rows m < mvalid.
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

__global__ __launch_bounds__(256) void k_gemm(const uint16_t *__restrict__ A, int lda,
                                              const uint16_t *__restrict__ B, int ldb, int K,
                                              const float *__restrict__ bias, float *__restrict__ zout,
                                              uint16_t *__restrict__ aout, int ldc, int mvalid)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + wave * 16, n0 = blockIdx.y * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4f32 acc[4];
    for (int b = 0; b < 4; b++) acc[b] = v4f32{0.f, 0.f, 0.f, 0.f};
    // K in blocks of four 16-deep MFMA steps: all loads of a block are issued
    // before its products, so their latencies overlap
    constexpr int KB = 4;
    for (int k1 = 0; k1 < K; k1 += 16 * KB) {
        v4i16 a[KB], bb[KB][4];
#pragma unroll
        for (int s = 0; s < KB; s++) {
            const int k0 = k1 + 16 * s;
            const bool in = k0 < K;
            a[s] = in ? load4_bf(A + (size_t)(m0 + r) * lda + k0 + kq) : v4i16{0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < 4; b++)
                bb[s][b] = in ? load4_bf(B + (size_t)(n0 + 16 * b + r) * ldb + k0 + kq) : v4i16{0, 0, 0, 0};
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
            if (m < mvalid) {
                float z = acc[b][j] + bias[n];
                zout[(size_t)m * ldc + n] = z;
                aout[(size_t)m * ldc + n] = f2bf(silu(z));
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

__global__ void k_zero(float *__restrict__ a, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.f;
}

// bf16 copy of parameter i; the three 128x128 weights also go transposed into
// wbfT ([layer][in][out], the operand layout of the backward products)
__device__ inline void put_bf(uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT, int i, float w)
{
    const uint16_t b = f2bf(w);
    wbf[i] = b;
    const int rel = i - OFF_W2, li = rel / (H * H + H), rem = rel - li * (H * H + H);
    if (rel >= 0 && li < 3 && rem < H * H) wbfT[li * H * H + (rem % H) * H + rem / H] = b;
}

__global__ void k_adam(float *__restrict__ master, uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT,
                       float *__restrict__ grad,
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
    put_bf(wbf, wbfT, i, w);
    grad[i] = 0.f;
}

__global__ void k_set_params(const float *__restrict__ theta, float *__restrict__ master,
                             uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT, float *__restrict__ grad,
                             float *__restrict__ m, float *__restrict__ v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    master[i] = theta[i];
    put_bf(wbf, wbfT, i, theta[i]);
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
__global__ void k_refresh(const float *__restrict__ master, uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT,
                          float *__restrict__ grad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    put_bf(wbf, wbfT, i, master[i]);
    grad[i] = 0.f;
}


// ---------------------------------------------------------------------------
// Training pass of one minibatch in two kernels.
//
// k_fb: forward, loss and backward of FB_P points per work-group of eight
// waves, all five layers, the products over units on gfx950's 16x16x32 bf16
// matrix instructions.  Activations and dL/dz stay in LDS, z in registers.
// The weight gradients of
// the 128x128 layers, dW = sum_p r(dz)[p][o] a[p][i], are contractions over
// all points of the minibatch: the work-group writes their bf16 factors
// (r(dz) and a, transposed: [unit][point]) to global memory, and its share of
// the small gradients (W1, W5, the biases) and of the loss to its own slot.
//
// k_grad_adam: one work-group per 16x16 tile of dW2, dW3, dW4 contracts the
// factors over the whole minibatch (four waves, each every fourth 32-point
// step, summed in a fixed order), a few more sum the small slots in slot
// order; each then applies Adam to its parameters.  The gradient is the same
// bits on every run.
//
// The bf16 roundings are those of the reference: weights, activations entering
// layers 2-5, and dL/dz of layers 2-4 where it meets a weight or an activation;
// x, dL/dy and dL/dz1 stay in fp32.  SiLU and its derivative take the hardware
// exponential and reciprocal here (a few fp32 ulps; the activations they feed
// are rounded to bf16).
//
// Fragment layout of the 16x16x32 product D = A B (lane l, r = l % 16,
// g = l / 16): A holds A[r][8g .. 8g+7], B holds B[8g .. 8g+7][r], D holds
// D[4g + j][r], j = 0..3.  A [point][unit] tile (16 x 128) is split over the
// waves of k_fb by columns: wave w holds units 16 w .. 16 w + 15.
constexpr int FB_P = 16;          // points per work-group
constexpr int FB_WG = 512;        // eight waves
constexpr int RS = H + 8;         // row stride (bf16) of [point][unit] arrays: rows 16 bytes apart mod 256
constexpr int WS = H + 8;         // row stride of the staged 128x128 weight
// small-gradient slot: W1, b1, b2, b3, b4, W5, b5
constexpr int SM_W1 = 0, SM_B1 = SM_W1 + H * NIN, SM_B2 = SM_B1 + H, SM_W5 = SM_B2 + 3 * H, SM_B5 = SM_W5 + NOUT * H;
constexpr int NSMALL = SM_B5 + NOUT;

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// eight bf16 at a 16-byte aligned address as one matrix operand
__device__ inline v8bf ld8(const uint16_t *p) { return __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u *>(p)); }

__device__ inline v4f32 mma32(v8bf a, v8bf b, v4f32 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

__device__ inline float silu_fast(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ inline float dsilu_fast(float z)
{
    float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// a 128x128 bf16 matrix (row-major, 128 per row) into sW with row stride WS
__device__ inline void stage_w(const uint16_t *__restrict__ src, uint16_t *sW)
{
    for (int c = threadIdx.x; c < H * H / 8; c += FB_WG) {
        const int o = c >> 4, i0 = (c & 15) * 8;
        *reinterpret_cast<v4u *>(sW + o * WS + i0) = *reinterpret_cast<const v4u *>(src + o * H + i0);
    }
}

// the same staging split in two: the loads into registers (issued early, so
// that their latency overlaps other work) and the stores into sW
struct WPre {
    v4u v[H * H / 8 / FB_WG];
};
__device__ inline void w_load(const uint16_t *__restrict__ src, WPre &pre)
{
#pragma unroll
    for (int k = 0; k < H * H / 8 / FB_WG; k++) {
        const int c = threadIdx.x + k * FB_WG, o = c >> 4, i0 = (c & 15) * 8;
        pre.v[k] = *reinterpret_cast<const v4u *>(src + o * H + i0);
    }
}
__device__ inline void w_store(const WPre &pre, uint16_t *sW)
{
#pragma unroll
    for (int k = 0; k < H * H / 8 / FB_WG; k++) {
        const int c = threadIdx.x + k * FB_WG, o = c >> 4, i0 = (c & 15) * 8;
        *reinterpret_cast<v4u *>(sW + o * WS + i0) = pre.v[k];
    }
}

// column sums over the work-group's points of a [point][unit] tile held in the
// product layout into red[H]
__device__ inline void col_sums(v4f32 d, float *red)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    float s = (d[0] + d[1]) + (d[2] + d[3]);
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (g == 0) red[16 * w + r] = s;
}

// work-group barrier that orders LDS only: the global stores of the pass (the
// factors and slots, read by the next kernel) stay in flight across it
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// four bf16 of consecutive points as one 8-byte store
__device__ inline void put4(uint16_t *dst, const uint16_t *b4)
{
    *reinterpret_cast<uint2 *>(dst) = make_uint2(b4[0] | ((uint32_t)b4[1] << 16), b4[2] | ((uint32_t)b4[3] << 16));
}

// One minibatch of a graph-replayed epoch, written by the host before each
// replay: its first point and size, the weight of its dL/dy, and the Adam
// bias corrections of its step.  Each graph node holds the address of its own
// record, so a null record means the kernel arguments name the minibatch.
struct MbRec {
    int64_t b0;
    int n;
    float scale, c1, c2;
};

// fT: bf16 factors [2][3][H][ldp]; fT[0][li] = r(dz) of layer li + 2, fT[1][li]
// = a of layer li + 1 (the input of W_{li+2}), point p of the minibatch at
// column p; small: [slot][NSMALL]; lpart: [slot]
__global__ __launch_bounds__(FB_WG) void k_fb(const float *__restrict__ X, const float *__restrict__ Y, int n,
                                              float scale, float lscale, const uint16_t *__restrict__ wbf,
                                              const uint16_t *__restrict__ wbfT, const float *__restrict__ master,
                                              uint16_t *__restrict__ fT, int ldp, float *__restrict__ small,
                                              float *__restrict__ lpart, const MbRec *__restrict__ rec)
{
    if (rec) {
        const MbRec mb = *rec;
        n = mb.n;
        X += mb.b0 * NIN;
        Y += mb.b0 * NOUT;
        scale = mb.scale;
        if ((int)blockIdx.x * FB_P >= n) return;     // the grid covers a full minibatch
    }
    __shared__ __align__(16) uint16_t sW[H * WS];
    __shared__ __align__(16) uint16_t sRow[2][FB_P * RS];
    __shared__ float sX[FB_P * NIN], sDy[FB_P * NOUT], sRed[H], sLoss[FB_WG / 64], sDz1[FB_P * H];
    __shared__ float sW1[H * NIN], sW5[NOUT * H], sB[4 * H + NOUT];   // bf16 weights as float; biases

    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, r = l & 15, g = l >> 4;
    const int o = 16 * w + r;                          // this lane's unit in the product layout
    const int p0 = blockIdx.x * FB_P;
    float *sm = small + (size_t)blockIdx.x * NSMALL;
    // the 128x128 layers li = 0, 1, 2 (W2, W3, W4) and their biases; z of layer li + 1
    auto offW = [](int li) { return OFF_W2 + li * (H * H + H); };
    auto offB = [](int li) { return OFF_W2 + li * (H * H + H) + H * H; };
    // a lane holds the same points and unit in every layer: it keeps its z of
    // layers 1-4 in registers for the backward pass
    float zk[4][4];
    // this lane's four consecutive points of unit u in factor f of layer li
    auto fcol = [&](int f, int li, int u) { return fT + ((size_t)(f * 3 + li) * H + u) * ldp + p0 + 4 * g; };
    static_assert(OFF_W3 == OFF_W2 + H * H + H && OFF_W4 == OFF_W3 + H * H + H && OFF_B4 == OFF_W4 + H * H,
                  "layer offsets");

    for (int i = tid; i < FB_P * NIN; i += FB_WG) sX[i] = p0 + i / NIN < n ? X[(size_t)p0 * NIN + i] : 0.f;
    for (int i = tid; i < H * NIN; i += FB_WG) sW1[i] = bf2f(wbf[OFF_W1 + i]);
    for (int i = tid; i < NOUT * H; i += FB_WG) sW5[i] = bf2f(wbf[OFF_W5 + i]);
    for (int i = tid; i < 4 * H + NOUT; i += FB_WG)
        sB[i] = master[i < H ? OFF_B1 + i : i < 4 * H ? offB(i / H - 1) + i % H : OFF_B5 + i - 4 * H];
    stage_w(wbf + OFF_W2, sW);
    lds_barrier();

    // layer 1 (vector ALUs): z1 = W1 x + b1
    {
        uint16_t a4[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int p = 4 * g + j;
            float z = sB[o];
            for (int k = 0; k < NIN; k++) z += sW1[o * NIN + k] * sX[p * NIN + k];
            zk[0][j] = z;
            a4[j] = f2bf(silu_fast(z));
            sRow[0][p * RS + o] = a4[j];
        }
        put4(fcol(1, 0, o), a4);
    }
    lds_barrier();

    // layers 2-4 on the matrix cores
    WPre pre;
#pragma unroll
    for (int li = 0; li < 3; li++) {
        const uint16_t *in = sRow[li & 1];
        uint16_t *out = sRow[(li + 1) & 1];
        // the next weights (W3, W4, then W4 transposed for the backward pass) load during this product
        w_load(li < 2 ? wbf + offW(li + 1) : wbfT + 2 * H * H, pre);
        v4f32 acc = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < H / 32; ks++)
            acc = mma32(ld8(in + r * RS + 32 * ks + 8 * g), ld8(sW + o * WS + 32 * ks + 8 * g), acc);
        lds_barrier();
        if (li < 2) w_store(pre, sW);
        const float bias = sB[(li + 1) * H + o];
        uint16_t a4[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int p = 4 * g + j;
            const float z = acc[j] + bias;
            zk[li + 1][j] = z;
            a4[j] = f2bf(silu_fast(z));
            out[p * RS + o] = a4[j];
        }
        if (li < 2) put4(fcol(1, li + 1, o), a4);
        lds_barrier();
    }
    const uint16_t *a4s = sRow[1];                    // a4, row-major

    // layer 5, the loss and dL/dy = 2 (y - Y) scale (zero on padding rows):
    // eight threads per output split the 128-term sums
    {
        const int q = tid >> 3, p = q >> 2, o5 = q & 3, h = tid & 7;
        float y = 0.f;
        for (int k = 16 * h; k < 16 * h + 16; k++) y += sW5[o5 * H + k] * bf2f(a4s[p * RS + k]);
        y += __shfl_xor(y, 1, 64);
        y += __shfl_xor(y, 2, 64);
        y += __shfl_xor(y, 4, 64);
        y += sB[4 * H + o5];
        const float d = p0 + p < n ? y - Y[(size_t)(p0 + p) * NOUT + o5] : 0.f;
        float lt = 0.f;
        if (h == 0) {
            sDy[q] = 2.f * d * scale;
            lt = d * d * lscale;
        }
        for (int off = 32; off > 0; off >>= 1) lt += __shfl_xor(lt, off, 64);
        if (l == 0) sLoss[w] = lt;
    }
    lds_barrier();
    if (tid == 0) {
        float s = 0.f;
        for (int i = 0; i < FB_WG / 64; i++) s += sLoss[i];
        lpart[blockIdx.x] = s;
    }
    // dW5 = dy^T a4, db5 = sum dy
    {
        const int o5 = tid >> 7, k = tid & (H - 1);
        float s = 0.f;
        for (int p = 0; p < FB_P; p++) s += sDy[p * NOUT + o5] * bf2f(a4s[p * RS + k]);
        sm[SM_W5 + tid] = s;
    }
    if (tid < NOUT) {
        float s = 0.f;
        for (int p = 0; p < FB_P; p++) s += sDy[p * NOUT + tid];
        sm[SM_B5 + tid] = s;
    }
    // dz4 = (dy W5) * dsilu(z4), in the product layout
    v4f32 dz;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int p = 4 * g + j;
        float da = 0.f;
        for (int o5 = 0; o5 < NOUT; o5++) da += sDy[p * NOUT + o5] * sW5[o5 * H + o];
        dz[j] = da * dsilu_fast(zk[3][j]);
    }
    lds_barrier();

    // layers 4, 3, 2: bias gradients and the r(dz) factor of the weight
    // gradients, then dL/dz of the layer below
    uint16_t *dzRow = sRow[0];
#pragma unroll
    for (int li = 2; li >= 0; li--) {
        col_sums(dz, sRed);
        {
            uint16_t b4[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                b4[j] = f2bf(dz[j]);
                dzRow[(4 * g + j) * RS + o] = b4[j];
            }
            put4(fcol(0, li, o), b4);
        }
        w_store(pre, sW);                             // W transposed: sW[i][o] = W[o][i]
        lds_barrier();
        if (li > 0) w_load(wbfT + (li - 1) * H * H, pre);
        if (tid < H) sm[SM_B2 + li * H + tid] = sRed[tid];
        // da[p][i] = sum_o r(dz)[p][o] W[o][i]; dz of the layer below = da dsilu(z)
        v4f32 acc = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < H / 32; ks++)
            acc = mma32(ld8(dzRow + r * RS + 32 * ks + 8 * g), ld8(sW + o * WS + 32 * ks + 8 * g), acc);
#pragma unroll
        for (int j = 0; j < 4; j++) dz[j] = acc[j] * dsilu_fast(zk[li][j]);
        lds_barrier();
    }

    // layer 1: db1 = sum dz1, dW1 = dz1^T x (both in fp32)
    col_sums(dz, sRed);
#pragma unroll
    for (int j = 0; j < 4; j++) sDz1[(4 * g + j) * H + o] = dz[j];
    lds_barrier();
    if (tid < H) sm[SM_B1 + tid] = sRed[tid];
    for (int idx = tid; idx < H * NIN; idx += FB_WG) {
        const int oo = idx / NIN, k = idx - oo * NIN;
        float s = 0.f;
        for (int p = 0; p < FB_P; p++) s += sDz1[p * H + oo] * sX[p * NIN + k];
        sm[SM_W1 + idx] = s;
    }
}

// gradient gs of parameter i into grad, or (adam) an Adam step
__device__ inline void apply_grad(int i, float gs, float *__restrict__ grad, float *__restrict__ master,
                                  uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT, float *__restrict__ m,
                                  float *__restrict__ v, int adam, float lr, float b1, float b2, float eps, float c1,
                                  float c2)
{
    if (!adam) {
        grad[i] = gs;
        return;
    }
    float mi = b1 * m[i] + (1.f - b1) * gs, vi = b2 * v[i] + (1.f - b2) * gs * gs;
    m[i] = mi;
    v[i] = vi;
    float wv = master[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    master[i] = wv;
    put_bf(wbf, wbfT, i, wv);
}

// parameter index of small-slot entry e
__device__ inline int small_param(int e)
{
    return e < SM_B1 ? OFF_W1 + e : e < SM_B2 ? OFF_B1 + e - SM_B1
         : e < SM_W5 ? OFF_W2 + ((e - SM_B2) / H) * (H * H + H) + H * H + (e - SM_B2) % H
         : e < SM_B5 ? OFF_W5 + e - SM_W5 : OFF_B5 + e - SM_B5;
}

constexpr int GA_TILES = 3 * (H / 16) * (H / 16);               // 16x16 tiles of dW2, dW3, dW4
constexpr int GA_WG = 512;
constexpr int GA_SMALL = (NSMALL + 63) / 64;                    // 64 small-slot entries per work-group

// Work-groups 0 .. GA_TILES-1: one 16x16 tile of dW2-dW4 over np points (np a
// multiple of 16), eight waves each taking every eighth 32-point step, eight
// steps' loads issued before their products; the waves' sums are added in a
// fixed order.  The rest: 64 small-slot entries each, eight threads per entry
// (slots c = part mod 8, sixteen loads in flight), added in a fixed order;
// work-group GA_TILES also adds the loss slots to *loss.
__global__ __launch_bounds__(GA_WG) void k_grad_adam(const uint16_t *__restrict__ fT, int ldp, int np,
                                                     const float *__restrict__ small, int nslot,
                                                     const float *__restrict__ lpart, float *__restrict__ loss,
                                                     float *__restrict__ grad, float *__restrict__ master,
                                                     uint16_t *__restrict__ wbf, uint16_t *__restrict__ wbfT,
                                                     float *__restrict__ m, float *__restrict__ v, int adam, float lr,
                                                     float b1, float b2, float eps, float c1, float c2,
                                                     const MbRec *__restrict__ rec)
{
    __shared__ float red[8][256];
    const int tid = threadIdx.x;
    if (rec) {
        const MbRec mb = *rec;
        nslot = (mb.n + FB_P - 1) / FB_P;
        np = nslot * FB_P;
        c1 = mb.c1;
        c2 = mb.c2;
    }
    if (blockIdx.x < GA_TILES) {
        const int li = blockIdx.x / 64, t = blockIdx.x % 64, to = t >> 3, ti = t & 7;
        const int w = tid >> 6, l = tid & 63, r = l & 15, g = l >> 4;
        const uint16_t *dzT = fT + ((size_t)(0 * 3 + li) * H + 16 * to + r) * ldp;
        const uint16_t *aT = fT + ((size_t)(1 * 3 + li) * H + 16 * ti + r) * ldp;
        const v8bf zero = __builtin_bit_cast(v8bf, v4u{0u, 0u, 0u, 0u});
        v4f32 acc = v4f32{0.f, 0.f, 0.f, 0.f};
        const int nst = (np + 31) / 32;
        for (int s0 = w; s0 < nst; s0 += 64) {
            v8bf fa[8], fb[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int p = 32 * (s0 + 8 * u) + 8 * g;
                const bool in = p < np;
                fa[u] = in ? ld8(dzT + p) : zero;
                fb[u] = in ? ld8(aT + p) : zero;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) acc = mma32(fa[u], fb[u], acc);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) red[w][(4 * g + j) * 16 + r] = acc[j];
        __syncthreads();
        if (tid < 256) {
            const float gs = ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid])) +
                             ((red[4][tid] + red[5][tid]) + (red[6][tid] + red[7][tid]));
            const int i = OFF_W2 + li * (H * H + H) + (16 * to + (tid >> 4)) * H + 16 * ti + (tid & 15);
            apply_grad(i, gs, grad, master, wbf, wbfT, m, v, adam, lr, b1, b2, eps, c1, c2);
        }
    } else {
        const int q = tid & 63, part = tid >> 6;
        const int e = (blockIdx.x - GA_TILES) * 64 + q;
        if (blockIdx.x == GA_TILES && tid == 0) {
            float s = *loss;
            for (int c = 0; c < nslot; c++) s += lpart[c];
            *loss = s;
        }
        float s16[16];
#pragma unroll
        for (int u = 0; u < 16; u++) s16[u] = 0.f;
        if (e < NSMALL) {
            int c = part;
            for (; c + 8 * 15 < nslot; c += 128)
#pragma unroll
                for (int u = 0; u < 16; u++) s16[u] += small[(size_t)(c + 8 * u) * NSMALL + e];
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (c + 8 * u < nslot) s16[u] += small[(size_t)(c + 8 * u) * NSMALL + e];
        }
#pragma unroll
        for (int hh = 8; hh > 0; hh >>= 1)
#pragma unroll
            for (int u = 0; u < hh; u++) s16[u] += s16[u + hh];
        red[part][q] = s16[0];
        __syncthreads();
        if (part == 0 && e < NSMALL) {
            const float gs = ((red[0][q] + red[1][q]) + (red[2][q] + red[3][q])) +
                             ((red[4][q] + red[5][q]) + (red[6][q] + red[7][q]));
            apply_grad(small_param(e), gs, grad, master, wbf, wbfT, m, v, adam, lr, b1, b2, eps, c1, c2);
        }
    }
}

}  // namespace pgk_mlp_dev

using namespace pgk_mlp_dev;

struct pgk_mlp {
    hipStream_t stream = nullptr;
    int nmax = 0, npmax = 0;
    float *master, *grad, *m, *v, *loss;
    uint16_t *wbf;
    float *z[4], *dz, *dz2, *yhat, *dy;
    float *small, *lpart;           // per-work-group slots of the small gradients and of the loss
    uint16_t *fT;                   // bf16 factors of the 128x128 weight gradients, [2][3][H][ldp]
    int ldp = 0;                    // points per factor row (nmax rounded up to 16)
    uint16_t *wbfT;                 // transposed bf16 copies of W2, W3, W4
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
    const size_t nslot = (size_t)(nmax + FB_P - 1) / FB_P;
    o[18] = take(4ull * nslot * NSMALL);  // small-gradient slots
    o[19] = take(4ull * nslot);           // loss slots
    o[20] = take(2ull * 3 * H * H);       // transposed bf16 W2, W3, W4
    o[21] = take(2ull * 2 * 3 * H * (nslot * FB_P));   // weight-gradient factors
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
    size_t o[22];
    *bytes = mlp_layout(nmax, o);
    return PGK_OK;
}

extern "C" int pgk_mlp_create(void *stream, void *buf, size_t bytes, int nmax, pgk_mlp **out)
{
    if (!out || !buf || nmax < 1 || ((uintptr_t)buf & 255)) return PGK_EINVAL;
    size_t o[22];
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
    m->small = (float *)(b + o[18]);
    m->lpart = (float *)(b + o[19]);
    m->wbfT = (uint16_t *)(b + o[20]);
    m->fT = (uint16_t *)(b + o[21]);
    m->ldp = (nmax + FB_P - 1) / FB_P * FB_P;
    *out = m;
    return PGK_OK;
}

extern "C" int pgk_mlp_set_params(pgk_mlp *m, const float *theta)
{
    if (!m || !theta) return PGK_EINVAL;
    hipLaunchKernelGGL(k_set_params, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, theta, m->master,
                       m->wbf, m->wbfT, m->grad, m->m, m->v);
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
        hipLaunchKernelGGL(k_gemm, dim3(np / 64, H / 64, 1), dim3(256), 0, m->stream, m->a[l], H, m->wbf + offW[l], H,
                           H, m->master + offB[l], m->z[l + 1], m->a[l + 1], H, np);
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

// forward and backward of one minibatch (n <= nmax) in the fused kernel: one
// gradient and loss slot per work-group of FB_P points; the squared errors
// carry weight lscale, dL/dy = 2 (yhat - y) scale
static int fused_pass(pgk_mlp *m, const float *X, const float *Y, int n, float scale, float lscale)
{
    const int nslot = (n + FB_P - 1) / FB_P;
    hipLaunchKernelGGL(k_fb, dim3(nslot), dim3(FB_WG), 0, m->stream, X, Y, n, scale, lscale, m->wbf, m->wbfT,
                       m->master, m->fT, m->ldp, m->small, m->lpart, nullptr);
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

// the gradient of the last fused pass (the weight-gradient contractions and
// the small slots) into m->grad, or (adam) into an Adam step; the loss slots
// are added to m->loss
static int sum_slots(pgk_mlp *m, int n, bool adam, float lr, float beta1, float beta2, float eps)
{
    const int nslot = (n + FB_P - 1) / FB_P;
    float c1 = 0.f, c2 = 0.f;
    if (adam) {
        m->t++;
        c1 = 1.f / (1.f - powf(beta1, (float)m->t));
        c2 = 1.f / (1.f - powf(beta2, (float)m->t));
    }
    hipLaunchKernelGGL(k_grad_adam, dim3(GA_TILES + GA_SMALL), dim3(GA_WG), 0, m->stream, m->fT, m->ldp, nslot * FB_P,
                       m->small, nslot, m->lpart, m->loss, m->grad, m->master, m->wbf, m->wbfT, m->m, m->v,
                       adam ? 1 : 0, lr, beta1, beta2, eps, c1, c2, nullptr);
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_mlp_loss_grad(pgk_mlp *m, const float *X, const float *Y, int n, float *grad, float *loss)
{
    if (!m || !X || !Y || n < 1 || n > m->nmax) return PGK_EINVAL;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, m->stream, m->loss, 1);
    int rc = fused_pass(m, X, Y, n, 1.0f / (4.0f * n), 1.0f / (4.0f * n));
    if (rc == PGK_OK) rc = sum_slots(m, n, false, 0.f, 0.f, 0.f, 0.f);
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
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->master, m->wbf, m->wbfT,
                       m->grad, m->m, m->v, lr, beta1, beta2, eps, c1, c2);
    MHIP(m, hipGetLastError());
    return PGK_OK;
}

// Training epochs as one replayed HIP graph: the graph zeroes the loss and
// holds, per minibatch, k_fb and k_grad_adam, each node with the address of
// its minibatch's record (MbRec).  Before each replay the host shuffles the
// minibatch order and writes the epoch's records (first point, size, Adam
// bias corrections) into the first activation buffer, which the training pass
// does not use.  The same minibatches, in the same order, with the same
// arithmetic as direct launches.
struct TrainRes {
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MbRec *hrec = nullptr;
    ~TrainRes()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        if (hrec) (void)hipHostFree(hrec);
    }
};

extern "C" int pgk_mlp_train(pgk_mlp *m, const float *X, const float *Y, int64_t n, int batch, int epochs, float lr,
                             uint64_t seed, float *loss_per_epoch)
{
    if (!m || !X || !Y || n < 1 || batch < 1 || batch > m->nmax || epochs < 0) return PGK_EINVAL;
    const int64_t nb = (n + batch - 1) / batch;
    if ((size_t)nb * sizeof(MbRec) > 4ull * m->npmax * H) {
        m->err = "too many minibatches for the record buffer (raise nmax)";
        return PGK_EINVAL;
    }
    if ((int64_t)m->t + nb * epochs > INT32_MAX) {
        m->err = "Adam step count would overflow";
        return PGK_EINVAL;
    }
    if (epochs == 0) return PGK_OK;
    TrainRes res;
    MHIP(m, hipHostMalloc((void **)&res.hrec, (size_t)nb * sizeof(MbRec), hipHostMallocDefault));
    std::vector<int64_t> order(nb);
    MbRec *drec = reinterpret_cast<MbRec *>(m->z[0]);
    const float lscale = 1.0f / (4.0f * (float)n), beta1 = 0.9f, beta2 = 0.999f;
    // record the epoch
    MHIP(m, hipStreamCreateWithFlags(&res.cs, hipStreamNonBlocking));
    MHIP(m, hipStreamBeginCapture(res.cs, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, res.cs, m->loss, 1);
    const int nwg = (batch + FB_P - 1) / FB_P;
    for (int64_t i = 0; i < nb; i++) {
        hipLaunchKernelGGL(k_fb, dim3(nwg), dim3(FB_WG), 0, res.cs, X, Y, 0, 0.f, lscale, m->wbf, m->wbfT, m->master,
                           m->fT, m->ldp, m->small, m->lpart, drec + i);
        hipLaunchKernelGGL(k_grad_adam, dim3(GA_TILES + GA_SMALL), dim3(GA_WG), 0, res.cs, m->fT, m->ldp, 0, m->small,
                           0, m->lpart, m->loss, m->grad, m->master, m->wbf, m->wbfT, m->m, m->v, 1, lr, beta1, beta2,
                           1e-8f, 0.f, 0.f, drec + i);
    }
    hipError_t ce = hipStreamEndCapture(res.cs, &res.graph);
    if (ce != hipSuccess) {
        m->err = std::string("graph capture: ") + hipGetErrorString(ce);
        return PGK_EDEVICE;
    }
    MHIP(m, hipGraphInstantiate(&res.exec, res.graph, nullptr, nullptr, 0));
    uint64_t s = seed ? seed : 0x9E3779B97F4A7C15ull;
    for (int e = 0; e < epochs; e++) {
        MHIP(m, hipStreamSynchronize(m->stream));   // the last epoch's records have been read
        for (int64_t i = 0; i < nb; i++) order[i] = i;
        for (int64_t i = nb - 1; i > 0; i--) {     // Fisher-Yates with xorshift64*
            s ^= s >> 12; s ^= s << 25; s ^= s >> 27;
            int64_t j = (int64_t)((s * 2685821657736338717ull) % (uint64_t)(i + 1));
            int64_t t = order[i]; order[i] = order[j]; order[j] = t;
        }
        for (int64_t i = 0; i < nb; i++) {
            MbRec &r = res.hrec[i];
            r.b0 = order[i] * batch;
            r.n = (int)(n - r.b0 < batch ? n - r.b0 : batch);
            r.scale = 1.0f / (4.0f * r.n);
            const float t = (float)(m->t + 1);   // the bias corrections of direct Adam steps
            r.c1 = 1.f / (1.f - powf(beta1, t));
            r.c2 = 1.f / (1.f - powf(beta2, t));
            m->t++;
        }
        MHIP(m, hipMemcpyAsync(drec, res.hrec, (size_t)nb * sizeof(MbRec), hipMemcpyHostToDevice, m->stream));
        MHIP(m, hipGraphLaunch(res.exec, m->stream));
        // the squared errors are weighted 1/(4 n): the epoch's sum is the
        // mean over all n points, whatever the size of the last minibatch
        if (loss_per_epoch) {
            float l;
            MHIP(m, hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
            MHIP(m, hipStreamSynchronize(m->stream));
            loss_per_epoch[e] = l;
        }
    }
    MHIP(m, hipStreamSynchronize(m->stream));
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
                       m->wbf, m->wbfT, m->grad, m->m, m->v);
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
    hipLaunchKernelGGL(k_refresh, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->master, m->wbf, m->wbfT,
                       m->grad);
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
        hipLaunchKernelGGL(k_gemm, dim3(np / 64, H / 64, 1), dim3(256), 0, st, a[l & 1], H, wbf + offW[l], H, H,
                           theta + offB[l], z, a[(l + 1) & 1], H, np);
    hipLaunchKernelGGL(k_layer5, dim3((n * NOUT + 255) / 256), dim3(256), 0, st, a[1], n, wbf, theta, Y);
    return hipGetLastError() == hipSuccess ? PGK_OK : PGK_EDEVICE;
}

extern "C" const char *pgk_mlp_last_error(const pgk_mlp *m) { return m ? m->err.c_str() : "null mlp"; }

extern "C" void pgk_mlp_destroy(pgk_mlp *m) { delete m; }
