// Learned warm start: a 12-128-128-3 ReLU multilayer perceptron that predicts
// each contact's impulse at the start of a time step (any initial solution of
// Alg. 1 is admissible, Sect. 5), run and trained with BF16 matrix cores.
//
// Every layer is a product [rows x K] . [K x N] computed with
// v_mfma_f32_16x16x16_bf16 (FP32 accumulation).  Lane l of a wavefront holds,
// for one 16x16x16 step:
//   A (16 rows x 16 k):  row l % 16, k = 4 (l / 16) + e,  e = 0..3
//   B (16 k x 16 cols):  col l % 16, k = 4 (l / 16) + e
//   D (16 x 16, FP32):   col l % 16, row = 4 (l / 16) + e
// Weights are kept as FP32 master copies and repacked after every update into
// BF16 B-fragments (each lane reads its 4 values as one 8-byte load); the
// transposed fragments of W2 and W3 serve the backward products, and
// v_mfma_f32_16x16x32_bf16 A-fragments of W2^T and W3^T (8 values per lane)
// the inference.  Hidden
// activations pass between layers through LDS in BF16.
//
// Weight vector layout (18,563 values): W1[12][128], b1[128], W2[128][128],
// b2[128], W3[128][3], b3[3]; y = x W + b per layer, ReLU after layers 1, 2.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <new>

#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int NF = 12, NH = 128, NO = 3;
constexpr int OFF_W1 = 0, OFF_B1 = NF * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH * NO, NPAR = OFF_B3 + NO;
// fragment tables (in 4-value groups of one lane)
constexpr int F1 = 0;                   // W1:   nt(8) x lane(64) x 4
constexpr int F2 = F1 + 8 * 64 * 4;     // W2:   kt(8) x nt(8) x lane x 4
constexpr int F3 = F2 + 64 * 64 * 4;    // W3:   kt(8) x lane x 4 (cols 3..15 zero)
constexpr int G3 = F3 + 8 * 64 * 4;     // W3^T: nt(8) x lane x 4 (k 3..15 zero)
constexpr int G2 = G3 + 8 * 64 * 4;     // W2^T: kt(8) x nt(8) x lane x 4
constexpr int H2 = G2 + 64 * 64 * 4;    // W2^T as 16x16x32 A-fragments: kt2(4) x mt(8) x lane x 8
constexpr int H3 = H2 + 32 * 64 * 8;    // W3^T as 16x16x32 A-fragments: kt2(4) x lane x 8 (rows 3..15 zero)
constexpr int NFRAG = H3 + 4 * 64 * 8;  // 57,344 BF16 values

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 hbf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 hbf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

__device__ inline f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(hbf16x8, a), __builtin_bit_cast(hbf16x8, b), c,
                                                    0, 0, 0);
}

// Two 4-value fragments side by side: the 8 k-values of one lane of a 16x16x32 operand.
__device__ inline s16x8 cat8(bf16x4 lo, bf16x4 hi) {
    s16x8 r;
    r[0] = lo[0];
    r[1] = lo[1];
    r[2] = lo[2];
    r[3] = lo[3];
    r[4] = hi[0];
    r[5] = hi[1];
    r[6] = hi[2];
    r[7] = hi[3];
    return r;
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// ReLU of four FP32 values rounded to BF16 (round to nearest even, two values
// per conversion instruction); ReLU is taken on the BF16 bit patterns as
// 16-bit integers, where every negative value (and -0) is below 0.
__device__ inline bf16x4 relu_bf16(f32x4 v) {
    const f32x2 lo = {v[0], v[1]}, hi = {v[2], v[3]};
    const s16x2 z = {0, 0};
    const s16x2 a = __builtin_elementwise_max(__builtin_bit_cast(s16x2, __builtin_convertvector(lo, hbf16x2)), z);
    const s16x2 b = __builtin_elementwise_max(__builtin_bit_cast(s16x2, __builtin_convertvector(hi, hbf16x2)), z);
    bf16x4 r;
    r[0] = a[0];
    r[1] = a[1];
    r[2] = b[0];
    r[3] = b[1];
    return r;
}

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ inline unsigned short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ inline bf16x4 frag(const unsigned short *t, int idx4) {
    return *reinterpret_cast<const bf16x4 *>(t + 4 * idx4);
}

__global__ void __launch_bounds__(256) k_pack(const float *w, unsigned short *fr) {
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= NFRAG) return;
    const int e = o & 3, g = o >> 2;
    float v = 0.0f;
    if (o < F2) {  // W1 B-fragments: k = feature, n = hidden
        const int lane = g & 63, nt = g >> 6;
        const int k = 4 * (lane >> 4) + e, n = nt * 16 + (lane & 15);
        v = k < NF ? w[OFF_W1 + k * NH + n] : 0.0f;
    } else if (o < F3) {
        const int h = g - F2 / 4, lane = h & 63, nt = (h >> 6) & 7, kt = h >> 9;
        const int k = kt * 16 + 4 * (lane >> 4) + e, n = nt * 16 + (lane & 15);
        v = w[OFF_W2 + k * NH + n];
    } else if (o < G3) {
        const int h = g - F3 / 4, lane = h & 63, kt = h >> 6;
        const int k = kt * 16 + 4 * (lane >> 4) + e, n = lane & 15;
        v = n < NO ? w[OFF_W3 + k * NO + n] : 0.0f;
    } else if (o < G2) {  // W3^T: k = output, n = hidden
        const int h = g - G3 / 4, lane = h & 63, nt = h >> 6;
        const int k = 4 * (lane >> 4) + e, n = nt * 16 + (lane & 15);
        v = k < NO ? w[OFF_W3 + n * NO + k] : 0.0f;
    } else if (o < H2) {  // W2^T
        const int h = g - G2 / 4, lane = h & 63, nt = (h >> 6) & 7, kt = h >> 9;
        const int k = kt * 16 + 4 * (lane >> 4) + e, n = nt * 16 + (lane & 15);
        v = w[OFF_W2 + n * NH + k];
    } else {
        // 16x16x32 A-fragments of W^T for the transposed inference.  Lane (m = lane % 16, q = lane / 16),
        // element e8 = 0..7 carries the input feature f = 32 kt2 + 4 q + e8 (e8 < 4) or 32 kt2 + 16 + 4 q +
        // e8 - 4 (e8 >= 4): the features that lane holds of two consecutive 16-feature output tiles of the
        // previous layer, so that those tiles form the B operand as they are (the contraction order over k is
        // free as long as A and B use the same one).
        const int h = o < H3 ? o - H2 : o - H3;
        const int e8 = h & 7, lane = (h >> 3) & 63, q = lane >> 4;
        const int fidx = h >> 9;  // fragment: kt2 * 8 + mt (W2), kt2 (W3)
        const int kt2 = o < H3 ? fidx >> 3 : fidx;
        const int f = 32 * kt2 + (e8 < 4 ? 4 * q + e8 : 16 + 4 * q + e8 - 4);
        if (o < H3) {
            const int mt = fidx & 7, m = mt * 16 + (lane & 15);
            v = w[OFF_W2 + f * NH + m];
        } else {
            const int m = lane & 15;
            v = m < NO ? w[OFF_W3 + f * NO + m] : 0.0f;
        }
    }
    fr[o] = to_bf16(v);
}

// Rows of LDS tiles are padded by 4 BF16 values to spread banks.
constexpr int HS = NH + 4;  // hidden row stride
constexpr int XS = 16 + 4;  // feature / output row stride

// Forward of the 16-row tile at LDS rows r0..r0+15 of x (BF16, XS stride):
// h1, h2 (BF16, HS stride) receive the post-ReLU activations, the return
// value the output pre-activation in D layout (cols 0..2 valid).
__device__ inline f32x4 forward_tile(const unsigned short *fr, const float *w, const unsigned short *x,
                                     unsigned short *h1, unsigned short *h2, int r0, int lane) {
    const int r = lane & 15, kq = lane >> 4;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x4 a;
    for (int e = 0; e < 4; ++e) a[e] = (short)x[(r0 + r) * XS + 4 * kq + e];
    for (int nt = 0; nt < 8; ++nt) {
        const f32x4 d = mfma(a, frag(fr, F1 / 4 + nt * 64 + lane), zero);
        const int col = nt * 16 + (lane & 15);
        const float b = w[OFF_B1 + col];
        for (int e = 0; e < 4; ++e) {
            const float v = d[e] + b;
            h1[(r0 + 4 * kq + e) * HS + col] = to_bf16(v > 0.0f ? v : 0.0f);
        }
    }
    __syncthreads();  // every wave of the block calls this in lockstep
    f32x4 acc[8];
    for (int nt = 0; nt < 8; ++nt) acc[nt] = zero;
    for (int kt = 0; kt < 8; ++kt) {
        const bf16x4 a2 = *reinterpret_cast<const bf16x4 *>(h1 + (r0 + r) * HS + kt * 16 + 4 * kq);
        for (int nt = 0; nt < 8; ++nt) acc[nt] = mfma(a2, frag(fr, F2 / 4 + (kt * 8 + nt) * 64 + lane), acc[nt]);
    }
    for (int nt = 0; nt < 8; ++nt) {
        const int col = nt * 16 + (lane & 15);
        const float b = w[OFF_B2 + col];
        for (int e = 0; e < 4; ++e) {
            const float v = acc[nt][e] + b;
            h2[(r0 + 4 * kq + e) * HS + col] = to_bf16(v > 0.0f ? v : 0.0f);
        }
    }
    __syncthreads();
    f32x4 y = zero;
    for (int kt = 0; kt < 8; ++kt) {
        const bf16x4 a3 = *reinterpret_cast<const bf16x4 *>(h2 + (r0 + r) * HS + kt * 16 + 4 * kq);
        y = mfma(a3, frag(fr, F3 / 4 + kt * 64 + lane), y);
    }
    return y;
}

// Inference: y[n][3] = MLP(x[n][12]), computed transposed, H^T = W^T X^T:
// the weights are the A operand and a wave's 16 rows the B operand.  The D
// layout of one layer (column = row of the batch, row = feature) is the B
// layout of the next, so activations stay in registers.  Layer 1 (K = 12,
// padded to 16) uses 16x16x16 products, whose A-fragment of W^T is the packed
// B-fragment of W (same lane layout); layers 2 and 3 use the double-rate
// 16x16x32 products with their own fragment tables.  Each wave keeps all
// weight fragments in registers while it walks its 16-row tiles.
__global__ void __launch_bounds__(256) k_forward(const unsigned short *fr, const float *w, const float *x, int64_t n,
                                                 float *y) {
    __shared__ __align__(16) float bias[2 * NH + 16];
    for (int q = threadIdx.x; q < 2 * NH + 16; q += 256)
        bias[q] = q < NH ? w[OFF_B1 + q] : q < 2 * NH ? w[OFF_B2 + q - NH] : (q - 2 * NH < NO ? w[OFF_B3 + q - 2 * NH] : 0.0f);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    bf16x4 a1[8];
    s16x8 a2[32], a3[4];
#pragma unroll
    for (int t = 0; t < 8; ++t) a1[t] = frag(fr, F1 / 4 + t * 64 + lane);
#pragma unroll
    for (int t = 0; t < 32; ++t) a2[t] = *reinterpret_cast<const s16x8 *>(fr + H2 + 8 * (t * 64 + lane));
#pragma unroll
    for (int t = 0; t < 4; ++t) a3[t] = *reinterpret_cast<const s16x8 *>(fr + H3 + 8 * (t * 64 + lane));
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t tiles = (n + 15) / 16;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    // the inputs of the B fragment of x^T for tile t (column = row t*16 + col, k = feature 4 kq + e, 16-byte
    // aligned), zero past the end; converted to BF16 only when used, so the load of the next tile stays in flight
    auto load_x = [&](int64_t t) {
        const int64_t row = t * 16 + col;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (row < n && 4 * kq < NF) v = *reinterpret_cast<const float4 *>(x + row * NF + 4 * kq);
        return v;
    };
    int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    float4 xr = load_x(t), xr1 = load_x(t + nwaves);
    for (; t < tiles; t += nwaves) {
        const int64_t row = t * 16 + col;
        const float4 xn = load_x(t + 2 * nwaves);  // rows two tiles ahead load while this one computes
        bf16x4 xb;
        xb[0] = (short)to_bf16(xr.x);
        xb[1] = (short)to_bf16(xr.y);
        xb[2] = (short)to_bf16(xr.z);
        xb[3] = (short)to_bf16(xr.w);
        // the accumulators start at the bias of their four output features (D rows 4 kq .. 4 kq + 3)
        bf16x4 h1[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
            h1[mt] = relu_bf16(mfma(a1[mt], xb, *reinterpret_cast<const f32x4 *>(bias + mt * 16 + 4 * kq)));
        f32x4 acc[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt] = *reinterpret_cast<const f32x4 *>(bias + NH + mt * 16 + 4 * kq);
#pragma unroll
        for (int kt2 = 0; kt2 < 4; ++kt2) {
            const s16x8 b = cat8(h1[2 * kt2], h1[2 * kt2 + 1]);
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) acc[mt] = mfma32(a2[kt2 * 8 + mt], b, acc[mt]);
        }
        bf16x4 h2[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) h2[mt] = relu_bf16(acc[mt]);
        f32x4 yo = *reinterpret_cast<const f32x4 *>(bias + 2 * NH + 4 * kq), yo2 = zero;  // two chains
#pragma unroll
        for (int kt2 = 0; kt2 < 4; kt2 += 2) {
            yo = mfma32(a3[kt2], cat8(h2[2 * kt2], h2[2 * kt2 + 1]), yo);
            yo2 = mfma32(a3[kt2 + 1], cat8(h2[2 * kt2 + 2], h2[2 * kt2 + 3]), yo2);
        }
        yo = yo + yo2;
        if (kq == 0 && row < n)
#pragma unroll
            for (int e = 0; e < NO; ++e) y[row * NO + e] = yo[e];
        xr = xr1;
        xr1 = xn;
    }
}

// Gradient of L = 1/(2B) sum |y - t|^2 over the minibatch idx[off .. off+bsz)
// (idx may be NULL: identity).  Block b writes its partial gradient to
// part[b][NPAR] and its partial sum of squared errors to lpart[b].
__global__ void __launch_bounds__(256) k_grad(const unsigned short *fr, const float *w, const float *x, const float *t,
                                              const int32_t *idx, int64_t off, int64_t bsz, float *part,
                                              float *lpart) {
    __shared__ unsigned short xs[64 * XS];
    __shared__ unsigned short h1[64 * HS];
    __shared__ unsigned short h2[64 * HS];
    __shared__ unsigned short dy[64 * XS];
    __shared__ unsigned short g2[64 * HS];
    __shared__ unsigned short g1[64 * HS];
    __shared__ float lred[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tid = threadIdx.x;
    const int r = lane & 15, kq = lane >> 4;
    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 aw2[16], aw1[2], aw3[2];
    for (int q = 0; q < 16; ++q) aw2[q] = zero;
    aw1[0] = aw1[1] = aw3[0] = aw3[1] = zero;
    float db1 = 0.0f, db2 = 0.0f, db3 = 0.0f, loss = 0.0f;
    const float inv_b = 1.0f / (float)bsz;
    const int64_t tiles = (bsz + 63) / 64;
    for (int64_t bt = blockIdx.x; bt < tiles; bt += gridDim.x) {
        for (int q = tid; q < 64 * 16; q += 256) {
            const int row = q >> 4, k = q & 15;
            const int64_t pos = bt * 64 + row;
            float v = 0.0f;
            if (pos < bsz && k < NF) {
                const int64_t s = idx ? (int64_t)idx[off + pos] : off + pos;
                v = x[s * NF + k];
            }
            xs[row * XS + k] = to_bf16(v);
        }
        __syncthreads();
        // forward of this wave's 16 rows; dY = (y - t) / B
        const f32x4 d = forward_tile(fr, w, xs, h1, h2, wave * 16, lane);
        {
            const int col = lane & 15;
            for (int e = 0; e < 4; ++e) {
                const int row = wave * 16 + 4 * kq + e;
                const int64_t pos = bt * 64 + row;
                float g = 0.0f;
                if (col < NO && pos < bsz) {
                    const int64_t s = idx ? (int64_t)idx[off + pos] : off + pos;
                    const float err = d[e] + w[OFF_B3 + col] - t[s * NO + col];
                    loss += err * err;
                    g = err * inv_b;
                }
                dy[row * XS + col] = to_bf16(g);
            }
        }
        __syncthreads();
        // dH2 = (dY W3^T) * [h2 > 0]
        {
            const bf16x4 a = *reinterpret_cast<const bf16x4 *>(dy + (wave * 16 + r) * XS + 4 * kq);
            for (int nt = 0; nt < 8; ++nt) {
                const f32x4 g = mfma(a, frag(fr, G3 / 4 + nt * 64 + lane), zero);
                const int col = nt * 16 + (lane & 15);
                for (int e = 0; e < 4; ++e) {
                    const int row = wave * 16 + 4 * kq + e;
                    g2[row * HS + col] = h2[row * HS + col] != 0 ? to_bf16(g[e]) : (unsigned short)0;
                }
            }
        }
        __syncthreads();
        // dH1 = (dH2 W2^T) * [h1 > 0]
        {
            f32x4 acc[8];
            for (int nt = 0; nt < 8; ++nt) acc[nt] = zero;
            for (int kt = 0; kt < 8; ++kt) {
                const bf16x4 a = *reinterpret_cast<const bf16x4 *>(g2 + (wave * 16 + r) * HS + kt * 16 + 4 * kq);
                for (int nt = 0; nt < 8; ++nt)
                    acc[nt] = mfma(a, frag(fr, G2 / 4 + (kt * 8 + nt) * 64 + lane), acc[nt]);
            }
            for (int nt = 0; nt < 8; ++nt) {
                const int col = nt * 16 + (lane & 15);
                for (int e = 0; e < 4; ++e) {
                    const int row = wave * 16 + 4 * kq + e;
                    g1[row * HS + col] = h1[row * HS + col] != 0 ? to_bf16(acc[nt][e]) : (unsigned short)0;
                }
            }
        }
        __syncthreads();
        // weight gradients over the 64 rows (K = samples, 4 steps of 16); wave w owns fixed output tiles
        for (int kt = 0; kt < 4; ++kt) {
            const int s0 = kt * 16 + 4 * kq;
            // dW2 = H1^T dH2: tiles (mt = 2w, 2w+1) x (nt = 0..7)
            for (int m = 0; m < 2; ++m) {
                const int i = (2 * wave + m) * 16 + r;
                bf16x4 a;
                for (int e = 0; e < 4; ++e) a[e] = (short)h1[(s0 + e) * HS + i];
                for (int nt = 0; nt < 8; ++nt) {
                    bf16x4 b;
                    for (int e = 0; e < 4; ++e) b[e] = (short)g2[(s0 + e) * HS + nt * 16 + r];
                    aw2[m * 8 + nt] = mfma(a, b, aw2[m * 8 + nt]);
                }
            }
            // dW3 = H2^T dY: tiles mt = 2w, 2w+1
            {
                bf16x4 b;
                for (int e = 0; e < 4; ++e) b[e] = (short)dy[(s0 + e) * XS + r];
                for (int m = 0; m < 2; ++m) {
                    const int i = (2 * wave + m) * 16 + r;
                    bf16x4 a;
                    for (int e = 0; e < 4; ++e) a[e] = (short)h2[(s0 + e) * HS + i];
                    aw3[m] = mfma(a, b, aw3[m]);
                }
            }
            // dW1 = X^T dH1: tiles nt = 2w, 2w+1
            {
                bf16x4 a;
                for (int e = 0; e < 4; ++e) a[e] = (short)xs[(s0 + e) * XS + r];
                for (int m = 0; m < 2; ++m) {
                    const int nt = 2 * wave + m;
                    bf16x4 b;
                    for (int e = 0; e < 4; ++e) b[e] = (short)g1[(s0 + e) * HS + nt * 16 + r];
                    aw1[m] = mfma(a, b, aw1[m]);
                }
            }
        }
        // bias gradients: column sums in row order
        if (tid < NH) {
            float s1 = 0.0f, s2 = 0.0f;
            for (int row = 0; row < 64; ++row) {
                s1 += from_bf16(g1[row * HS + tid]);
                s2 += from_bf16(g2[row * HS + tid]);
            }
            db1 += s1;
            db2 += s2;
        } else if (tid < NH + NO) {
            float s3 = 0.0f;
            for (int row = 0; row < 64; ++row) s3 += from_bf16(dy[row * XS + (tid - NH)]);
            db3 += s3;
        }
        __syncthreads();
    }
    float *pg = part + (int64_t)blockIdx.x * NPAR;
    for (int m = 0; m < 2; ++m)
        for (int nt = 0; nt < 8; ++nt) {
            const int j = nt * 16 + r;
            for (int e = 0; e < 4; ++e) {
                const int i = (2 * wave + m) * 16 + 4 * kq + e;
                pg[OFF_W2 + i * NH + j] = aw2[m * 8 + nt][e];
            }
        }
    for (int m = 0; m < 2; ++m) {
        for (int e = 0; e < 4; ++e) {
            const int i = (2 * wave + m) * 16 + 4 * kq + e;
            if (r < NO) pg[OFF_W3 + i * NO + r] = aw3[m][e];
            const int f = 4 * kq + e, j = (2 * wave + m) * 16 + r;
            if (f < NF) pg[OFF_W1 + f * NH + j] = aw1[m][e];
        }
    }
    if (tid < NH) {
        pg[OFF_B1 + tid] = db1;
        pg[OFF_B2 + tid] = db2;
    } else if (tid < NH + NO) {
        pg[OFF_B3 + tid - NH] = db3;
    }
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (lane == 0) lred[wave] = loss;
    __syncthreads();
    if (tid == 0) lpart[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
}

// Sum of the per-block partials in block order (deterministic).
__global__ void __launch_bounds__(256) k_reduce(const float *part, int nblocks, float *grad) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPAR) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * NPAR + p];
    grad[p] = s;
}

__global__ void __launch_bounds__(256) k_adam(float *w, const float *g, float *m, float *v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPAR) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] = w[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace

int mlp_param_count() { return NPAR; }
int mlp_frag_count() { return NFRAG; }
int mlp_grad_blocks(int64_t bsz) {
    const int64_t tiles = (bsz + 63) / 64;
    return (int)std::min<int64_t>(tiles, 1024);
}

nbgs_status launch_mlp_pack(const float *w, unsigned short *fr, hipStream_t s) {
    k_pack<<<(NFRAG + 255) / 256, 256, 0, s>>>(w, fr);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_mlp_forward(const unsigned short *fr, const float *w, const float *x, int64_t n, float *y,
                               hipStream_t s) {
    if (n <= 0) return NBGS_OK;
    // one block of four waves per CU (the weight fragments fill the register file), each wave walking many
    // 16-row tiles
    const int64_t tiles = (n + 63) / 64;
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, cus);
    k_forward<<<grid, 256, 0, s>>>(fr, w, x, n, y);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_mlp_grad(const unsigned short *fr, const float *w, const float *x, const float *t,
                            const int32_t *idx, int64_t off, int64_t bsz, float *part, float *lpart, float *grad,
                            hipStream_t s) {
    const int nb = mlp_grad_blocks(bsz);
    k_grad<<<nb, 256, 0, s>>>(fr, w, x, t, idx, off, bsz, part, lpart);
    NBGS_HIP(hipGetLastError());
    k_reduce<<<(NPAR + 255) / 256, 256, 0, s>>>(part, nb, grad);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_mlp_adam(float *w, const float *g, float *m, float *v, int64_t step, float lr, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    k_adam<<<(NPAR + 255) / 256, 256, 0, s>>>(w, g, m, v, lr, b1, b2, eps, c1, c2);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

}  // namespace nbgs

// ------------------------------------------------------------------ C ABI

struct nbgs_mlp_s {
    // device memory of the network (the caller's workspace); first, so that it outlives every buffer carved from it
    nbgs::Arena arena;
    hipStream_t s = nullptr;
    nbgs::DevBuf<float> w, m, v, grad, part, lpart;
    nbgs::DevBuf<unsigned short> fr;
    nbgs::DevBuf<int32_t> idx;
    // training pairs collected from solved steps (nbgs_mlp_collect): features [max_samples x 12], targets [x 3]
    nbgs::DevBuf<float> store_feat, store_tgt;
    int64_t max_samples = 0, n_stored = 0;
    int64_t step = 0;
    float *host = nullptr;  // pinned staging
};

using namespace nbgs;

namespace nbgs {
const unsigned short *mlp_frag_ptr(nbgs_mlp_t mlp) { return mlp->fr.p; }
const float *mlp_weight_ptr(nbgs_mlp_t mlp) { return mlp->w.p; }

// Upper bound of a network's device memory (nbgs_mlp_workspace_query): the
// weights, Adam moments, gradient and packed BF16 fragments, the per-block
// gradient partials of up to 1,024 blocks (76 MB), and per training sample
// its shuffled index and its collected features and targets (64 B); ten per
// cent for alignment.
size_t mlp_workspace_bytes(int64_t max_samples) {
    const double fixed = 4.0 * NPAR * 4.0 + 2.0 * NFRAG + 1025.0 * NPAR * 4.0 + 1024.0 * 4.0 + 1024.0 * 1024.0;
    const size_t b = (size_t)(1.1 * (fixed + 64.0 * (double)max_samples));
    return (b + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1);
}

// Room for n more collected samples (CAPACITY past max_samples): where they go.
nbgs_status mlp_store_slot(nbgs_mlp_t mlp, int64_t n, float **feat, float **tgt) {
    if (mlp->n_stored + n > mlp->max_samples) {
        set_error("%lld more samples do not fit into the %lld the network's store holds (%lld taken)", (long long)n,
                  (long long)mlp->max_samples, (long long)mlp->n_stored);
        return NBGS_ERR_CAPACITY;
    }
    ArenaScope arena_scope(&mlp->arena);
    NBGS_TRY(mlp->store_feat.reserve(12 * (size_t)(mlp->max_samples > 0 ? mlp->max_samples : 1), 1.0));
    NBGS_TRY(mlp->store_tgt.reserve(3 * (size_t)(mlp->max_samples > 0 ? mlp->max_samples : 1), 1.0));
    *feat = mlp->store_feat.p + 12 * mlp->n_stored;
    *tgt = mlp->store_tgt.p + 3 * mlp->n_stored;
    return NBGS_OK;
}

void mlp_store_commit(nbgs_mlp_t mlp, int64_t n) { mlp->n_stored += n; }
}  // namespace nbgs

// Scratch of nbgs_mlp_loss_grad_static: the per-block gradient partials and
// loss partials of at most kStaticGradBlocks blocks of 64 samples (4.75 MB),
// a copy on every GPU the library runs on, held until the process ends.  In
// host code the array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr).
constexpr int kStaticGradBlocks = 64;
constexpr int64_t kStaticMaxSamples = (int64_t)kStaticGradBlocks * 64;
constexpr size_t kScratchFloats = (size_t)kStaticGradBlocks * NPAR + kStaticGradBlocks;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<float *> g_scratch_dev[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's copy of the scratch array.
nbgs_status scratch_ptr(float **out) {
    int dev = 0;
    NBGS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d: the static scratch is kept for devices 0 .. %d", dev, kMaxDevices - 1);
        return NBGS_ERR_DEVICE;
    }
    float *p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_dev[dev].load(std::memory_order_acquire);
        if (!p) {
            void *q = nullptr;
            const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !q) {
                set_error("hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                          hipGetErrorString(e));
                return NBGS_ERR_DEVICE;
            }
            p = static_cast<float *>(q);
            g_scratch_dev[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return NBGS_OK;
}

}  // namespace

// A NULL network is refused; its arena takes the buffers allocated until the
// entry point returns.
#define NBGS_MGUARD(mlp)                                                                                        \
    if (!(mlp)) {                                                                                               \
        set_error("network handle is NULL");                                                                    \
        return NBGS_ERR_INVALID_ARG;                                                                            \
    }                                                                                                           \
    ArenaScope arena_scope_(&(mlp)->arena)

namespace {

// Deterministic initial weights: uniform in +-sqrt(6 / fan_in) for the two
// hidden layers (He uniform), +-sqrt(6 / fan_in) / 10 for the output layer,
// zero biases; the uniform numbers come from splitmix64(seed + index).
void init_weights(uint64_t seed, std::vector<float> &w) {
    w.assign(NPAR, 0.0f);
    auto uni = [&](int64_t i) {
        uint64_t z = seed + (uint64_t)i * 0x9e3779b97f4a7c15ull + 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z = z ^ (z >> 31);
        return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    };
    for (int i = 0; i < NF * NH; ++i) w[OFF_W1 + i] = (float)(uni(OFF_W1 + i) * std::sqrt(6.0 / NF));
    for (int i = 0; i < NH * NH; ++i) w[OFF_W2 + i] = (float)(uni(OFF_W2 + i) * std::sqrt(6.0 / NH));
    for (int i = 0; i < NH * NO; ++i) w[OFF_W3 + i] = (float)(uni(OFF_W3 + i) * std::sqrt(6.0 / NH) * 0.1);
}

nbgs_status upload(nbgs_mlp_t mlp, const float *host_w) {
    NBGS_HIP(hipMemcpyAsync(mlp->w.p, host_w, sizeof(float) * NPAR, hipMemcpyHostToDevice, mlp->s));
    NBGS_HIP(hipMemsetAsync(mlp->m.p, 0, sizeof(float) * NPAR, mlp->s));
    NBGS_HIP(hipMemsetAsync(mlp->v.p, 0, sizeof(float) * NPAR, mlp->s));
    mlp->step = 0;
    NBGS_TRY(launch_mlp_pack(mlp->w.p, mlp->fr.p, mlp->s));
    NBGS_HIP(hipStreamSynchronize(mlp->s));
    return NBGS_OK;
}

}  // namespace

extern "C" {

nbgs_status nbgs_mlp_workspace_query(int64_t max_samples, size_t *bytes) {
    if (!bytes || max_samples < 0) {
        set_error("bad arguments to nbgs_mlp_workspace_query");
        return NBGS_ERR_INVALID_ARG;
    }
    *bytes = mlp_workspace_bytes(max_samples);
    return NBGS_OK;
}

nbgs_status nbgs_mlp_create(uint64_t seed, int64_t max_samples, void *workspace, size_t workspace_bytes,
                            void *hip_stream, nbgs_mlp_t *out) {
    if (!out || max_samples < 0) {
        set_error("out is NULL or max_samples negative");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    nbgs_mlp_t mlp = new (std::nothrow) nbgs_mlp_s();
    if (!mlp) {
        set_error("host allocation failed");
        return NBGS_ERR_OUT_OF_MEMORY;
    }
    mlp->s = (hipStream_t)hip_stream;
    mlp->max_samples = max_samples;
    mlp->arena.reset(workspace, workspace_bytes);
    if (!mlp->arena.bound()) {
        delete mlp;
        set_error("the workspace is NULL or too small (nbgs_mlp_workspace_query gives its size)");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    nbgs_status st = NBGS_OK;
    for (DevBuf<float> *b : {&mlp->w, &mlp->m, &mlp->v, &mlp->grad})
        if (st == NBGS_OK) st = b->reserve(NPAR, 1.0);
    if (st == NBGS_OK) st = mlp->fr.reserve(NFRAG, 1.0);
    if (st == NBGS_OK && hipHostMalloc((void **)&mlp->host, sizeof(float) * (NPAR + 64)) != hipSuccess) {
        set_error("pinned host allocation failed");
        st = NBGS_ERR_OUT_OF_MEMORY;
    }
    if (st == NBGS_OK) {
        std::vector<float> w;
        init_weights(seed, w);
        std::memcpy(mlp->host, w.data(), sizeof(float) * NPAR);
        st = upload(mlp, mlp->host);
    }
    if (st != NBGS_OK) {
        nbgs_mlp_destroy(mlp);
        return st;
    }
    *out = mlp;
    return NBGS_OK;
}

nbgs_status nbgs_mlp_destroy(nbgs_mlp_t mlp) {
    if (!mlp) return NBGS_OK;
    (void)hipStreamSynchronize(mlp->s);
    if (mlp->host) (void)hipHostFree(mlp->host);
    delete mlp;
    return NBGS_OK;
}

int32_t nbgs_mlp_param_count(void) { return NPAR; }

nbgs_status nbgs_mlp_set_weights(nbgs_mlp_t mlp, const float *w) {
    if (!mlp || !w) {
        set_error("mlp or weights NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    std::memcpy(mlp->host, w, sizeof(float) * NPAR);
    return upload(mlp, mlp->host);
}

nbgs_status nbgs_mlp_get_weights(nbgs_mlp_t mlp, float *w) {
    if (!mlp || !w) {
        set_error("mlp or weights NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    NBGS_HIP(hipMemcpyAsync(mlp->host, mlp->w.p, sizeof(float) * NPAR, hipMemcpyDeviceToHost, mlp->s));
    NBGS_HIP(hipStreamSynchronize(mlp->s));
    std::memcpy(w, mlp->host, sizeof(float) * NPAR);
    return NBGS_OK;
}

nbgs_status nbgs_mlp_forward(nbgs_mlp_t mlp, const float *feat, int64_t n, float *out) {
    if (!mlp || n < 0 || (n > 0 && (!feat || !out))) {
        set_error("bad arguments to nbgs_mlp_forward");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    if (reinterpret_cast<uintptr_t>(feat) % 16 != 0) {
        set_error("nbgs_mlp_forward needs 16-byte aligned features");
        return NBGS_ERR_INVALID_ARG;
    }
    return launch_mlp_forward(mlp->fr.p, mlp->w.p, feat, n, out, mlp->s);
}

nbgs_status nbgs_mlp_loss_grad(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n, float *grad,
                               double *loss) {
    if (!mlp || n < 1 || !feat || !target) {
        set_error("bad arguments to nbgs_mlp_loss_grad");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    const int nb = mlp_grad_blocks(n);
    NBGS_TRY(mlp->part.reserve((size_t)nb * NPAR));
    NBGS_TRY(mlp->lpart.reserve((size_t)nb));
    NBGS_TRY(launch_mlp_grad(mlp->fr.p, mlp->w.p, feat, target, nullptr, 0, n, mlp->part.p, mlp->lpart.p,
                             grad ? grad : mlp->grad.p, mlp->s));
    if (loss) {
        std::vector<float> lp(nb);
        NBGS_HIP(hipMemcpyAsync(mlp->host, mlp->lpart.p, sizeof(float) * std::min(nb, 64), hipMemcpyDeviceToHost,
                                mlp->s));
        NBGS_HIP(hipStreamSynchronize(mlp->s));
        if (nb > 64) NBGS_HIP(hipMemcpy(lp.data(), mlp->lpart.p, sizeof(float) * nb, hipMemcpyDeviceToHost));
        else std::memcpy(lp.data(), mlp->host, sizeof(float) * nb);
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += lp[b];
        *loss = s / (2.0 * (double)n);
    }
    return NBGS_OK;
}

nbgs_status nbgs_mlp_loss_grad_static(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n,
                                      float *grad, double *loss) {
    if (!mlp || n < 1 || !feat || !target || !grad) {
        set_error("bad arguments to nbgs_mlp_loss_grad_static");
        return NBGS_ERR_INVALID_ARG;
    }
    if (n > kStaticMaxSamples) {
        set_error("%lld samples: nbgs_mlp_loss_grad_static takes at most %lld (its static scratch holds the partial "
                  "sums of %d blocks of 64)", (long long)n, (long long)kStaticMaxSamples, kStaticGradBlocks);
        return NBGS_ERR_INVALID_ARG;
    }
    float *scr = nullptr;
    NBGS_TRY(scratch_ptr(&scr));
    const int nb = mlp_grad_blocks(n);  // at most kStaticGradBlocks here; every block writes its partials whole
    float *part = scr, *lpart = scr + (size_t)kStaticGradBlocks * NPAR;
    NBGS_TRY(launch_mlp_grad(mlp->fr.p, mlp->w.p, feat, target, nullptr, 0, n, part, lpart, grad, mlp->s));
    if (loss) {
        NBGS_HIP(hipMemcpyAsync(mlp->host, lpart, sizeof(float) * nb, hipMemcpyDeviceToHost, mlp->s));
        NBGS_HIP(hipStreamSynchronize(mlp->s));
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += mlp->host[b];
        *loss = s / (2.0 * (double)n);
    }
    return NBGS_OK;
}

nbgs_status nbgs_mlp_train(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n, int32_t epochs,
                           int32_t batch, float lr, uint64_t shuffle_seed, double *final_loss) {
    if (!mlp || n < 1 || !feat || !target || epochs < 1 || batch < 1 || !(lr > 0.0f)) {
        set_error("bad arguments to nbgs_mlp_train");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&mlp->arena);
    const int64_t bsz_max = std::min<int64_t>(batch, n);
    const int nb = mlp_grad_blocks(bsz_max);
    NBGS_TRY(mlp->part.reserve((size_t)nb * NPAR));
    NBGS_TRY(mlp->lpart.reserve((size_t)nb));
    NBGS_TRY(mlp->idx.reserve((size_t)n));
    std::vector<int32_t> perm(n);
    double last = 0.0;
    for (int32_t ep = 0; ep < epochs; ++ep) {
        // Fisher-Yates with splitmix64 draws
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        uint64_t st = shuffle_seed + 0x632be59bd9b4e019ull * (uint64_t)(ep + 1);
        for (int64_t i = n - 1; i > 0; --i) {
            st += 0x9e3779b97f4a7c15ull;
            uint64_t z = st;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            z = z ^ (z >> 31);
            const int64_t j = (int64_t)(z % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        NBGS_HIP(hipMemcpyAsync(mlp->idx.p, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, mlp->s));
        NBGS_HIP(hipStreamSynchronize(mlp->s));  // perm is reused next epoch
        double ep_loss = 0.0;
        int64_t ep_count = 0;
        for (int64_t off = 0; off < n; off += bsz_max) {
            const int64_t bsz = std::min<int64_t>(bsz_max, n - off);
            NBGS_TRY(launch_mlp_grad(mlp->fr.p, mlp->w.p, feat, target, mlp->idx.p, off, bsz, mlp->part.p,
                                     mlp->lpart.p, mlp->grad.p, mlp->s));
            NBGS_TRY(launch_mlp_adam(mlp->w.p, mlp->grad.p, mlp->m.p, mlp->v.p, ++mlp->step, lr, mlp->s));
            NBGS_TRY(launch_mlp_pack(mlp->w.p, mlp->fr.p, mlp->s));
            if (ep == epochs - 1) {
                const int nbl = mlp_grad_blocks(bsz);
                std::vector<float> lp(nbl);
                NBGS_HIP(hipMemcpyAsync(lp.data(), mlp->lpart.p, sizeof(float) * nbl, hipMemcpyDeviceToHost, mlp->s));
                NBGS_HIP(hipStreamSynchronize(mlp->s));
                for (int b = 0; b < nbl; ++b) ep_loss += lp[b];
                ep_count += bsz;
            }
        }
        if (ep == epochs - 1) last = ep_loss / (2.0 * (double)ep_count);
    }
    if (final_loss) *final_loss = last;
    NBGS_HIP(hipStreamSynchronize(mlp->s));
    return NBGS_OK;
}

nbgs_status nbgs_mlp_train_collected(nbgs_mlp_t mlp, int32_t epochs, int32_t batch, float lr, uint64_t shuffle_seed,
                                     double *final_loss) {
    NBGS_MGUARD(mlp);
    if (mlp->n_stored < 1) {
        set_error("no samples collected (nbgs_mlp_collect)");
        return NBGS_ERR_STATE;
    }
    return nbgs_mlp_train(mlp, mlp->store_feat.p, mlp->store_tgt.p, mlp->n_stored, epochs, batch, lr, shuffle_seed,
                          final_loss);
}

nbgs_status nbgs_mlp_collected(nbgs_mlp_t mlp, int64_t *n, const float **feat, const float **target) {
    NBGS_MGUARD(mlp);
    if (n) *n = mlp->n_stored;
    if (feat) *feat = mlp->store_feat.p;
    if (target) *target = mlp->store_tgt.p;
    return NBGS_OK;
}

nbgs_status nbgs_mlp_clear_collected(nbgs_mlp_t mlp) {
    NBGS_MGUARD(mlp);
    mlp->n_stored = 0;
    return NBGS_OK;
}

}  // extern "C"
