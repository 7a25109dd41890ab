// tsat_learned.hip -- gfx950 kernels of the learned proposal: per-variable
// features with signed neighbour aggregation over the occurrence store, and a
// per-variable MLP 16 -> 128 -> 128 -> 1 whose dense layers run on MFMA
// (BF16 operands with FP32 accumulation forward, FP32 operands backward),
// with a deterministic split reduction of the gradient fused with Adam.
//
// The network and its features are not part of the paper: they implement
// the learned initialiser that proposes soft assignments to the
// gradient-based search of Sec. IV-A in place of its N(0,1) start.
#include <hip/hip_runtime.h>

#include "tsat_learned.h"

namespace tsat {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

// One thread per variable walks its occurrence records (positive occurrences
// first, then negative ones; each record lists the other literals of the
// clause in clause order).  Clauses holding a variable and its negation are
// skipped.  Round 0 counts and writes the base features and the channels h0;
// round r (1..3) sums sgn(l_v) sgn(l_u) h_{r-1}[u] over co-literals.
__global__ __launch_bounds__(256) void features_kernel(FeatArgs a)
{
    const int32_t v = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (v >= a.V) return;
    const uint32_t end = a.occ_off[v + 1], mid = a.occ_mid[v];
    const uint32_t pk1 = (uint32_t)(a.pure_k - 1);
    int32_t pos = 0, neg = 0, wsum = 0, z = 0;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t w = a.occ_off[v];
    while (w < end) {
        const bool negv = w >= mid;
        uint32_t km1, base;
        if (a.pure_k) {
            km1 = pk1;
            base = w * pk1;
            w += 1;
        } else {
            km1 = a.occ_data[w];
            base = w + 1;
            w += 1 + km1;
        }
        bool taut = false;
        uint32_t prev_var = 0xffffffffu;
        for (uint32_t j = 0; j < km1; ++j) {
            const uint32_t u = a.occ_data[base + j] >> 1;
            taut |= (u == (uint32_t)v) | (u == prev_var);
            prev_var = u;
        }
        if (taut) continue;
        if (a.round == 0) {
            pos += negv ? 0 : 1;
            neg += negv ? 1 : 0;
            wsum += (int32_t)km1 + 1;
            z += (int32_t)km1;
        } else {
            float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
            for (uint32_t j = 0; j < km1; ++j) {
                const uint32_t c = a.occ_data[base + j];
                const float4 h = a.h_prev[c >> 1];
                if (c & 1u) {
                    s.x -= h.x; s.y -= h.y; s.z -= h.z; s.w -= h.w;
                } else {
                    s.x += h.x; s.y += h.y; s.z += h.z; s.w += h.w;
                }
            }
            if (negv) {
                acc.x -= s.x; acc.y -= s.y; acc.z -= s.z; acc.w -= s.w;
            } else {
                acc.x += s.x; acc.y += s.y; acc.z += s.z; acc.w += s.w;
            }
        }
    }
    float* x = a.X + (int64_t)v * kFeat;
    if (a.round == 0) {
        const int32_t deg = pos + neg;
        const float f0 = log1pf((float)pos), f1 = log1pf((float)neg);
        const float bias = (float)(pos - neg) / (float)(deg > 1 ? deg : 1);
        x[0] = f0;
        x[1] = f1;
        x[2] = bias;
        x[3] = deg > 0 ? (float)wsum / (float)deg * 0.25f : 0.f;
        a.h_next[v] = make_float4(bias, (float)(pos - neg) / sqrtf((float)(deg > 1 ? deg : 1)), f0 - f1, 1.f);
        a.zinv[v] = 1.f / (float)(z > 1 ? z : 1);
    } else {
        const float zi = a.zinv[v];
        const float4 h = make_float4(acc.x * zi, acc.y * zi, acc.z * zi, acc.w * zi);
        a.h_next[v] = h;
        x[4 * a.round + 0] = h.x;
        x[4 * a.round + 1] = h.y;
        x[4 * a.round + 2] = h.z;
        x[4 * a.round + 3] = h.w;
    }
}

hipError_t launch_features(const FeatArgs& a, hipStream_t st)
{
    if (a.V <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((a.V + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MLP helpers
// ---------------------------------------------------------------------------

// round to nearest bfloat16, ties to even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// v_mfma_f32_16x16x16_bf16: A[i][k] from lane i + 16*(k/4), element k%4;
// B[k][j] from lane j + 16*(k/4), element k%4; D[i][j] in lane j + 16*(i/4),
// element i%4.
__device__ __forceinline__ v4f mfma_bf16(uint2 a, uint2 b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, a), __builtin_bit_cast(v4s, b), c, 0,
                                                      0, 0);
}
// v_mfma_f32_16x16x4_f32: A[i][k] from lane i + 16*k, B[k][j] from lane
// j + 16*k, D as above.
__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 slot of W1[f][c] among the layer-1 B operands: column tile c/16,
// lane c%16 + 16*(f/4), element f%4
__device__ __forceinline__ int w1_slot(int f, int c) { return ((c >> 4) * 64 + (c & 15) + 16 * (f >> 2)) * 4 + (f & 3); }
// BF16 slot of W2[k][c] among the layer-2 B operands: k-step k/16, column
// tile c/16, lane c%16 + 16*((k%16)/4), element k%4
__device__ __forceinline__ int w2_slot(int k, int c)
{
    return (((k >> 4) * 8 + (c >> 4)) * 64 + (c & 15) + 16 * ((k & 15) >> 2)) * 4 + (k & 3);
}

__device__ __forceinline__ void write_operand(const MlpDev& d, int e, float p)
{
    if (e < kOffB1) {
        reinterpret_cast<uint16_t*>(d.w1op)[w1_slot(e / kHid, e % kHid)] = (uint16_t)bf16_bits(p);
    } else if (e >= kOffW2 && e < kOffB2) {
        const int k = (e - kOffW2) / kHid, c = (e - kOffW2) % kHid;
        reinterpret_cast<uint16_t*>(d.w2op)[w2_slot(k, c)] = (uint16_t)bf16_bits(p);
    } else if (e >= kOffW3 && e < kOffB3) {
        d.w3q[e - kOffW3] = bf16_value(bf16_bits(p));
    }
}

__global__ void mlp_quantize_kernel(MlpDev d)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kNumParams) write_operand(d, e, d.params[e]);
}

constexpr int kH1S = 136; // BF16 row stride of an h1 tile
constexpr int kDS = 132;  // FP32 row stride of a da tile
constexpr int kXS = 20;   // FP32 row stride of the rounded-input tile
constexpr int kRed = 3 * kHid + 2;

// ---------------------------------------------------------------------------
// MLP forward / backward
// ---------------------------------------------------------------------------

// A block of 4 waves takes 64 rows at a time (16 per wave).  Layer 1 is one
// MFMA per 16-column tile (K = 16); its rounded ReLU output goes through LDS
// into the A layout of layer 2 (8 K-steps x 8 column tiles against the W2
// operands held in LDS); layer 3 is a dot product per row.  With TRAIN, the
// block then forms dLoss/da2 per row and accumulates, over all its rows,
//   dW2 = h1q^T da2   (each wave 2 of the 8 row tiles of dW2, FP32 MFMA),
//   dh1 = da2 W2q^T   (each wave its own 16 rows),
//   dW1 = xq^T da1    (each wave 2 of the 8 column tiles),
// and the bias / w3 gradients, in a fixed order; its sums go to one slot of
// the partial buffer, which mlp_reduce_kernel adds up in block order.
template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_kernel(MlpDev d, const float* __restrict__ X, const float* __restrict__ y,
                                                  const float* __restrict__ wt, int64_t B,
                                                  float* __restrict__ logits, float* __restrict__ probs)
{
    __shared__ uint2 s_w2[8 * 8 * 64];
    __shared__ __align__(16) uint16_t s_h1[4][16 * kH1S];
    __shared__ __align__(16) float s_da[TRAIN ? 4 : 1][TRAIN ? 16 * kDS : 1];
    __shared__ __align__(16) float s_xq[TRAIN ? 64 * kXS : 1];
    __shared__ float s_red[TRAIN ? 4 * kRed : 1];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, r = lane & 15, q = lane >> 4;
    for (int e = tid; e < 8 * 8 * 64; e += 256) s_w2[e] = d.w2op[e];
    uint2 w1[8];
    float b1c[8], b2c[8], w3c[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        w1[n] = d.w1op[n * 64 + lane];
        b1c[n] = d.params[kOffB1 + 16 * n + r];
        b2c[n] = d.params[kOffB2 + 16 * n + r];
        w3c[n] = d.w3q[16 * n + r];
    }
    const float b3 = d.params[kOffB3];
    __syncthreads();

    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    v4f gW2[2][8], gW1[2];
    float gb1[8], gb2[8], gw3[8], gb3 = 0.f, gloss = 0.f;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        gW2[0][n] = zero;
        gW2[1][n] = zero;
        gb1[n] = gb2[n] = gw3[n] = 0.f;
    }
    gW1[0] = gW1[1] = zero;
    const float invB = 1.f / (float)B;
    const int64_t nsuper = (B + 63) / 64;
    uint16_t* h1 = s_h1[wv];
    float* da = s_da[TRAIN ? wv : 0];

    for (int64_t sup = blockIdx.x; sup < nsuper; sup += gridDim.x) {
        const int64_t row0 = sup * 64 + wv * 16;
        const int64_t row = row0 + r;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < B) x = *reinterpret_cast<const float4*>(X + row * kFeat + 4 * q);
        const uint32_t e0 = bf16_bits(x.x), e1 = bf16_bits(x.y), e2 = bf16_bits(x.z), e3 = bf16_bits(x.w);
        const uint2 ax = make_uint2(e0 | (e1 << 16), e2 | (e3 << 16));
        if (TRAIN)
            *reinterpret_cast<float4*>(&s_xq[(wv * 16 + r) * kXS + 4 * q]) =
                make_float4(bf16_value(e0), bf16_value(e1), bf16_value(e2), bf16_value(e3));
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const v4f c = mfma_bf16(ax, w1[n], zero);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                h1[(4 * q + rr) * kH1S + 16 * n + r] = (uint16_t)bf16_bits(fmaxf(c[rr] + b1c[n], 0.f));
        }
        __syncthreads();
        v4f acc[8];
#pragma unroll
        for (int n = 0; n < 8; ++n) acc[n] = zero;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint2 ah = *reinterpret_cast<const uint2*>(&h1[r * kH1S + 16 * s + 4 * q]);
#pragma unroll
            for (int n = 0; n < 8; ++n) acc[n] = mfma_bf16(ah, s_w2[(s * 8 + n) * 64 + lane], acc[n]);
        }
        float out[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) out[rr] += fmaxf(acc[n][rr] + b2c[n], 0.f) * w3c[n];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            out[rr] += __shfl_xor(out[rr], 1);
            out[rr] += __shfl_xor(out[rr], 2);
            out[rr] += __shfl_xor(out[rr], 4);
            out[rr] += __shfl_xor(out[rr], 8);
            out[rr] += b3;
        }
        if (!TRAIN) {
            if (r == 0) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int64_t ro = row0 + 4 * q + rr;
                    if (ro < B) {
                        if (logits) logits[ro] = out[rr];
                        if (probs) probs[ro] = 1.f / (1.f + expf(-out[rr]));
                    }
                }
            }
            __syncthreads(); // the next iteration rewrites the h1 tiles
            continue;
        }
        // ---- backward ----
        float dout[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t ro = row0 + 4 * q + rr;
            dout[rr] = 0.f;
            if (ro < B) {
                const float yy = y[ro], ww = wt ? wt[ro] : 1.f, z = out[rr];
                dout[rr] = ww * (1.f / (1.f + expf(-z)) - yy) * invB;
                if (r == 0) gloss += ww * (fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - yy * z) * invB;
            }
        }
        if (r == 0) gb3 += (dout[0] + dout[1]) + (dout[2] + dout[3]);
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const float a2 = acc[n][rr] + b2c[n];
                const float g = a2 > 0.f ? dout[rr] * w3c[n] : 0.f;
                da[(4 * q + rr) * kDS + 16 * n + r] = g;
                gb2[n] += g;
                gw3[n] += fmaxf(a2, 0.f) * dout[rr];
            }
        __syncthreads();
        // dW2 row tiles 2*wv and 2*wv+1 over the 64 rows
        for (int t = 0; t < 16; ++t) {
            const int rw = 4 * t + q, sw = rw >> 4, lr = rw & 15;
            const float ha0 = bf16_value(s_h1[sw][lr * kH1S + 16 * (2 * wv) + r]);
            const float ha1 = bf16_value(s_h1[sw][lr * kH1S + 16 * (2 * wv + 1) + r]);
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                const float db = s_da[TRAIN ? sw : 0][lr * kDS + 16 * n + r];
                gW2[0][n] = mfma_f32(ha0, db, gW2[0][n]);
                gW2[1][n] = mfma_f32(ha1, db, gW2[1][n]);
            }
        }
        // dh1 of this wave's rows: sum over columns of da2 * W2q
        v4f dh[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) dh[m] = zero;
        const uint16_t* w2e = reinterpret_cast<const uint16_t*>(s_w2);
        for (int t = 0; t < 32; ++t) {
            const int col = 4 * t + q;
            const float aa = da[r * kDS + col];
#pragma unroll
            for (int m = 0; m < 8; ++m) dh[m] = mfma_f32(aa, bf16_value(w2e[w2_slot(16 * m + r, col)]), dh[m]);
        }
        __syncthreads(); // every wave is done with the da2 tiles
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int kk = 16 * m + r;
                const float g = bf16_value(h1[(4 * q + rr) * kH1S + kk]) > 0.f ? dh[m][rr] : 0.f;
                da[(4 * q + rr) * kDS + kk] = g;
                gb1[m] += g;
            }
        __syncthreads();
        // dW1 column tiles 2*wv and 2*wv+1 over the 64 rows
        for (int t = 0; t < 16; ++t) {
            const int rw = 4 * t + q, sw = rw >> 4, lr = rw & 15;
            const float xa = s_xq[rw * kXS + r];
#pragma unroll
            for (int mm = 0; mm < 2; ++mm)
                gW1[mm] = mfma_f32(xa, s_da[TRAIN ? sw : 0][lr * kDS + 16 * (2 * wv + mm) + r], gW1[mm]);
        }
        __syncthreads(); // the next super-tile rewrites every tile
    }
    if (!TRAIN) return;

    float* P = d.partial + (int64_t)blockIdx.x * kPartialStride;
#pragma unroll
    for (int mm = 0; mm < 2; ++mm) {
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                P[kOffW2 + (16 * (2 * wv + mm) + 4 * q + rr) * kHid + 16 * n + r] = gW2[mm][n][rr];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) P[kOffW1 + (4 * q + rr) * kHid + 16 * (2 * wv + mm) + r] = gW1[mm][rr];
    }
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        gb1[n] += __shfl_xor(gb1[n], 16);
        gb1[n] += __shfl_xor(gb1[n], 32);
        gb2[n] += __shfl_xor(gb2[n], 16);
        gb2[n] += __shfl_xor(gb2[n], 32);
        gw3[n] += __shfl_xor(gw3[n], 16);
        gw3[n] += __shfl_xor(gw3[n], 32);
    }
    gb3 += __shfl_xor(gb3, 16);
    gb3 += __shfl_xor(gb3, 32);
    gloss += __shfl_xor(gloss, 16);
    gloss += __shfl_xor(gloss, 32);
    if (q == 0) {
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            s_red[wv * kRed + 16 * n + r] = gb1[n];
            s_red[wv * kRed + kHid + 16 * n + r] = gb2[n];
            s_red[wv * kRed + 2 * kHid + 16 * n + r] = gw3[n];
        }
    }
    if (lane == 0) {
        s_red[wv * kRed + 3 * kHid] = gb3;
        s_red[wv * kRed + 3 * kHid + 1] = gloss;
    }
    __syncthreads();
    for (int e = tid; e < kRed; e += 256) {
        const float sum = ((s_red[e] + s_red[kRed + e]) + s_red[2 * kRed + e]) + s_red[3 * kRed + e];
        int dst;
        if (e < kHid) dst = kOffB1 + e;
        else if (e < 2 * kHid) dst = kOffB2 + e - kHid;
        else if (e < 3 * kHid) dst = kOffW3 + e - 2 * kHid;
        else if (e == 3 * kHid) dst = kOffB3;
        else dst = kNumParams; // loss
        P[dst] = sum;
    }
}

__global__ void mlp_reduce_kernel(MlpDev d, int blocks, int adam, float lr, float beta1, float beta2, float eps,
                                  float bc1, float bc2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > kNumParams) return;
    float g = 0.f;
    for (int b = 0; b < blocks; ++b) g += d.partial[(int64_t)b * kPartialStride + e];
    if (e == kNumParams) {
        *d.loss = g;
        return;
    }
    d.grad[e] = g;
    if (!adam) return;
    const float m = beta1 * d.m[e] + (1.f - beta1) * g;
    const float v = beta2 * d.v[e] + (1.f - beta2) * g * g;
    d.m[e] = m;
    d.v[e] = v;
    const float p = d.params[e] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    d.params[e] = p;
    write_operand(d, e, p);
}

hipError_t launch_mlp_forward(const MlpDev& d, const float* X, int64_t B, float* logits, float* probs,
                              hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    const int64_t nsuper = (B + 63) / 64;
    const int blocks = (int)(nsuper < 768 ? nsuper : 768);
    hipLaunchKernelGGL(mlp_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, d, X, (const float*)nullptr,
                       (const float*)nullptr, B, logits, probs);
    return hipGetLastError();
}

int mlp_train_blocks(int64_t B)
{
    const int64_t nsuper = (B + 63) / 64;
    return (int)(nsuper < 256 ? (nsuper > 0 ? nsuper : 1) : 256);
}

hipError_t launch_mlp_backward(const MlpDev& d, const float* X, const float* y, const float* w, int64_t B,
                               hipStream_t st)
{
    hipLaunchKernelGGL(mlp_kernel<true>, dim3((unsigned)mlp_train_blocks(B)), dim3(256), 0, st, d, X, y, w, B,
                       (float*)nullptr, (float*)nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const MlpDev& d, int blocks, int adam, float lr, float beta1, float beta2, float eps,
                             float bc1, float bc2, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNumParams + 1 + 255) / 256), dim3(256), 0, st, d, blocks, adam, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_quantize(const MlpDev& d, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_quantize_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, st, d);
    return hipGetLastError();
}

} // namespace tsat
