// tsat_learned.h -- device-side interface of the learned proposal kernels:
// per-variable features over the occurrence store, the per-variable MLP
// (BF16 operands, FP32 accumulation on MFMA) with its backward pass and Adam,
// and the initialisation of a batch from a proposal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsat {

constexpr int kFeat = 16;     // features per variable
constexpr int kHid = 128;     // hidden width of both layers
// flat parameter vector: W1 [16][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kNumParams = kOffB3 + 1; // 18817
constexpr int kPartialStride = kNumParams + 1; // per-block partial gradient + loss

struct FeatArgs {
    int32_t V;
    int32_t pure_k;            // 0: records carry their own (k-1) header
    const uint32_t* occ_off;   // [V+1]
    const uint32_t* occ_mid;   // [V]
    const uint32_t* occ_data;
    const float4* h_prev;      // [V] channels of the previous round (rounds 1..3)
    float4* h_next;            // [V]
    float* zinv;               // [V] 1 / max(1, co-literal count), written by round 0
    float* X;                  // [V][16]
    int32_t round;             // 0: base features and h0; 1..3: aggregation
};

struct MlpDev {
    float* params;     // [kNumParams] FP32 master values
    float* m;          // [kNumParams] Adam first moment
    float* v;          // [kNumParams] Adam second moment
    float* grad;       // [kNumParams] last gradient
    uint2* w1op;       // [8][64] BF16x4 operands of layer 1 (rounded W1)
    uint2* w2op;       // [8][8][64] BF16x4 operands of layer 2 (rounded W2)
    float* w3q;        // [128] rounded w3 as FP32
    float* partial;    // [blocks][kPartialStride]
    float* loss;       // [1]
};

struct PropArgs {
    int32_t V, N;
    uint64_t seed;
    int32_t mode;              // 1: Eq. 5 mean mode (rows kept at positive mean)
    const float* p;            // [V] P(x_v = true)
    float* theta;              // [V][N]
};

hipError_t launch_features(const FeatArgs& a, hipStream_t st);
// forward of B rows: logits[B] (may be NULL) and probabilities sigmoid(logit) (may be NULL)
hipError_t launch_mlp_forward(const MlpDev& d, const float* X, int64_t B, float* logits, float* probs,
                              hipStream_t st);
int mlp_train_blocks(int64_t B);
// weighted BCE gradient of B rows into d.partial (mlp_train_blocks(B) blocks)
hipError_t launch_mlp_backward(const MlpDev& d, const float* X, const float* y, const float* w, int64_t B,
                               hipStream_t st);
// sum the partials into d.grad and d.loss; if adam, one Adam step at 1-based t
// (bias corrections 1 - beta^t passed in) and re-rounding of the operands
hipError_t launch_mlp_reduce(const MlpDev& d, int blocks, int adam, float lr, float beta1, float beta2, float eps,
                             float bc1, float bc2, hipStream_t st);
// re-round the operands from d.params (after the parameters were set)
hipError_t launch_mlp_quantize(const MlpDev& d, hipStream_t st);
hipError_t launch_init_proposal(const PropArgs& a, hipStream_t st);

} // namespace tsat

struct tsat_mlp;
namespace tsat {
// host side: device view and device ordinal of a network handle
int32_t mlp_view(::tsat_mlp* m, MlpDev* out, int32_t* device);
} // namespace tsat
