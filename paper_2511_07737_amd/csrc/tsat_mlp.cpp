// tsat_mlp.cpp -- host side of the learned-proposal network: parameter and
// optimizer buffers, and the entry points of tsat.h that drive the MLP
// kernels of tsat_learned.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "tsat.h"
#include "tsat_host_util.h"
#include "tsat_learned.h"

using namespace tsat;
using namespace tsat_host;

namespace {
constexpr int kMaxTrainBlocks = 256;
constexpr double kBeta1 = 0.9, kBeta2 = 0.999, kEps = 1e-8;
} // namespace

struct tsat_mlp {
    int32_t device = 0;
    DBuf params, m, v, grad, w1op, w2op, w3q, partial, loss;
    int64_t t = 0;
    bool have_grad = false;
    MlpDev view() const
    {
        MlpDev d;
        d.params = params.as<float>();
        d.m = m.as<float>();
        d.v = v.as<float>();
        d.grad = grad.as<float>();
        d.w1op = w1op.as<uint2>();
        d.w2op = w2op.as<uint2>();
        d.w3q = w3q.as<float>();
        d.partial = partial.as<float>();
        d.loss = loss.as<float>();
        return d;
    }
};

namespace tsat {
int32_t mlp_view(::tsat_mlp* m, MlpDev* out, int32_t* device)
{
    if (!m) return fail(TSAT_E_ARG, "network is NULL");
    *out = m->view();
    *device = m->device;
    return TSAT_OK;
}
} // namespace tsat

static int32_t mlp_dev(tsat_mlp* m)
{
    if (!m) return fail(TSAT_E_ARG, "network is NULL");
    HIPCHK(hipSetDevice(m->device));
    return TSAT_OK;
}

static bool finite_all(const float* p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

static int32_t upload_params(tsat_mlp* m, const float* params)
{
    if (!params) return fail(TSAT_E_ARG, "params is NULL");
    if (!finite_all(params, kNumParams)) return fail(TSAT_E_ARG, "params hold a NaN or Inf");
    HIPCHK(hipMemcpy(m->params.p, params, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(m->m.p, 0, sizeof(float) * kNumParams));
    HIPCHK(hipMemset(m->v.p, 0, sizeof(float) * kNumParams));
    HIPCHK(launch_mlp_quantize(m->view(), nullptr));
    HIPCHK(hipDeviceSynchronize());
    m->t = 0;
    m->have_grad = false;
    return TSAT_OK;
}

extern "C" {

int32_t tsat_mlp_create(int32_t device, const float* params, tsat_mlp** out)
{
    g_err.clear();
    if (!out) return fail(TSAT_E_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(TSAT_E_HIP, "no HIP device available");
    }
    if (device < 0 || device >= count) return fail(TSAT_E_ARG, "device %d out of range (%d devices)", device, count);
    tsat_mlp* m = new (std::nothrow) tsat_mlp();
    if (!m) return fail(TSAT_E_OOM, "host allocation failed");
    m->device = device;
    int32_t rc = mlp_dev(m);
    const size_t np = sizeof(float) * kNumParams;
    if (rc == TSAT_OK) rc = m->params.alloc(np, "network parameters");
    if (rc == TSAT_OK) rc = m->m.alloc(np, "Adam moments");
    if (rc == TSAT_OK) rc = m->v.alloc(np, "Adam moments");
    if (rc == TSAT_OK) rc = m->grad.alloc(np, "network gradient");
    if (rc == TSAT_OK) rc = m->w1op.alloc(8 * 64 * sizeof(uint2), "layer-1 operands");
    if (rc == TSAT_OK) rc = m->w2op.alloc(8 * 8 * 64 * sizeof(uint2), "layer-2 operands");
    if (rc == TSAT_OK) rc = m->w3q.alloc(kHid * sizeof(float), "layer-3 operands");
    if (rc == TSAT_OK) rc = m->partial.alloc((size_t)kMaxTrainBlocks * kPartialStride * sizeof(float), "gradient partials");
    if (rc == TSAT_OK) rc = m->loss.alloc(sizeof(float), "loss");
    if (rc == TSAT_OK) rc = upload_params(m, params);
    if (rc != TSAT_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return TSAT_OK;
}

void tsat_mlp_destroy(tsat_mlp* m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    delete m;
}

int32_t tsat_mlp_set_params(tsat_mlp* m, const float* params)
{
    g_err.clear();
    RET(mlp_dev(m));
    HIPCHK(hipDeviceSynchronize());
    return upload_params(m, params);
}

int32_t tsat_mlp_get_params(tsat_mlp* m, float* params)
{
    g_err.clear();
    RET(mlp_dev(m));
    if (!params) return fail(TSAT_E_ARG, "params is NULL");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(params, m->params.p, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
    return TSAT_OK;
}

int32_t tsat_mlp_get_grad(tsat_mlp* m, float* grad, float* loss)
{
    g_err.clear();
    RET(mlp_dev(m));
    if (!m->have_grad) return fail(TSAT_E_STATE, "no train step yet");
    HIPCHK(hipDeviceSynchronize());
    if (grad) HIPCHK(hipMemcpy(grad, m->grad.p, sizeof(float) * kNumParams, hipMemcpyDeviceToHost));
    if (loss) HIPCHK(hipMemcpy(loss, m->loss.p, sizeof(float), hipMemcpyDeviceToHost));
    return TSAT_OK;
}

int64_t tsat_mlp_step_count(const tsat_mlp* m) { return m ? m->t : 0; }

int32_t tsat_mlp_forward_dev(tsat_mlp* m, const float* X, int64_t B, float* logits, float* probs, void* stream)
{
    g_err.clear();
    RET(mlp_dev(m));
    if (B < 0) return fail(TSAT_E_ARG, "B must be >= 0");
    if (B == 0) return TSAT_OK;
    if (!X || (!logits && !probs)) return fail(TSAT_E_ARG, "X and at least one output are required");
    if (reinterpret_cast<uintptr_t>(X) % 16) return fail(TSAT_E_ARG, "X must be 16-byte aligned");
    HIPCHK(launch_mlp_forward(m->view(), X, B, logits, probs, (hipStream_t)stream));
    return TSAT_OK;
}

int32_t tsat_mlp_train_step_dev(tsat_mlp* m, const float* X, const float* y, const float* w, int64_t B, float lr,
                                void* stream)
{
    g_err.clear();
    RET(mlp_dev(m));
    if (B < 1) return fail(TSAT_E_ARG, "B must be >= 1");
    if (!X || !y) return fail(TSAT_E_ARG, "X and y are required");
    if (reinterpret_cast<uintptr_t>(X) % 16) return fail(TSAT_E_ARG, "X must be 16-byte aligned");
    if (!std::isfinite(lr)) return fail(TSAT_E_ARG, "lr must be finite");
    const hipStream_t st = (hipStream_t)stream;
    const MlpDev d = m->view();
    const int blocks = mlp_train_blocks(B);
    HIPCHK(launch_mlp_backward(d, X, y, w, B, st));
    const bool adam = lr > 0.f;
    const int64_t t = m->t + (adam ? 1 : 0);
    const float bc1 = adam ? (float)(1.0 - std::pow(kBeta1, (double)t)) : 1.f;
    const float bc2 = adam ? (float)(1.0 - std::pow(kBeta2, (double)t)) : 1.f;
    HIPCHK(launch_mlp_reduce(d, blocks, adam ? 1 : 0, lr, (float)kBeta1, (float)kBeta2, (float)kEps, bc1, bc2, st));
    m->t = t;
    m->have_grad = true;
    return TSAT_OK;
}

} // extern "C"
