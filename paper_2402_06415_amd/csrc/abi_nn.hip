// extern "C" entry points of the learned proposal (include/ising_nn.h):
// validation and dispatch.  No device memory is allocated here.
#include <math.h>

#include "abi_common.hpp"
#include "ising_nn.h"
#include "nn.hpp"

namespace {

using ising::abi::aligned256;
using ising::abi::set_error;

int validate(const ising_nn* net) {
    if (!net)
        return set_error(ISING_E_INVALID, "net pointer is NULL");
    if (net->abi_version != ISING_ABI_VERSION)
        return set_error(ISING_E_INVALID, "abi_version %d, library has %d", net->abi_version,
                         ISING_ABI_VERSION);
    if (net->channels != ISING_NN_CHANNELS)
        return set_error(ISING_E_UNSUPPORTED, "channels = %d: the kernels are built for %d",
                         net->channels, ISING_NN_CHANNELS);
    if (net->L < 2 || net->L > ISING_NN_MAX_L)
        return set_error(ISING_E_INVALID, "L = %d outside 2..%d", net->L, ISING_NN_MAX_L);
    if (net->max_batch < 1 || net->max_batch > 65536)
        return set_error(ISING_E_INVALID, "max_batch = %d outside 1..65536", net->max_batch);
    if (!net->master || !net->weights || !net->grad || !net->adam_m || !net->adam_v)
        return set_error(ISING_E_INVALID, "parameter buffers must be non-NULL device pointers");
    if (!net->workspace || !aligned256(net->workspace))
        return set_error(ISING_E_INVALID,
                         "workspace must be a non-NULL 256-byte aligned device pointer");
    return ISING_OK;
}

int check_batch_args(const ising_nn* net, const void* s, int64_t stride, int32_t batch) {
    if (batch < 1 || batch > net->max_batch)
        return set_error(ISING_E_INVALID, "batch = %d outside 1..max_batch (%d)", batch,
                         net->max_batch);
    if (!s)
        return set_error(ISING_E_INVALID, "configuration pointer is NULL");
    if (stride < (int64_t)net->L * net->L)
        return set_error(ISING_E_INVALID, "stride %lld < L*L", (long long)stride);
    return ISING_OK;
}

unsigned char* ws_of(const ising_nn* net) { return reinterpret_cast<unsigned char*>(net->workspace); }

ising::Key key_of(uint64_t seed) {
    return ising::Key{(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
}

}  // namespace

extern "C" {

int32_t ising_nn_param_count(int32_t channels) {
    return channels == ISING_NN_CHANNELS ? ising::nn_param_count() : 0;
}

size_t ising_nn_workspace_bytes(int32_t L, int32_t channels, int32_t max_batch) {
    if (channels != ISING_NN_CHANNELS || L < 2 || L > ISING_NN_MAX_L || max_batch < 1 ||
        max_batch > 65536)
        return 0;
    return ising::nn_ws_layout(L, max_batch).bytes;
}

int ising_nn_round_weights(const ising_nn* net, void* hip_stream) {
    int rc = validate(net);
    if (rc)
        return rc;
    const ising::NNWs lay = ising::nn_ws_layout(net->L, net->max_batch);
    HIP_TRY(ising::launch_nn_round(net->master, net->weights,
                                   reinterpret_cast<float*>(ws_of(net) + lay.wexp),
                                   reinterpret_cast<hipStream_t>(hip_stream)),
            "nn round");
    return ISING_OK;
}

int ising_nn_logq(const ising_nn* net, const int8_t* s_dev, int64_t stride, int32_t batch,
                  int32_t symmetric, float* logq_dev, void* hip_stream) {
    int rc = validate(net);
    if (rc)
        return rc;
    if ((rc = check_batch_args(net, s_dev, stride, batch)))
        return rc;
    if (!logq_dev)
        return set_error(ISING_E_INVALID, "logq_dev is NULL");
    if (symmetric != 0 && symmetric != 1)
        return set_error(ISING_E_INVALID, "symmetric must be 0 or 1");
    const ising::NNWs lay = ising::nn_ws_layout(net->L, net->max_batch);
    const float* wexp = reinterpret_cast<const float*>(ws_of(net) + lay.wexp);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // the whole lattice in LDS where it fits, else the sampler's wavefront
    // in teacher-forcing mode: the same bits either way
    const size_t lds = ising::nn_lattice_lds_bytes(net->L);
    if (lds && lds <= (size_t)ising::abi::device_max_lds())
        HIP_TRY(ising::launch_nn_lattice(wexp, net->L, batch, symmetric, s_dev, stride, logq_dev,
                                         ising::abi::device_cus(), st),
                "nn logq");
    else
        HIP_TRY(ising::launch_nn_wave(wexp, net->L, batch, 0, symmetric, s_dev, stride,
                                      ising::Key{0u, 0u}, 0u, 0u, nullptr, 0, logq_dev, st),
                "nn logq");
    return ISING_OK;
}

int ising_nn_grad(const ising_nn* net, const int8_t* s_dev, int64_t stride, int32_t batch,
                  float* loss_dev, void* hip_stream) {
    int rc = validate(net);
    if (rc)
        return rc;
    if ((rc = check_batch_args(net, s_dev, stride, batch)))
        return rc;
    const ising::NNWs lay = ising::nn_ws_layout(net->L, net->max_batch);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(net);
    HIP_TRY(ising::launch_nn_forward(s_dev, stride, batch, net->L, lay, ws,
                                     reinterpret_cast<float*>(ws + lay.logq), true, 1.f, st),
            "nn forward");
    HIP_TRY(ising::launch_nn_backward(s_dev, stride, batch, net->L, lay, ws, net->grad, loss_dev,
                                      st),
            "nn backward");
    return ISING_OK;
}

int ising_nn_adam(const ising_nn* net, float lr, float b1, float b2, float eps, int32_t step,
                  void* hip_stream) {
    int rc = validate(net);
    if (rc)
        return rc;
    if (step < 1)
        return set_error(ISING_E_INVALID, "step = %d < 1", step);
    if (!(lr > 0.f) || isinf(lr) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) ||
        !(eps > 0.f) || isinf(eps))
        return set_error(ISING_E_INVALID, "Adam hyper-parameters out of range");
    // bias corrections computed on the host in double
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
    const ising::NNWs lay = ising::nn_ws_layout(net->L, net->max_batch);
    HIP_TRY(ising::launch_nn_adam(net->master, net->adam_m, net->adam_v, net->grad, net->weights,
                                  reinterpret_cast<float*>(ws_of(net) + lay.wexp), lr, b1, b2, eps,
                                  c1, c2, reinterpret_cast<hipStream_t>(hip_stream)),
            "nn adam");
    return ISING_OK;
}

int ising_nn_sample(const ising_nn* net, int32_t batch, uint64_t seed, uint32_t chain0,
                    uint32_t draw, int32_t symmetric, int8_t* s_out, int64_t stride,
                    float* logq_out, void* hip_stream) {
    int rc = validate(net);
    if (rc)
        return rc;
    if ((rc = check_batch_args(net, s_out, stride, batch)))
        return rc;
    if ((uint64_t)chain0 + (uint64_t)batch - 1 > 0xFFFFFFFFull)
        return set_error(ISING_E_INVALID, "chain0 + batch - 1 exceeds 2^32 - 1");
    if (symmetric != 0 && symmetric != 1)
        return set_error(ISING_E_INVALID, "symmetric must be 0 or 1");
    const ising::NNWs lay = ising::nn_ws_layout(net->L, net->max_batch);
    HIP_TRY(ising::launch_nn_wave(reinterpret_cast<const float*>(ws_of(net) + lay.wexp), net->L,
                                  batch, 1, symmetric, nullptr, 0, key_of(seed), chain0, draw,
                                  s_out, stride, logq_out,
                                  reinterpret_cast<hipStream_t>(hip_stream)),
            "nn sample");
    return ISING_OK;
}

int ising_batch_mh(const ising_batch* b, int32_t L_prop, const int8_t* prop_dev,
                   int64_t prop_stride, const float* logq_cur_dev, const float* logq_prop_dev,
                   const double* beta_dev, uint32_t draw, int32_t* accepted_dev,
                   void* hip_stream) {
    if (!b)
        return set_error(ISING_E_INVALID, "batch pointer is NULL");
    if (b->abi_version != ISING_ABI_VERSION || b->count < 1 || b->count > ISING_BATCH_MAX_COUNT ||
        !b->spins || !aligned256(b->spins) || !b->workspace || !aligned256(b->workspace))
        return set_error(ISING_E_INVALID, "invalid batch description");
    if (L_prop < 2 || L_prop > ISING_NN_MAX_L || L_prop > b->max_L)
        return set_error(ISING_E_INVALID, "L_prop = %d outside 2..min(%d, max_L)", L_prop,
                         ISING_NN_MAX_L);
    if (!prop_dev || !logq_cur_dev || !logq_prop_dev || !beta_dev)
        return set_error(ISING_E_INVALID, "NULL device pointer");
    if (prop_stride < (int64_t)L_prop * L_prop)
        return set_error(ISING_E_INVALID, "prop_stride < L_prop^2");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(b->workspace);
    const ising::Key key{(uint32_t)(b->seed & 0xFFFFFFFFu), (uint32_t)(b->seed >> 32)};
    HIP_TRY(ising::launch_batch_mh(ws, b->count, b->spins_bytes, b->max_L, b->spins, L_prop,
                                   prop_dev, prop_stride, logq_cur_dev, logq_prop_dev, beta_dev, key,
                                   draw, accepted_dev, st),
            "batch mh");
    return ISING_OK;
}

}  // extern "C"
