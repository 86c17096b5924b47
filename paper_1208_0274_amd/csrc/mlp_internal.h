// The work predictor shared by the MLP library and the search.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "alae.h"

struct alae_mlp {
    int device = 0;
    float *d_params = nullptr;  // ALAE_MLP_PARAMS floats
    float *d_grad = nullptr;
    float *d_m1 = nullptr;      // Adam moments
    float *d_m2 = nullptr;
    double *d_loss = nullptr;
    uint64_t adam_t = 0;
    // staging of host-side calls
    float *d_x = nullptr;
    float *d_t = nullptr;
    uint32_t *d_idx = nullptr;
    size_t data_cap = 0;
};

namespace alae {
// y[i] = network(x[i*F .. i*F+F)) for i < n, on stream s.
alae_status mlp_predict_device(const alae_mlp *net, const float *d_x, uint32_t n, float *d_y, hipStream_t s);
}  // namespace alae
