// mlp_internal.hpp -- a view of a network's device parameters for the library's own kernels (the
// surrogate's fused inference); not part of the public ABI.
#pragma once

#include <stdint.h>

#include "mlp.h"

namespace mlpk {

struct NetView {
    int n;                                 // layers
    int32_t w[MLP_MAX_LAYERS + 1];         // widths
    const uint16_t *wb[MLP_MAX_LAYERS];    // BF16 weights of layer i, [w[i+1]][w[i]] row-major
    const float *bias[MLP_MAX_LAYERS];     // FP32 biases of layer i, [w[i+1]]
};

NetView net_view(const mlp_t *m);

}  // namespace mlpk
