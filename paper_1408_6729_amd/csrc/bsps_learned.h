// bsps_learned.h -- learned bucketing (not in the paper): a linear root model
// selecting one of L linear leaf models of the key distribution, trained on the
// sorted sample with forward, backward (gradient + Gram sums) and Newton-update
// kernels, and a per-key ranking that predicts the bucket and then checks it
// exactly against the splitters.
#pragma once
#include "bsps_device.h"

extern "C" size_t bsps_model_bytes(int32_t leaves) { return 16 + 16 + (size_t)(leaves > 0 ? leaves : 4096) * 12; }
extern "C" size_t bsps_fit_workspace_bytes(int64_t N, int32_t leaves) {
    return (size_t)(N > 0 ? N : 1) * 8 + (size_t)(leaves > 0 ? leaves : 4096) * 64 + 4096;
}
