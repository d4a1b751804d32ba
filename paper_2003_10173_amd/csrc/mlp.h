// Learned first-round sample counts (internal interface of mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "h2.h"

namespace h2 {
// y[0:batch] = network(X[batch x 16, row-major]) (device pointers)
void mlp_forward(const h2_mlp* M, int batch, const float* X, float* y, hipStream_t s);
// training records of builds (features of every sibling pair, log(1 + columns needed))
bool records_on();
void records_add(const std::vector<float>& feats, const std::vector<float>& targets);
}  // namespace h2
