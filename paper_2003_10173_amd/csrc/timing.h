// Launch timing of selected kernels (see timing.cpp).
#pragma once
#include <hip/hip_runtime.h>

namespace h2 {
bool timing_on();
// returns a token (-1 when timing is off); record the launch between the calls
int timing_begin(hipStream_t s);
// work: algorithmic flops or bytes of the launch; if dev_count is given, the
// int it points to after the launch, times work_per_count, is added
void timing_end(int token, const char* name, hipStream_t s, double work,
                const int* dev_count = nullptr, double work_per_count = 0.0);
}  // namespace h2
