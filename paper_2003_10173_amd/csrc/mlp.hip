// Placeholder translation unit for the learned sample-count model kernels.
#include "internal.h"
