// MLP surrogate kernels (placeholder translation unit).
#include <hip/hip_runtime.h>
