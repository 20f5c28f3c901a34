// Small utility kernels shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cr {

// fill with zero (used instead of hipMemsetAsync so that callers may capture the work in a graph)
template <typename T>
__global__ void k_fill_zero(T* __restrict__ p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = T{};
}

template <typename T>
inline void fill_zero(T* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

}  // namespace cr
