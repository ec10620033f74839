// Optimiser of the mesh-morphing loop: Adam (Kingma and Ba, 2015, Algorithm 1) over a
// flat FP32 parameter array.  Memory-bound: 16 B read and 12 B written per parameter.
#include "wn_internal.hpp"

namespace wn {

__global__ __launch_bounds__(kBlock) void k_adam(float *__restrict__ x, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                 float lr, float b1, float b2, float c1, float c2, float eps) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
        m[i] = mi;
        v[i] = vi;
        // bias-corrected moments: c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
        x[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

hipError_t launch_adam(float *x, const float *g, float *m, float *v, int64_t n, int64_t t, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const double c1 = 1.0 / (1.0 - pow((double)b1, (double)t));
    const double c2 = 1.0 / (1.0 - pow((double)b2, (double)t));
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const int grid = (int)(blocks < 4096 ? blocks : 4096);
    k_adam<<<grid, kBlock, 0, s>>>(x, g, m, v, n, lr, b1, b2, (float)c1, (float)c2, eps);
    return hipGetLastError();
}

}  // namespace wn
