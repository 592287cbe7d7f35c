// Adam (Kingma and Ba 2015) on device, with the bias correction the
// thesis's summary omits for simplicity (Ch. 3, Adagrad / RMSProp / Adam):
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   x <- x - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
#include <cmath>

#include "dr_host.h"

namespace dr {

__global__ void k_adam(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Step count kept on the device (for captured graphs): every lane reads t - 1
// from *step, one lane of the last kernel increments it.
__global__ void k_adam_counted(float* __restrict__ x, const float* __restrict__ g, float* __restrict__ m,
                               float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                               const long long* __restrict__ step) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = (double)(*step + 1);
    float c1 = (float)(1.0 - pow((double)b1, t)), c2 = (float)(1.0 - pow((double)b2, t));
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    x[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_step_inc(long long* step) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
}

}  // namespace dr

extern "C" drStatus drAdamStep(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                               float eps, int64_t step, hipStream_t st) {
    if (!x || !g || !m || !v || n < 0 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return DR_ERROR_INVALID_VALUE;
    if (n == 0) return DR_SUCCESS;
    double c1 = 1.0 - std::pow((double)beta1, (double)step), c2 = 1.0 - std::pow((double)beta2, (double)step);
    int bs = 256;
    long nb = (n + bs - 1) / bs;
    dr::k_adam<<<(unsigned)nb, bs, 0, st>>>(x, g, m, v, n, lr, beta1, beta2, eps, (float)c1, (float)c2);
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}

extern "C" drStatus drAdamStepCounted(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                                      float beta2, float eps, int64_t* step, hipStream_t st) {
    if (!x || !g || !m || !v || !step || n < 0 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return DR_ERROR_INVALID_VALUE;
    if (n > 0) {
        long nb = (n + 255) / 256;
        dr::k_adam_counted<<<(unsigned)nb, 256, 0, st>>>(x, g, m, v, n, lr, beta1, beta2, eps,
                                                         reinterpret_cast<const long long*>(step));
    }
    dr::k_step_inc<<<1, 1, 0, st>>>(reinterpret_cast<long long*>(step));
    return hipGetLastError() == hipSuccess ? DR_SUCCESS : DR_ERROR_DEVICE;
}
