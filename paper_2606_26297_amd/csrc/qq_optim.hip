// qq_optim.hip -- device Adam step for graph-captured optimisation loops.
//
// The optimiser of the paper's search is Adam (optimisation-overhead section;
// there with an SPSA gradient estimate, here with the exact adjoint gradient).
// One launch updates every parameter of every start from the gradients the
// evaluation left in device memory, so an optimisation step
// [energy + gradient -> Adam] runs without host involvement and can be
// captured in a HIP graph and replayed.
//
// Update (Kingma and Ba), per parameter, with step counter t (1-based):
//   m <- b1 m + (1 - b1) g ;  v <- b2 v + (1 - b2) g^2
//   x <- x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
// The counter lives in device memory and is advanced by the kernel, so every
// replay of a captured step is the same launch.
#include "qq_internal.h"

namespace qq {
namespace {

// One workgroup: the step counter is read once and advanced after every update.
__global__ void __launch_bounds__(256) adam_kernel(const AdamArgs a)
{
    __shared__ int s_t;
    const int tid = threadIdx.x;
    if (tid == 0) s_t = *a.step + 1;
    __syncthreads();
    const int t = s_t;
    const double c1 = 1.0 - pow(a.beta1, (double)t);
    const double c2 = 1.0 - pow(a.beta2, (double)t);
    const int twop = 2 * a.p;
    const int total = a.B * twop;
    for (int i = tid; i < total; i += blockDim.x) {
        const int b = i / twop, j = i - b * twop;
        const double g = a.result[(size_t)b * (1 + twop) + 1 + j];
        const double m = fma(a.beta1, a.m[i], (1.0 - a.beta1) * g);
        const double v = fma(a.beta2, a.v[i], (1.0 - a.beta2) * g * g);
        a.m[i] = m;
        a.v[i] = v;
        a.x[i] -= a.lr * (m / c1) / (sqrt(v / c2) + a.eps);
        if (a.grad_out) a.grad_out[i] = g;
    }
    for (int b = tid; b < a.B; b += blockDim.x) {
        const double e = a.result[(size_t)b * (1 + twop)];
        a.energy_out[b] = e;
        if (a.history_len > 0) a.history[(size_t)((t - 1) % a.history_len) * a.B + b] = e;
    }
    __syncthreads();
    if (tid == 0) *a.step = t;
}

__global__ void fill_f64_kernel(double *p, double v, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

hipError_t launch_adam(const AdamArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace qq
