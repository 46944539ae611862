// qq_plain.hip -- the plain complex128 form of the same computation, one kernel per gate.
//
// This is the measurement baseline: the state |+>^n is evolved by one phase
// kernel per layer (eq. (10)) and one RX kernel per qubit and layer
// (eq. (13)), the energy (eq. (17)) is one reduction, and the gradient uses the
// same adjoint equations as the fused path without fusion: per layer and
// qubit a <lambda|X_q|psi> reduction and two RX kernels, then a
// <lambda|C|psi> reduction and two phase kernels.  One parameter set per call.
#include "qq_internal.h"
#include "qq_twopi.h"

namespace qq {
namespace {

constexpr int kB = 256;

template <typename DT>
__device__ __forceinline__ double cz(const void *d, uint64_t i)
{
    return (double)static_cast<const DT *>(d)[i];
}

__global__ void plain_init(double2 *psi, uint64_t dim, double amp)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) psi[z] = make_double2(amp, 0.0);
}

// psi *= exp(-i sign gamma C)
template <typename DT>
__global__ void plain_phase(double2 *psi, const void *diag, uint64_t dim, double gamma, double sign)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const double th = gamma * cz<DT>(diag, z);
        const double k = rint(th * QQ_INV_TWO_PI);
        const double r = fma(-k, QQ_TWO_PI_LO, fma(-k, QQ_TWO_PI_HI, th));
        double s, c;
        sincos(r, &s, &c);
        s *= sign;
        const double2 v = psi[z];
        psi[z] = make_double2(v.x * c + v.y * s, v.y * c - v.x * s);
    }
}

// RX on qubit q: (a, b) -> (c a - i s b, -i s a + c b)
__global__ void plain_rx(double2 *psi, uint64_t half, int q, double c, double s)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t lo = (1ull << q) - 1;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < half; k += stride) {
        const uint64_t z0 = ((k & ~lo) << 1) | (k & lo);
        const uint64_t z1 = z0 | (1ull << q);
        const double2 a = psi[z0], b = psi[z1];
        psi[z0] = make_double2(c * a.x + s * b.y, c * a.y - s * b.x);
        psi[z1] = make_double2(c * b.x + s * a.y, c * b.y - s * a.x);
    }
}

__device__ void block_store(double v, double *out)
{
    __shared__ double red[kB];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

template <typename DT>
__global__ void plain_energy(const double2 *psi, const void *diag, uint64_t dim, double *partial)
{
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const double2 v = psi[z];
        acc += (v.x * v.x + v.y * v.y) * cz<DT>(diag, z);
    }
    block_store(acc, partial);
}

template <typename DT>
__global__ void plain_lambda(const double2 *psi, const void *diag, double2 *lam, uint64_t dim)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const double c = cz<DT>(diag, z);
        lam[z] = make_double2(c * psi[z].x, c * psi[z].y);
    }
}

// Im sum over pairs of qubit q of conj(l0) a1 + conj(l1) a0  (= Im <lambda|X_q|psi>)
__global__ void plain_xq(const double2 *psi, const double2 *lam, uint64_t half, int q, double *partial)
{
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t lo = (1ull << q) - 1;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < half; k += stride) {
        const uint64_t z0 = ((k & ~lo) << 1) | (k & lo);
        const uint64_t z1 = z0 | (1ull << q);
        const double2 a0 = psi[z0], a1 = psi[z1], l0 = lam[z0], l1 = lam[z1];
        acc += (l0.x * a1.y - l0.y * a1.x) + (l1.x * a0.y - l1.y * a0.x);
    }
    block_store(acc, partial);
}

// Im sum conj(lambda) C psi
template <typename DT>
__global__ void plain_gc(const double2 *psi, const double2 *lam, const void *diag, uint64_t dim, double *partial)
{
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const double2 a = psi[z], l = lam[z];
        acc += cz<DT>(diag, z) * (l.x * a.y - l.y * a.x);
    }
    block_store(acc, partial);
}

// result[idx] (= or +=) scale * sum(partial[0..nb))
__global__ void plain_reduce(const double *partial, int nb, double *result, int idx, double scale, int add)
{
    __shared__ double red[kB];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nb; k += kB) acc += partial[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) result[idx] = (add ? result[idx] : 0.0) + scale * red[0];
}

template <typename DT>
hipError_t run_plain_t(const PlainArgs &a, hipStream_t s)
{
    double2 *psi = static_cast<double2 *>(a.psi);
    double2 *lam = static_cast<double2 *>(a.lam);
    const uint64_t half = a.dim / 2;
    const dim3 g(a.nblocks), blk(kB);
    hipLaunchKernelGGL(plain_init, g, blk, 0, s, psi, a.dim, 1.0 / std::sqrt((double)a.dim));
    for (int k = 0; k < a.p; ++k) {
        const double gam = a.params[2 * k], bet = a.params[2 * k + 1];
        hipLaunchKernelGGL(plain_phase<DT>, g, blk, 0, s, psi, a.diag, a.dim, gam, 1.0);
        for (int q = 0; q < a.n; ++q)
            hipLaunchKernelGGL(plain_rx, g, blk, 0, s, psi, half, q, std::cos(bet), std::sin(bet));
    }
    hipLaunchKernelGGL(plain_energy<DT>, g, blk, 0, s, psi, a.diag, a.dim, a.partial);
    hipLaunchKernelGGL(plain_reduce, dim3(1), blk, 0, s, a.partial, a.nblocks, a.result, 0, 1.0, 0);
    if (a.grad) {
        hipLaunchKernelGGL(plain_lambda<DT>, g, blk, 0, s, psi, a.diag, lam, a.dim);
        for (int k = a.p - 1; k >= 0; --k) {
            const double gam = a.params[2 * k], bet = a.params[2 * k + 1];
            for (int q = 0; q < a.n; ++q) {
                hipLaunchKernelGGL(plain_xq, g, blk, 0, s, psi, lam, half, q, a.partial);
                hipLaunchKernelGGL(plain_reduce, dim3(1), blk, 0, s, a.partial, a.nblocks, a.result, 2 + 2 * k, 2.0,
                                   q > 0);
            }
            for (int q = 0; q < a.n; ++q) {
                hipLaunchKernelGGL(plain_rx, g, blk, 0, s, psi, half, q, std::cos(bet), -std::sin(bet));
                hipLaunchKernelGGL(plain_rx, g, blk, 0, s, lam, half, q, std::cos(bet), -std::sin(bet));
            }
            hipLaunchKernelGGL(plain_gc<DT>, g, blk, 0, s, psi, lam, a.diag, a.dim, a.partial);
            hipLaunchKernelGGL(plain_reduce, dim3(1), blk, 0, s, a.partial, a.nblocks, a.result, 1 + 2 * k, 2.0, 0);
            if (k > 0) {
                hipLaunchKernelGGL(plain_phase<DT>, g, blk, 0, s, psi, a.diag, a.dim, gam, -1.0);
                hipLaunchKernelGGL(plain_phase<DT>, g, blk, 0, s, lam, a.diag, a.dim, gam, -1.0);
            }
        }
    }
    return hipGetLastError();
}

}  // namespace

hipError_t run_plain(const PlainArgs &a, hipStream_t s)
{
    switch (a.diag_type) {
    case DIAG_F64: return run_plain_t<double>(a, s);
    case DIAG_I32: return run_plain_t<int32_t>(a, s);
    default: return run_plain_t<int16_t>(a, s);
    }
}

}  // namespace qq
