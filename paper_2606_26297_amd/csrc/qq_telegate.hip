// qq_telegate.hip -- gate-level trajectory of the distributed QAOA circuit with explicit TeleGate
// remote CNOTs (distributed circuit construction section): n data qubits plus two communication
// qubits, complex128.  Cross-QPU ZZ terms are realised through two remote CNOTs, each with two
// mid-circuit measurements and conditional Pauli corrections; the measurement outcomes are decided
// on the device from caller-given uniforms, so a trajectory runs without host round trips.
//
// Qubit layout: data qubits 0 .. n-1 (bit i-1 of the index is variable z_i), communication qubits
// n (on the control's QPU) and n + 1 (on the target's QPU).
#include "qq_device.h"

namespace qq {
namespace {

constexpr int kTgThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void tg_init(double2 *psi, uint64_t dim, int n, double amp)
{
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += (uint64_t)gridDim.x * blockDim.x)
        psi[z] = make_double2((z >> n) == 0 ? amp : 0.0, 0.0);
}

// psi(z) *= exp(-i gamma (C(z_data) - C_x(z_data))): the phase of every term local to a QPU.
template <typename DT>
__global__ void tg_local_phase(double2 *psi, uint64_t dim, uint64_t dmask, const DT *diag, const DT *cross, double gamma)
{
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t d = z & dmask;
        const double th = -gamma * ((double)diag[d] - (double)cross[d]);
        double s, c;
        sincos(th, &s, &c);
        psi[z] = cmul(psi[z], make_double2(c, s));
    }
}

// diag(1, e^{i phi}) on qubit q
__global__ void tg_phase1(double2 *psi, uint64_t dim, int q, double c, double s)
{
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += (uint64_t)gridDim.x * blockDim.x)
        if ((z >> q) & 1ull) psi[z] = cmul(psi[z], make_double2(c, s));
}

// Two-level operations over the pairs (z, z | 2^t) with bit t of z clear.
__device__ __forceinline__ uint64_t pair_index(uint64_t k, int t)
{
    const uint64_t lo = k & ((1ull << t) - 1ull);
    return ((k >> t) << (t + 1)) | lo;
}

// kind 0: CNOT with control c (bit c set swaps the pair); 1: Hadamard; 2: RX(2 beta) = (cos, -i sin)
// 3: X if outcome[slot]; 4: Z on qubit t if outcome[slot] (the phase of the bit-set member)
__global__ void tg_pair(double2 *psi, uint64_t half, int t, int kind, int c, double cb, double sb, const int *outcome,
                        int slot)
{
    if (kind >= 3 && outcome[slot] == 0) return;
    const double r = 0.70710678118654752440;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < half; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t z0 = pair_index(k, t), z1 = z0 | (1ull << t);
        const double2 a = psi[z0], b = psi[z1];
        if (kind == 0) {
            if ((z0 >> c) & 1ull) {
                psi[z0] = b;
                psi[z1] = a;
            }
        } else if (kind == 1) {
            psi[z0] = make_double2(r * (a.x + b.x), r * (a.y + b.y));
            psi[z1] = make_double2(r * (a.x - b.x), r * (a.y - b.y));
        } else if (kind == 2) {
            psi[z0] = make_double2(cb * a.x + sb * b.y, cb * a.y - sb * b.x);
            psi[z1] = make_double2(cb * b.x + sb * a.y, cb * b.y - sb * a.x);
        } else if (kind == 3) {
            psi[z0] = b;
            psi[z1] = a;
        } else {
            psi[z1] = make_double2(-b.x, -b.y);
        }
    }
}

// Probability of bit q = 1: per-workgroup partial sums (fixed order).
__global__ void __launch_bounds__(kTgThreads) tg_prob1(const double2 *psi, uint64_t half, int q, double *partial)
{
    __shared__ double red[kTgThreads];
    double acc = 0.0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < half; k += (uint64_t)gridDim.x * blockDim.x) {
        const double2 b = psi[pair_index(k, q) | (1ull << q)];
        acc += b.x * b.x + b.y * b.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kTgThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Outcome 1 when u < p1; the kept branch's renormalisation.
__global__ void tg_decide(const double *partial, int nblocks, double u, int *outcome, double *scale, int slot)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double p1 = 0.0;
    for (int i = 0; i < nblocks; ++i) p1 += partial[i];
    const int m = u < p1 ? 1 : 0;
    outcome[slot] = m;
    scale[slot] = 1.0 / sqrt(m ? p1 : 1.0 - p1);
}

__global__ void tg_collapse(double2 *psi, uint64_t dim, int q, const int *outcome, const double *scale, int slot)
{
    const uint64_t m = (uint64_t)outcome[slot];
    const double f = scale[slot];
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += (uint64_t)gridDim.x * blockDim.x) {
        const double2 a = psi[z];
        psi[z] = ((z >> q) & 1ull) == m ? make_double2(a.x * f, a.y * f) : make_double2(0.0, 0.0);
    }
}

// The protocol leaves the global phase (-1)^(m1 m2); removed so that trajectories compare with the
// exact state.
__global__ void tg_sign(double2 *psi, uint64_t dim, const int *outcome, int slot)
{
    if (!(outcome[slot] && outcome[slot + 1])) return;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += (uint64_t)gridDim.x * blockDim.x)
        psi[z] = make_double2(-psi[z].x, -psi[z].y);
}

int grid_of(uint64_t work)
{
    return (int)std::min<uint64_t>(std::max<uint64_t>((work + kTgThreads - 1) / kTgThreads, 1), 4096);
}

}  // namespace

hipError_t tg_launch_init(double2 *psi, int n, hipStream_t s)
{
    const uint64_t dim = 1ull << (n + 2);
    hipLaunchKernelGGL(tg_init, dim3(grid_of(dim)), dim3(kTgThreads), 0, s, psi, dim, n, 1.0 / sqrt((double)(1ull << n)));
    return hipGetLastError();
}

hipError_t tg_launch_local_phase(double2 *psi, int n, const void *diag, const void *cross, int diag_type, double gamma,
                                 hipStream_t s)
{
    const uint64_t dim = 1ull << (n + 2), dmask = (1ull << n) - 1ull;
    const dim3 g(grid_of(dim)), b(kTgThreads);
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL(tg_local_phase<double>, g, b, 0, s, psi, dim, dmask, static_cast<const double *>(diag),
                           static_cast<const double *>(cross), gamma);
        break;
    case DIAG_I32:
        hipLaunchKernelGGL(tg_local_phase<int32_t>, g, b, 0, s, psi, dim, dmask, static_cast<const int32_t *>(diag),
                           static_cast<const int32_t *>(cross), gamma);
        break;
    default:
        hipLaunchKernelGGL(tg_local_phase<int16_t>, g, b, 0, s, psi, dim, dmask, static_cast<const int16_t *>(diag),
                           static_cast<const int16_t *>(cross), gamma);
        break;
    }
    return hipGetLastError();
}

hipError_t tg_launch_phase1(double2 *psi, int nq, int q, double phi, hipStream_t s)
{
    const uint64_t dim = 1ull << nq;
    hipLaunchKernelGGL(tg_phase1, dim3(grid_of(dim)), dim3(kTgThreads), 0, s, psi, dim, q, cos(phi), sin(phi));
    return hipGetLastError();
}

hipError_t tg_launch_pair(double2 *psi, int nq, int t, int kind, int c, double cb, double sb, const int *outcome,
                          int slot, hipStream_t s)
{
    const uint64_t half = 1ull << (nq - 1);
    hipLaunchKernelGGL(tg_pair, dim3(grid_of(half)), dim3(kTgThreads), 0, s, psi, half, t, kind, c, cb, sb, outcome,
                       slot);
    return hipGetLastError();
}

hipError_t tg_launch_measure(double2 *psi, int nq, int q, double u, double *partial, int nblocks, int *outcome,
                             double *scale, int slot, hipStream_t s)
{
    const uint64_t dim = 1ull << nq, half = dim >> 1;
    hipLaunchKernelGGL(tg_prob1, dim3(nblocks), dim3(kTgThreads), 0, s, psi, half, q, partial);
    hipLaunchKernelGGL(tg_decide, dim3(1), dim3(64), 0, s, partial, nblocks, u, outcome, scale, slot);
    hipLaunchKernelGGL(tg_collapse, dim3(grid_of(dim)), dim3(kTgThreads), 0, s, psi, dim, q, outcome, scale, slot);
    return hipGetLastError();
}

hipError_t tg_launch_sign(double2 *psi, int nq, const int *outcome, int slot, hipStream_t s)
{
    const uint64_t dim = 1ull << nq;
    hipLaunchKernelGGL(tg_sign, dim3(grid_of(dim)), dim3(kTgThreads), 0, s, psi, dim, outcome, slot);
    return hipGetLastError();
}

}  // namespace qq
