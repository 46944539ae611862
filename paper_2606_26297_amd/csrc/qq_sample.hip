// qq_sample.hip -- shots from the exact output distribution P(z) = |psi(z)|^2 of the final state
// (computational-basis measurement, and the final shot-based evaluation of the measurement
// decoding section, drawn here from the exact state rather than a circuit simulator).
//
// A shot with uniform u in [0, 1) takes the first basis index z whose cumulative probability
// sum_{y <= z} P(y) exceeds u * sum_y P(y) (inverse transform in basis order).  The search is
// hierarchical: blocks of 4096 consecutive indices, each summed row by row (64 consecutive entries
// per row, one per lane), and a prefix over the block sums (formed on the host in index order);
// a shot finds its block by binary search over that prefix, then scans the block's rows with the
// same row sums, so a block's scan ends exactly at the sum the prefix used.  All sums are FP64 in
// a fixed order; results are reproducible.
#include "qq_device.h"

namespace qq {
namespace {

constexpr int kRows = 64;  // rows of 64 entries per block of 4096 indices

template <typename C2>
__device__ __forceinline__ double prob_at(const C2 *psi, uint64_t z, uint64_t dim)
{
    if (z >= dim) return 0.0;
    const double re = (double)psi[z].x, im = (double)psi[z].y;
    return fma(re, re, im * im);
}

// Inclusive sum over lanes 0..lane of the wave (fixed order).
__device__ __forceinline__ double wave_scan(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// One wave per block: the block's probability mass, rows accumulated in order.
template <typename C2>
__global__ void __launch_bounds__(256) block_mass_kernel(const C2 *psi, uint64_t dim, uint64_t nblk, double *mass)
{
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nblk; b += waves) {
        const uint64_t base = b * (uint64_t)(kRows * 64);
        double acc = 0.0;
        for (int row = 0; row < kRows; ++row) {
            const double s = wave_scan(prob_at(psi, base + (uint64_t)row * 64 + lane, dim), lane);
            acc = __shfl(acc + s, 63, 64);
        }
        if (lane == 0) mass[b] = acc;
    }
}

// One wave per shot.  start[b] = sum of the masses of blocks before b, start[nblk] = total;
// last_blk: the last block of nonzero mass.
template <typename C2>
__global__ void __launch_bounds__(256) shot_kernel(const C2 *psi, uint64_t dim, uint64_t nblk, const double *start,
                                                   uint64_t last_blk, const double *u, int64_t shots, uint64_t *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double total = start[nblk];
    for (int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); s < shots; s += waves) {
        const double us = u[s];
        const double t = us * total;
        uint64_t lo = last_blk;
        double r = INFINITY;  // no entry reaches it: the scan below ends on the block's last nonzero entry
        if (us >= 0.0 && t < total) {
            // first block whose end exceeds t (at most last_blk, whose end is the total)
            lo = 0;
            uint64_t hi = last_blk;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (start[mid + 1] > t) hi = mid;
                else lo = mid + 1;
            }
            r = t - start[lo];
        }
        // uniforms outside [0, 1) (or whose product with the total rounds up to it) take the last
        // index of nonzero probability
        const uint64_t base = lo * (uint64_t)(kRows * 64);
        uint64_t idx = base, last_pos = base;
        bool found = false;
        double acc = 0.0;
        for (int row = 0; row < kRows && !found; ++row) {
            const uint64_t z = base + (uint64_t)row * 64 + lane;
            const double v = prob_at(psi, z, dim);
            const double pre = acc + wave_scan(v, lane);
            const uint64_t hit = __ballot(pre > r);
            if (hit) {
                idx = base + (uint64_t)row * 64 + (uint64_t)(__ffsll((long long)hit) - 1);
                found = true;
            } else {
                const uint64_t pos = __ballot(v > 0.0);
                if (pos) last_pos = base + (uint64_t)row * 64 + (uint64_t)(63 - __clzll((long long)pos));
                acc = __shfl(pre, 63, 64);
            }
        }
        // rounding can leave r at or beyond the block's mass: take its last entry of nonzero probability
        if (!found) idx = last_pos;
        if (lane == 0) out[s] = idx;
    }
}

template <typename DT>
__global__ void gather_cost_kernel(const DT *diag, const uint64_t *idx, int64_t count, double *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)diag[idx[i]];
}

int grid_for(uint64_t waves_needed)
{
    const uint64_t wg = (waves_needed + 3) / 4;
    return (int)std::min<uint64_t>(std::max<uint64_t>(wg, 1), 8192);
}

}  // namespace

hipError_t launch_block_mass(const void *psi, bool c128, uint64_t dim, uint64_t nblk, double *mass, hipStream_t s)
{
    const dim3 grid(grid_for(nblk)), block(256);
    if (c128)
        hipLaunchKernelGGL(block_mass_kernel<double2>, grid, block, 0, s, static_cast<const double2 *>(psi), dim, nblk,
                           mass);
    else
        hipLaunchKernelGGL(block_mass_kernel<float2>, grid, block, 0, s, static_cast<const float2 *>(psi), dim, nblk,
                           mass);
    return hipGetLastError();
}

hipError_t launch_shots(const void *psi, bool c128, uint64_t dim, uint64_t nblk, const double *start,
                        uint64_t last_blk, const double *u, int64_t shots, uint64_t *out, hipStream_t s)
{
    const dim3 grid(grid_for((uint64_t)shots)), block(256);
    if (c128)
        hipLaunchKernelGGL(shot_kernel<double2>, grid, block, 0, s, static_cast<const double2 *>(psi), dim, nblk, start,
                           last_blk, u, shots, out);
    else
        hipLaunchKernelGGL(shot_kernel<float2>, grid, block, 0, s, static_cast<const float2 *>(psi), dim, nblk, start,
                           last_blk, u, shots, out);
    return hipGetLastError();
}

hipError_t launch_gather_cost(const void *diag, int diag_type, const uint64_t *idx, int64_t count, double *out,
                              hipStream_t s)
{
    const int grid = (int)std::min<int64_t>(std::max<int64_t>((count + 255) / 256, 1), 4096);
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL(gather_cost_kernel<double>, dim3(grid), dim3(256), 0, s, static_cast<const double *>(diag),
                           idx, count, out);
        break;
    case DIAG_I32:
        hipLaunchKernelGGL(gather_cost_kernel<int32_t>, dim3(grid), dim3(256), 0, s,
                           static_cast<const int32_t *>(diag), idx, count, out);
        break;
    default:
        hipLaunchKernelGGL(gather_cost_kernel<int16_t>, dim3(grid), dim3(256), 0, s,
                           static_cast<const int16_t *>(diag), idx, count, out);
        break;
    }
    return hipGetLastError();
}

}  // namespace qq
