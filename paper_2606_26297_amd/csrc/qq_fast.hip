// qq_fast.hip -- complex64 pass kernels, one launch per pass, one kernel
// instantiation per pass kind and qubit-set geometry (bodies in qq_passes.h).
#include "qq_passes.h"

namespace qq {
namespace {

using namespace dev;
using namespace passes;

// One workgroup per (state b, workgroup slot g), tiles g, g + G, ...; FP64 partial sums per slot.
template <int KIND, bool HIGH, bool FULL, typename DT, bool PART, bool WIDE = false>
__device__ __forceinline__ void fast_pass_impl(const FastArgs &a)
{
    constexpr int NSLOT = kind_slots<KIND>();
    __shared__ float2 lds[kLdsSlots];
    __shared__ double s_red[kThreads / 64][4];

    const int t = threadIdx.x;
    int b, g;
    block_coords(a.B, a.G, b, g);
    double acc[3] = {0.0, 0.0, 0.0};
    // the per-pass kernels form the cost values from the per-tile tables (non-partitioned phases)
    run_pass<KIND, HIGH, FULL, DT, PART, WIDE, !PART>(a, lds, acc, t, b, g);

    if constexpr (NSLOT > 0) {
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            double xs = acc[s];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) xs += __shfl_xor(xs, d, 64);
            if (lane == 0) s_red[wave][s] = xs;
        }
        __syncthreads();
        if (t < NSLOT)
            a.partial[(size_t)(a.slot_base + t) * a.slot_stride + (size_t)b * a.G + g] =
                (s_red[0][t] + s_red[1][t]) + (s_red[2][t] + s_red[3][t]);
    }
}

template <int KIND, bool HIGH, bool FULL, typename DT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KIND >= FK_LASTG ? 3 : 4)))
fast_pass(const FastArgs a)
{
    fast_pass_impl<KIND, HIGH, FULL, DT, false>(a);
}

// The same passes with the phase applied as per-QPU local factors and the cross factor
// (kinds that apply a phase: first, turn, adjoint turn).
template <int KIND, bool HIGH, bool FULL, typename DT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KIND >= FK_LASTG ? 3 : 4)))
fast_pass_part(const FastArgs a)
{
    fast_pass_impl<KIND, HIGH, FULL, DT, true>(a);
}

// Partial high sets whose upper run starts at qubit 28 or above (n >= 32): a lane's offset in
// the layout whose lane bits sit on that run can exceed 4 GiB, so it is kept in 64 bits.
template <int KIND, typename DT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KIND >= FK_LASTG ? 3 : 4)))
fast_pass_wide(const FastArgs a)
{
    fast_pass_impl<KIND, true, false, DT, false, true>(a);
}

template <int KIND, typename DT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KIND >= FK_LASTG ? 3 : 4)))
fast_pass_part_wide(const FastArgs a)
{
    fast_pass_impl<KIND, true, false, DT, true, true>(a);
}

template <int KIND>
constexpr bool kind_phases()
{
    return KIND == FK_FIRST || KIND == FK_TURN || KIND == FK_BTURN;
}

template <int KIND, bool HIGH, bool FULL>
hipError_t launch_k(const FastArgs &a, int diag_type, bool part, hipStream_t s)
{
    const dim3 grid((unsigned)(a.B * a.G)), block(kThreads);
    if constexpr (kind_phases<KIND>()) {
        if (part) {
            switch (diag_type) {
            case DIAG_F64: hipLaunchKernelGGL((fast_pass_part<KIND, HIGH, FULL, double>), grid, block, 0, s, a); break;
            case DIAG_I32: hipLaunchKernelGGL((fast_pass_part<KIND, HIGH, FULL, int32_t>), grid, block, 0, s, a); break;
            default: hipLaunchKernelGGL((fast_pass_part<KIND, HIGH, FULL, int16_t>), grid, block, 0, s, a); break;
            }
            return hipGetLastError();
        }
    }
    switch (diag_type) {
    case DIAG_F64: hipLaunchKernelGGL((fast_pass<KIND, HIGH, FULL, double>), grid, block, 0, s, a); break;
    case DIAG_I32: hipLaunchKernelGGL((fast_pass<KIND, HIGH, FULL, int32_t>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((fast_pass<KIND, HIGH, FULL, int16_t>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_wide(const FastArgs &a, int diag_type, bool part, hipStream_t s)
{
    const dim3 grid((unsigned)(a.B * a.G)), block(kThreads);
    if constexpr (kind_phases<KIND>()) {
        if (part) {
            switch (diag_type) {
            case DIAG_F64: hipLaunchKernelGGL((fast_pass_part_wide<KIND, double>), grid, block, 0, s, a); break;
            case DIAG_I32: hipLaunchKernelGGL((fast_pass_part_wide<KIND, int32_t>), grid, block, 0, s, a); break;
            default: hipLaunchKernelGGL((fast_pass_part_wide<KIND, int16_t>), grid, block, 0, s, a); break;
            }
            return hipGetLastError();
        }
    }
    switch (diag_type) {
    case DIAG_F64: hipLaunchKernelGGL((fast_pass_wide<KIND, double>), grid, block, 0, s, a); break;
    case DIAG_I32: hipLaunchKernelGGL((fast_pass_wide<KIND, int32_t>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((fast_pass_wide<KIND, int16_t>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(const FastArgs &a, bool high, int diag_type, bool part, hipStream_t s)
{
    if (!high) return launch_k<KIND, false, true>(a, diag_type, part, s);  // the low set is always qubits 0..11
    // largest layout-1 lane offset: (15 + 3 * 2^q) amplitudes of 8 bytes, q = pos8 or its address
    // position with interleaved psi / lambda blocks
    const int q8 = a.pos8 + (a.ilv && a.pos8 >= a.ilv);
    const bool wide = ((15ull + (3ull << q8)) * 8ull) >> 32 != 0;
    if (a.active == 0x0ff0) {
        if (wide) return hipErrorInvalidValue;  // full high sets stay below qubit 28 for n <= 34
        return launch_k<KIND, true, true>(a, diag_type, part, s);
    }
    return wide ? launch_wide<KIND>(a, diag_type, part, s) : launch_k<KIND, true, false>(a, diag_type, part, s);
}

}  // namespace

hipError_t launch_fast_pass(int kind, bool high, int diag_type, const FastPassParams &pp, hipStream_t s)
{
    FastArgs a;
    a.B = pp.B;
    a.G = pp.G;
    a.p = pp.p;
    a.k = pp.k;
    a.tiles = pp.tiles;
    a.dim_mask = pp.dim_mask;
    a.pos4 = pp.pos4;
    a.pos8 = pp.pos8;
    a.w1 = pp.w1;
    a.w2 = pp.w2;
    a.active = pp.active;
    a.nact = __builtin_popcount(pp.active);
    a.store_psi = pp.store_psi;
    a.slot_base = pp.slot_base;
    a.slot_stride = pp.slot_stride;
    a.amp0 = pp.amp0;
    a.params = pp.params;
    a.diag = pp.diag;
    a.psi = static_cast<float2 *>(pp.psi);
    a.lam = static_cast<float2 *>(pp.lam);
    a.state_stride = pp.state_stride;
    a.partial = pp.partial;
    a.blocked = pp.blocked;
    a.part = pp.part_desc;
    a.tables = pp.part_tables;
    a.cq = pp.cq;
    a.pcq = pp.part_cq;
    a.pcq_runs = pp.part_cq_runs;
    a.shift = pp.shift;
    a.ctab = pp.ctab;
    a.cthr = pp.cthr;
    a.xtab = pp.xtab;
    a.xthr = pp.xthr;
    a.ilv = pp.ilv;
    const bool part = pp.part != 0;
    switch (kind) {
    case FK_FIRST: return launch_kind<FK_FIRST>(a, high, diag_type, part, s);
    case FK_MID: return launch_kind<FK_MID>(a, high, diag_type, part, s);
    case FK_TURN: return launch_kind<FK_TURN>(a, high, diag_type, part, s);
    case FK_LAST: return launch_kind<FK_LAST>(a, high, diag_type, part, s);
    case FK_LASTG: return launch_kind<FK_LASTG>(a, high, diag_type, part, s);
    case FK_BMID: return launch_kind<FK_BMID>(a, high, diag_type, part, s);
    case FK_BTURN: return launch_kind<FK_BTURN>(a, high, diag_type, part, s);
    case FK_BLAST: return launch_kind<FK_BLAST>(a, high, diag_type, part, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qq
