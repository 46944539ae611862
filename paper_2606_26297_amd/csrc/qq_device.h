// qq_device.h -- device helpers shared by the pass kernels (tile layouts, LDS transposes,
// butterflies, FP64 phase-argument reduction).
#pragma once

#include "qq_internal.h"
#include "qq_twopi.h"

namespace qq {
namespace dev {

template <typename R>
struct Cx;
template <>
struct Cx<float> {
    using T = float2;
};
template <>
struct Cx<double> {
    using T = double2;
};

template <typename C2, typename R>
__device__ __forceinline__ C2 mk(R x, R y)
{
    C2 v;
    v.x = x;
    v.y = y;
    return v;
}

// LDS slot of tile-local amplitude i: one padding slot after every 16 amplitudes.
// Keeps the slot affine in the register index for every layout (one base
// register plus immediate offsets) and spreads 64-bit accesses of a wave
// over distinct banks.
constexpr int kLdsSlots = kTile + kTile / 16;
__device__ __forceinline__ int swz(int i) { return i + (i >> 4); }

// First amplitude of tile `tile` when the tile's qubits are 0..3, a..a+3 and c..c+3
// (a + 4 <= c): the tile index fills the other qubits in ascending order,
// w1 = a - 4 bits below a and w2 = c - a - 4 bits between the runs, the rest above c + 3.
__device__ __forceinline__ uint64_t tile_base(uint64_t tile, int a, int c, int w1, int w2)
{
    const uint64_t lo = tile & ((1ull << w1) - 1);
    tile >>= w1;
    const uint64_t mid = tile & ((1ull << w2) - 1);
    tile >>= w2;
    return (lo << 4) | (mid << (a + 4)) | (tile << (c + 4));
}

// (state b, workgroup slot g) of this workgroup, XCD-aware.  Workgroups are
// dispatched round-robin over the 8 XCDs (block i runs on XCD i mod 8), each XCD
// with its own L2.  Renumbering so that the B workgroups sharing a tile index
// (all states of the batch, which read the same cost-diagonal entries) are
// consecutive on one XCD lets that L2 serve the diagonal to all of them.
__device__ __forceinline__ void block_coords(int B, int G, int &b, int &g)
{
    const uint32_t nb = (uint32_t)B * (uint32_t)G, i = blockIdx.x;
    uint32_t L = i;
    if ((nb & 7u) == 0) L = (i & 7u) * (nb >> 3) + (i >> 3);
    b = (int)(L % (uint32_t)B);
    g = (int)(L / (uint32_t)B);
}

// Wave-uniform 64-bit value (kept in scalar registers and opaque to loop-invariant hoisting).
__device__ __forceinline__ uint64_t uni64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T ld_at(uint64_t ubase, uint64_t voff)
{
    return *reinterpret_cast<const T *>(ubase + voff);
}
template <typename T>
__device__ __forceinline__ void st_at(uint64_t ubase, uint64_t voff, T v)
{
    *reinterpret_cast<T *>(ubase + voff) = v;
}

// Tile-local index held by thread t in register r under layout L:
//   L = 2: register bits are tile bits 8..11, thread bits are tile bits 0..7
//   L = 1: register bits are tile bits 4..7,  thread bits are tile bits 0..3, 8..11
//   L = 0: register bits are tile bits 0..3,  thread bits are tile bits 4..11
template <int L>
__device__ __forceinline__ int lidx(int t, int r)
{
    if constexpr (L == 2) return t + 256 * r;
    else if constexpr (L == 1) return (t & 15) + 16 * r + ((t >> 4) << 8);
    else return r + 16 * t;
}

template <typename DT>
__device__ __forceinline__ double ldc(const void *p, uint64_t i)
{
    return (double)(static_cast<const DT *>(p)[i]);
}

// theta mod 2 pi in [-pi, pi]: k = rint(theta / 2pi), r = (theta - k HI) - k LO with FMAs
// (Cody-Waite reduction with a double-double 2 pi).
__device__ __forceinline__ double reduce_2pi(double th)
{
    const double k = rint(th * QQ_INV_TWO_PI);
    const double r = fma(-k, QQ_TWO_PI_HI, th);
    return fma(-k, QQ_TWO_PI_LO, r);
}

__device__ __forceinline__ void phase_cs(double theta, float &c, float &s)
{
    const float r = (float)reduce_2pi(theta);
    sincosf(r, &s, &c);
}
__device__ __forceinline__ void phase_cs(double theta, double &c, double &s)
{
    sincos(reduce_2pi(theta), &s, &c);
}

// ---- LDS transposes -----------------------------------------------------------------------
// complex64: one round of float2 words; complex128: two rounds of doubles (x, then y),
// so both fit a 32 KiB buffer.
// LDS slot swz(lidx<L>(t, r)) written as base(t) + stride * r (t < 256):
//   L2: t + t/16 + 272 r ;  L1: (t mod 16) + 272 (t/16) + 17 r ;  L0: 17 t + r.
template <int L>
__device__ __forceinline__ int slot_base(int t)
{
    if constexpr (L == 2) return t + (t >> 4);
    else if constexpr (L == 1) return (t & 15) + 272 * (t >> 4);
    else return 17 * t;
}
template <int L>
constexpr int slot_stride()
{
    return L == 2 ? 272 : L == 1 ? 17 : 1;
}

template <int L, typename C2>
__device__ __forceinline__ void lds_put(float2 *lds, const C2 (&v)[kRegs], int t, int)
{
    float2 *p = lds + slot_base<L>(t);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) p[slot_stride<L>() * r] = v[r];
}
template <int L, typename C2>
__device__ __forceinline__ void lds_get(const float2 *lds, C2 (&v)[kRegs], int t, int)
{
    const float2 *p = lds + slot_base<L>(t);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) v[r] = p[slot_stride<L>() * r];
}
template <int L>
__device__ __forceinline__ void lds_put(double *lds, const double2 (&v)[kRegs], int t, int comp)
{
    double *p = lds + slot_base<L>(t);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) p[slot_stride<L>() * r] = comp ? v[r].y : v[r].x;
}
template <int L>
__device__ __forceinline__ void lds_get(const double *lds, double2 (&v)[kRegs], int t, int comp)
{
    const double *p = lds + slot_base<L>(t);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const double w = p[slot_stride<L>() * r];
        if (comp) v[r].y = w;
        else v[r].x = w;
    }
}

template <typename W, typename C2>
__device__ __forceinline__ void transpose1(W *lds, C2 (&v)[kRegs], int t, int from, int to)
{
    constexpr int rounds = sizeof(C2) / sizeof(W);
#pragma unroll
    for (int c = 0; c < rounds; ++c) {
        __syncthreads();
        if (from == 0) lds_put<0>(lds, v, t, c);
        else if (from == 1) lds_put<1>(lds, v, t, c);
        else lds_put<2>(lds, v, t, c);
        __syncthreads();
        if (to == 0) lds_get<0>(lds, v, t, c);
        else if (to == 1) lds_get<1>(lds, v, t, c);
        else lds_get<2>(lds, v, t, c);
    }
}

// ---- butterflies --------------------------------------------------------------------------
// RX(2 beta) on tile bit K of the register group: (a, b) -> (c a - i s b, -i s a + c b).
template <int K, typename C2, typename R>
__device__ __forceinline__ void rx_bit(C2 (&v)[kRegs], R c, R s)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if (r & (1 << K)) continue;
        const C2 a = v[r], b = v[r | (1 << K)];
        v[r] = mk<C2, R>(c * a.x + s * b.y, c * a.y - s * b.x);
        v[r | (1 << K)] = mk<C2, R>(c * b.x + s * a.y, c * b.y - s * a.x);
    }
}

// sum over pairs of bit K of Im(conj(l0) a1 + conj(l1) a0), FP64 (products of FP32 inputs are exact).
template <int K, typename C2>
__device__ __forceinline__ double xexp_bit(const C2 (&a)[kRegs], const C2 (&l)[kRegs])
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if (r & (1 << K)) continue;
        const int q = r | (1 << K);
        acc = fma((double)l[r].x, (double)a[q].y, acc);
        acc = fma(-(double)l[r].y, (double)a[q].x, acc);
        acc = fma((double)l[q].x, (double)a[r].y, acc);
        acc = fma(-(double)l[q].y, (double)a[r].x, acc);
    }
    return acc;
}

__device__ __forceinline__ void add_slot(double (&acc)[kMaxLocalSlots], int slot, double v)
{
    switch (slot) {
    case 0: acc[0] += v; break;
    case 1: acc[1] += v; break;
    case 2: acc[2] += v; break;
    case 3: acc[3] += v; break;
    default: break;
    }
}

// Index of the local table entry of a QPU: the bits of its variables, in ascending order.
__device__ __forceinline__ uint64_t compress_bits(uint64_t z, const uint8_t *vars, int nv)
{
    uint64_t u = 0;
    for (int j = 0; j < nv; ++j) u |= ((z >> vars[j]) & 1ull) << j;
    return u;
}

template <typename R, typename C2>
__device__ __forceinline__ void rot_phase(C2 &v, R c, R s)
{
    // v * (c - i s)
    v = mk<C2, R>(v.x * c + v.y * s, v.y * c - v.x * s);
}

}  // namespace dev
}  // namespace qq
