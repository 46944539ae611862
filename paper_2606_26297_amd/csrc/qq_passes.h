// qq_passes.h -- complex64 tile-pass bodies specialised per pass kind.
//
// Each pass streams a tile of 2^12 amplitudes per workgroup through registers
// (256 threads x 16 amplitudes; three 4-bit register groups rotated by LDS
// transposes), with the operation sequence, the layouts and the qubit-set
// geometry fixed at compile time so the register allocator sees one
// straight-line program.  Used by the per-pass kernels (one launch per pass)
// and by the persistent many-problem kernel (one work item per tile chunk).
//
// Mixer in factored form.  RX(2 beta) = cos(beta) I - i sin(beta) X is
// applied as sigma * M with
//     M = I - i t X,  t = tan(beta)        when |cos| >= |sin|   ("form A"),
//     M = u I - i X,  u = cot(beta)        otherwise             ("form B"),
// so each output component is one FMA.  t (or u) is rounded to float once and
// sigma = +-1/sqrt(1 + t^2) is computed in FP64 from the rounded value, which
// keeps sigma*M exactly unitary up to the final float rounding of
// sigma^(number of mixed qubits), applied once per mixer operation.  The
// inverse rotation flips the sign of t (form A) or of u and sigma (form B).
//
// d E / d beta_k = 2 Im sum_q <lambda|X_q|psi> is accumulated per register
// group as sum_r Im(conj(lambda_r) * sum_{q in group} psi_{r xor q}): FP32
// products over the 16 registers of a thread, added to FP64 accumulators.
#pragma once

#include <type_traits>

#include "qq_device.h"

namespace qq {
namespace passes {

using namespace dev;

// exp(-i theta) for theta = gamma C: w = (gamma / 2 pi) C in FP64 (revolutions), reduced
// to u = w - rint(w) in [-1/2, 1/2] in FP64, then the gfx950 hardware sine and cosine
// (argument in revolutions) on float(u).
__device__ __forceinline__ void phase_rev(double g2pi, double cz, float &c, float &s)
{
    const double w = g2pi * cz;
    const float u = (float)(w - rint(w));
    s = __builtin_amdgcn_sinf(u);
    c = __builtin_amdgcn_cosf(u);
}

// Scheduling fence after every 4th register of a loop that reads the cost
// diagonal: bounds how many FP64 loads and their consumers are in flight.
#define QQ_CHUNK_FENCE(r)                                   \
    if (((r) & 3) == 3) __builtin_amdgcn_sched_barrier(0)

// Global-memory access through a wave-uniform 64-bit base and a 32-bit per-thread offset.
// voff: a 32-bit per-lane byte offset (scalar base + vector offset addressing), or 64-bit where
// a lane's offset can reach 4 GiB (the strided layout of the highest qubit runs at n >= 32).
template <typename T, typename O = uint32_t>
__device__ __forceinline__ T gld(uint64_t sbase, O voff)
{
    if constexpr (std::is_same<T, float2>::value) {
        // state amplitudes are streamed once per pass: non-temporal
        const uint64_t u =
            __builtin_nontemporal_load(reinterpret_cast<const uint64_t __attribute__((address_space(1))) *>(sbase + voff));
        return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
    } else {
        return *reinterpret_cast<const T __attribute__((address_space(1))) *>(sbase + voff);
    }
}
template <typename O = uint32_t>
__device__ __forceinline__ void gst(uint64_t sbase, O voff, float2 x)
{
    const uint64_t u = (uint64_t)__float_as_uint(x.x) | ((uint64_t)__float_as_uint(x.y) << 32);
    __builtin_nontemporal_store(u, reinterpret_cast<uint64_t __attribute__((address_space(1))) *>(sbase + voff));
}

// Two registers through one 16-byte access per lane.  In the thread layouts qubit 0 is lane bit 0, so
// the two lanes of a lane pair hold neighbouring amplitudes: for registers (r, r + 1) the even lane
// accesses register r's amplitudes z and z + 1, the odd lane register r + 1's, and one swap of 8 bytes
// between the two lanes gives each lane its own two values (loads) or the pair its 16 bytes (stores).
// Half the address work and wider transfers for the same bytes.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_swap(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xb1, 0xf, 0xf, false);  // quad_perm [1, 0, 3, 2]
}

template <typename O>
__device__ __forceinline__ void gld_pair(uint64_t sbase, O voff, uint32_t odd, float2 &lo, float2 &hi)
{
    const u32x4 l =
        __builtin_nontemporal_load(reinterpret_cast<const u32x4 __attribute__((address_space(1))) *>(sbase + voff));
    // even lane: (r at z, r at z + 1), keeps the first, sends the second; odd lane: (r + 1 at z - 1, r + 1
    // at z), keeps the second, sends the first
    const uint32_t rx = lane_swap(odd ? l.x : l.z), ry = lane_swap(odd ? l.y : l.w);
    lo = odd ? make_float2(__uint_as_float(rx), __uint_as_float(ry)) : make_float2(__uint_as_float(l.x), __uint_as_float(l.y));
    hi = odd ? make_float2(__uint_as_float(l.z), __uint_as_float(l.w)) : make_float2(__uint_as_float(rx), __uint_as_float(ry));
}

template <typename O>
__device__ __forceinline__ void gst_pair(uint64_t sbase, O voff, uint32_t odd, float2 lo, float2 hi)
{
    const float2 snd = odd ? lo : hi;
    const uint32_t rx = lane_swap(__float_as_uint(snd.x)), ry = lane_swap(__float_as_uint(snd.y));
    u32x4 o;
    o.x = odd ? rx : __float_as_uint(lo.x);
    o.y = odd ? ry : __float_as_uint(lo.y);
    o.z = odd ? __float_as_uint(hi.x) : rx;
    o.w = odd ? __float_as_uint(hi.y) : ry;
    __builtin_nontemporal_store(o, reinterpret_cast<u32x4 __attribute__((address_space(1))) *>(sbase + voff));
}
// A wave-uniform value the optimiser must treat as unknown at this point (keeps
// uses inside the loop).  The read-first-lane is free for a value already in
// scalar registers and makes the scalar constraint legal where the compiler
// cannot prove uniformity itself.
__device__ __forceinline__ uint64_t opaque_u64(uint64_t x)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return ((uint64_t)hi << 32) | lo;
}

// Cost values of a thread's 16 registers from five loads of the diagonal.  C is quadratic in the
// bits of z (eq. (6)), so over the 4-cube of the register qubits R_0..R_3 above the thread's
// register-0 element z0,
//   C(z0 + sum_{j in r} 2^R_j) = C(z0) + sum_{j in r} [C(z0 + 2^R_j) - C(z0)] + sum_{j<k in r} b_{R_j R_k},
// and the last sum does not depend on z0.  cq[r] = sum_{k in r, k > j} b_{R_j R_k}, j the lowest
// bit of r, so C at register r follows from C at r - 2^j in two additions.  Exact for integer
// costs; for real ones within a few units in the last place of the stored values.  The loads read
// 5/16 of the diagonal bytes the pass would otherwise read.
using RegQ = const double __attribute__((address_space(4)));
struct RegCost {
    double v[16];  // entries are formed in ascending register order; only those still needed stay live
    double k[4];   // C(z0 + 2^R_j) - C(z0)
};

template <typename DT, typename O>
__device__ __forceinline__ void reg_cost_load(RegCost &c, uint64_t diag_a, uint64_t b, uint64_t rs, O vd)
{
    c.v[0] = (double)gld<DT>(diag_a + b * sizeof(DT), vd);
#pragma unroll
    for (int j = 0; j < 4; ++j) c.v[1 << j] = (double)gld<DT>(diag_a + (b + (rs << j)) * sizeof(DT), vd);
#pragma unroll
    for (int j = 0; j < 4; ++j) c.k[j] = c.v[1 << j] - c.v[0];
}

__device__ __forceinline__ double reg_cost(RegCost &c, RegQ *cq, int r)
{
    if ((r & (r - 1)) == 0) return c.v[r];
    const int j = __builtin_ctz(r);
    c.v[r] = (c.v[r - (1 << j)] + c.k[j]) + cq[r];
    return c.v[r];
}

// Cost values of a thread's 16 registers from the pass's per-tile table, without reading the cost
// diagonal.  C is quadratic (eq. (6)): with z0 = T + E, T the tile's base bits and E the thread's own
// bits (qubits 0..3, two lane and two wave qubits, in the order of the thread index t),
//   C(z0) = C(T) + P(E) + sum_{q in E} G_q(T),   G_q(T) = sum_{i in T} b_iq,
//   P(E) = sum_{j in E} l_j + sum_{j<k in E} b_jk,
// and the increment of register qubit R_j is C(z0 + 2^R_j) - C(z0) = G_Rj(T) + l_Rj + sum_{q in E} b_q,Rj.
// The table row holds C(T) plus the lane bits' sum per lane, the wave bits' sum per wave and the four
// G_Rj(T); the thread's P(E) and l_Rj + sum_{q in E} b_q,Rj are per-thread constants (thr, 8 doubles).
// Exact for integer costs; for real ones within a few units in the last place of the diagonal's
// canonical sums.

// The values one tile's formation reads: the lane's and the wave's entries and the four register
// increments of the row (wave-uniform, read through the constant address space so they take scalar
// loads), the thread's five constants.
struct TabVals {
    double lane, wave, reg[4], thr[5];
};

using cdouble_t = const __attribute__((address_space(4))) double;

__device__ __forceinline__ void tab_load(TabVals &tv, const double *row, const double *thr, int t, uint32_t wave)
{
    cdouble_t *u = (cdouble_t *)row;
    tv.lane = row[t & 63];
    tv.wave = u[64 + wave];
#pragma unroll
    for (int j = 0; j < 4; ++j) tv.reg[j] = u[68 + j];
#pragma unroll
    for (int j = 0; j < 5; ++j) tv.thr[j] = thr[j];
}

__device__ __forceinline__ void reg_cost_form(RegCost &c, const TabVals &tv)
{
    const double z = (tv.lane + tv.wave) + tv.thr[0];
    c.v[0] = z;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        c.k[j] = tv.reg[j] + tv.thr[1 + j];
        c.v[1 << j] = z + c.k[j];
    }
}

struct MixCoef {
    float m;      // t (form A) or u (form B), direction folded in
    int formB;
    float scale;  // sigma^(active qubits), applied after the operation
    double sig2;  // sigma^2
};

__device__ __forceinline__ MixCoef mix_coef(double beta, bool inverse, int nact)
{
    double s, c;
    sincos(beta, &s, &c);
    MixCoef r;
    double sigma;
    if (fabs(c) >= fabs(s)) {
        const float t = (float)(s / c);
        r.formB = 0;
        r.m = inverse ? -t : t;
        sigma = copysign(1.0, c) / sqrt(fma((double)t, (double)t, 1.0));
    } else {
        const float u = (float)(c / s);
        r.formB = 1;
        r.m = inverse ? -u : u;
        sigma = copysign(1.0, s) / sqrt(fma((double)u, (double)u, 1.0));
        if (inverse) sigma = -sigma;
    }
    r.sig2 = sigma * sigma;
    double sc = 1.0;
    for (int i = 0; i < nact; ++i) sc *= sigma;
    r.scale = (float)sc;
    return r;
}

// Scheduling fences between butterfly stages keep the stages in place (each
// stage is in-register and needs no temporaries); without them the scheduler
// interleaves stages and the register demand grows past the occupancy target.
#define QQ_STAGE_FENCE() __builtin_amdgcn_sched_barrier(0)

// Butterfly of bit K: form A  (a, b) -> (a - i t b, b - i t a);
//                     form B  (a, b) -> (u a - i b, u b - i a).
template <int K, bool FB>
__device__ __forceinline__ void bf(float2 (&v)[kRegs], float m)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if (r & (1 << K)) continue;
        const float2 a = v[r], b = v[r | (1 << K)];
        if constexpr (FB) {
            v[r] = make_float2(fmaf(m, a.x, b.y), fmaf(m, a.y, -b.x));
            v[r | (1 << K)] = make_float2(fmaf(m, b.x, a.y), fmaf(m, b.y, -a.x));
        } else {
            v[r] = make_float2(fmaf(m, b.y, a.x), fmaf(-m, b.x, a.y));
            v[r | (1 << K)] = make_float2(fmaf(m, a.y, b.x), fmaf(-m, a.x, b.y));
        }
    }
}

template <bool FB>
__device__ __forceinline__ void group_mix(float2 (&v)[kRegs], int mask, float m)
{
    if (mask & 1) bf<0, FB>(v, m);
    QQ_STAGE_FENCE();
    if (mask & 2) bf<1, FB>(v, m);
    QQ_STAGE_FENCE();
    if (mask & 4) bf<2, FB>(v, m);
    QQ_STAGE_FENCE();
    if (mask & 8) bf<3, FB>(v, m);
    QQ_STAGE_FENCE();
}

// sum over the active bits K of the group and the register pairs (r, r | 2^K) of
// Im(conj(l_r) a_{r|2^K} + conj(l_{r|2^K}) a_r)  =  sum_K Im <l| X_K |a>  restricted to the thread's registers.
template <int K>
__device__ __forceinline__ float xexp_bit(const float2 (&a)[kRegs], const float2 (&l)[kRegs], float acc)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if (r & (1 << K)) continue;
        const int q = r | (1 << K);
        acc = fmaf(l[r].x, a[q].y, acc);
        acc = fmaf(-l[r].y, a[q].x, acc);
        acc = fmaf(l[q].x, a[r].y, acc);
        acc = fmaf(-l[q].y, a[r].x, acc);
    }
    return acc;
}

__device__ __forceinline__ float xexp_group(const float2 (&a)[kRegs], const float2 (&l)[kRegs], int mask)
{
    float acc = 0.0f;
    if (mask & 1) acc = xexp_bit<0>(a, l, acc);
    QQ_STAGE_FENCE();
    if (mask & 2) acc = xexp_bit<1>(a, l, acc);
    QQ_STAGE_FENCE();
    if (mask & 4) acc = xexp_bit<2>(a, l, acc);
    QQ_STAGE_FENCE();
    if (mask & 8) acc = xexp_bit<3>(a, l, acc);
    QQ_STAGE_FENCE();
    return acc;
}

// Sets with inactive tile bits use the general butterfly (a, b) -> (p a - i q b, p b - i q a)
// on every bit, with (p, q) = (1, t) (form A) or (u, 1) (form B) on active bits and the
// identity (1, 0) on inactive ones: branch-free, so the register demand stays that of a
// full set, at one extra multiply per output component.
template <int K>
__device__ __forceinline__ void bfg(float2 (&v)[kRegs], float p, float q)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if (r & (1 << K)) continue;
        const float2 a = v[r], b = v[r | (1 << K)];
        v[r] = make_float2(fmaf(p, a.x, q * b.y), fmaf(p, a.y, -(q * b.x)));
        v[r | (1 << K)] = make_float2(fmaf(p, b.x, q * a.y), fmaf(p, b.y, -(q * a.x)));
    }
}

__device__ __forceinline__ void group_mix_pb(float2 (&v)[kRegs], int mask, float pa, float qa)
{
    bfg<0>(v, (mask & 1) ? pa : 1.0f, (mask & 1) ? qa : 0.0f);
    QQ_STAGE_FENCE();
    bfg<1>(v, (mask & 2) ? pa : 1.0f, (mask & 2) ? qa : 0.0f);
    QQ_STAGE_FENCE();
    bfg<2>(v, (mask & 4) ? pa : 1.0f, (mask & 4) ? qa : 0.0f);
    QQ_STAGE_FENCE();
    bfg<3>(v, (mask & 8) ? pa : 1.0f, (mask & 8) ? qa : 0.0f);
    QQ_STAGE_FENCE();
}

// xexp_group over the active bits of `mask` only, without branches.
__device__ __forceinline__ float xexp_group_pb(const float2 (&a)[kRegs], const float2 (&l)[kRegs], int mask)
{
    float acc = 0.0f;
    acc = fmaf((mask & 1) ? 1.0f : 0.0f, xexp_bit<0>(a, l, 0.0f), acc);
    QQ_STAGE_FENCE();
    acc = fmaf((mask & 2) ? 1.0f : 0.0f, xexp_bit<1>(a, l, 0.0f), acc);
    QQ_STAGE_FENCE();
    acc = fmaf((mask & 4) ? 1.0f : 0.0f, xexp_bit<2>(a, l, 0.0f), acc);
    QQ_STAGE_FENCE();
    acc = fmaf((mask & 8) ? 1.0f : 0.0f, xexp_bit<3>(a, l, 0.0f), acc);
    QQ_STAGE_FENCE();
    return acc;
}

template <int FROM, int TO>
__device__ __forceinline__ void xpose(float2 *lds, float2 (&v)[kRegs], int t)
{
    __syncthreads();
    lds_put<FROM>(lds, v, t, 0);
    __syncthreads();
    lds_get<TO>(lds, v, t, 0);
}

// Live states: ST bit 0 = psi (v[0]), bit 1 = lambda (v[1]).
template <int FROM, int TO, int NS, int ST>
__device__ __forceinline__ void xpose_all(float2 *lds, float2 (&v)[NS][kRegs], int t)
{
    if constexpr (ST & 1) xpose<FROM, TO>(lds, v[0], t);
    if constexpr (NS > 1 && (ST & 2)) xpose<FROM, TO>(lds, v[NS - 1], t);
}

template <int NS, int ST>
__device__ __forceinline__ void scale_all(float2 (&v)[NS][kRegs], float s)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if constexpr (ST & 1) v[0][r] = make_float2(v[0][r].x * s, v[0][r].y * s);
        if constexpr (NS > 1 && (ST & 2)) v[NS - 1][r] = make_float2(v[NS - 1][r].x * s, v[NS - 1][r].y * s);
    }
}

// x^k for 0 <= k < 16 without a loop (a loop here would split the straight-line
// tile body and raise its register demand).
__device__ __forceinline__ double pow_small(double x, int k)
{
    double r = (k & 1) ? x : 1.0;
    x *= x;
    r = (k & 2) ? r * x : r;
    x *= x;
    r = (k & 4) ? r * x : r;
    x *= x;
    return (k & 8) ? r * x : r;
}

// One mixer operation on the active tile bits, starting in layout FROM (2 or 1)
// and ending in the other one.  GB: accumulate sum_q Im<lambda|X_q|psi> (both states
// live); each group's partial is taken before its butterflies and rescaled by
// sigma^(2 done), where done = bits already mixed by the unnormalised factor M.
template <bool HIGH, bool FULL, int FROM, int NS, int ST, bool GB, bool FB>
__device__ __forceinline__ void mix_op(float2 *lds, float2 (&v)[NS][kRegs], int t, int active, const MixCoef &c,
                                       double &gacc)
{
    // FULL: every bit of the set's register groups is active (compile-time masks);
    // otherwise the general butterfly covers both forms (FB is not used).
    // Partial sets: the mask and the general-butterfly coefficients are made opaque
    // scalars here, so the per-bit coefficient selects are formed in scalar
    // registers at each use instead of hoisted out of the tile loop into vector ones.
    int am = active;
    float pa = 1.0f, qa = 0.0f;
    if constexpr (!FULL) {
        am = __builtin_amdgcn_readfirstlane(active);
        pa = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.formB ? c.m : 1.0f)));
        qa = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.formB ? 1.0f : c.m)));
        asm volatile("" : "+s"(am), "+s"(pa), "+s"(qa));
    }
    const int m0 = FULL ? (HIGH ? 0 : 15) : (am & 15);
    const int m1 = FULL ? 15 : ((am >> 4) & 15);
    const int m2 = FULL ? 15 : ((am >> 8) & 15);
    int done = 0;
    auto group = [&](int mask) {
        if constexpr (GB) {
            const float x = FULL ? xexp_group(v[0], v[1], mask) : xexp_group_pb(v[0], v[1], mask);
            gacc = fma((double)x, pow_small(c.sig2, done), gacc);
        }
        if constexpr (FULL) {
            if constexpr (ST & 1) group_mix<FB>(v[0], mask, c.m);
            if constexpr (NS > 1 && (ST & 2)) group_mix<FB>(v[NS - 1], mask, c.m);
        } else {
            if constexpr (ST & 1) group_mix_pb(v[0], mask, pa, qa);
            if constexpr (NS > 1 && (ST & 2)) group_mix_pb(v[NS - 1], mask, pa, qa);
        }
        done += __popc(mask);
    };
    if constexpr (!HIGH) {
        if constexpr (FROM == 2) {
            group(m2);
            xpose_all<2, 0, NS, ST>(lds, v, t);
            group(m0);
            xpose_all<0, 1, NS, ST>(lds, v, t);
            group(m1);
        } else {
            group(m1);
            xpose_all<1, 0, NS, ST>(lds, v, t);
            group(m0);
            xpose_all<0, 2, NS, ST>(lds, v, t);
            group(m2);
        }
    } else {
        if constexpr (FROM == 2) {
            group(m2);
            xpose_all<2, 1, NS, ST>(lds, v, t);
            group(m1);
        } else {
            group(m1);
            xpose_all<1, 2, NS, ST>(lds, v, t);
            group(m2);
        }
    }
    scale_all<NS, ST>(v, c.scale);
}

// Pass kinds (FastPassKind):
//   FK_FIRST  init, phase(0), mix(0)                                         -> psi
//   FK_MID    psi: mix(k)                                                    -> psi
//   FK_TURN   psi: mix(k), phase(k+1), mix(k+1)                              -> psi
//   FK_LAST   psi: mix(k), energy                                            (-> psi)
//   FK_LASTG  psi: mix(k), energy, lambda = C psi, unmix(k) + g_beta(k)      -> lambda
//   FK_BMID   psi, lambda: unmix(k) + g_beta(k)                              -> psi, lambda
//   FK_BTURN  psi, lambda: unmix(k) + g_beta(k), g_gamma(k), unphase(k), unmix(k-1) + g_beta(k-1)
//   FK_BLAST  psi, lambda: unmix(0) + g_beta(0), g_gamma(0)

struct FastArgs {
    int B, G, p, k;
    uint64_t tiles;
    uint64_t dim_mask;
    int pos4, pos8, w1, w2, active, nact;
    int store_psi;
    int slot_base, slot_stride;
    double amp0;
    const double *params;
    const void *diag;
    float2 *psi;
    float2 *lam;
    uint64_t state_stride;
    double *partial;
    int blocked;           // 0: tiles g, g + G, ... ; 1: tiles [g T/G, (g + 1) T/G) (T a multiple of G)
    const PartDesc *part;  // partitioned phases (PART bodies only)
    const void *tables;    // packed per-QPU local tables
    const double *cq;      // 16 pair sums of the register qubits of the layout the diagonal is read in
    const double *pcq;     // partitioned: pair sums of every factor, [factor][run start][16]
    // Centre of the cost for the accumulations: the energy, the adjoint seed lambda = (C - shift) psi
    // and the gamma-derivatives use C - shift (the mean of C), which leaves the gradient unchanged
    // (the seed's shift part is real and cancels) and keeps the complex64 terms at the scale of the
    // spread of C instead of its offset; the phases use C itself.  The reduction adds shift back to
    // the energy.
    double shift;
    int pcq_runs;          // run starts per factor (n - 3)
    // Cost table of the layout in which the pass reads the cost: ctab[tile][kCostRow] (per-lane,
    // per-wave and per-register parts of the tile's base-bit sums, see launch_cost_table) and
    // cthr[thread][8], the thread's own part (see reg_cost_form).
    const double *ctab;
    const double *cthr;
    // the same for the cross-QPU couplings alone (partitioned phases)
    const double *xtab;
    const double *xthr;
    // 0: psi and lambda are separate arrays; K > 0: their blocks of 2^K amplitudes alternate (lambda's
    // block right after psi's), so index bit q >= K of a state sits at address bit q + 1
    int ilv;
};

// ---- partitioned phase (eq. (16)) --------------------------------------------------------------
// The cost splits into per-QPU local parts C_m, each a function of that QPU's variables only (table
// m is indexed by those bits in ascending variable order), and the cross part C_x (a quadratic form
// over all of z, formed from its per-tile table).  The phase is applied as the product of
// exp(-i gamma C_m), m = 0..M-1, and exp(-i gamma C_x), each argument reduced on its own.  Table
// index of amplitude z for QPU m: the bits of z on the QPU's variables, gathered in order.  The
// gather is additive over disjoint bit sets, so for z = zb | e | (register bits) it is gather(zb)
// (per tile, scalar) + gather(e) (per lane) + the register bits' contributions (scalar, one per
// register bit).

// 2^(rank of qubit q among the QPU's variables) if q is on the QPU, else 0.
__device__ __forceinline__ uint32_t part_contrib(uint64_t vmask, int q)
{
    return ((vmask >> q) & 1ull) ? (1u << __popcll(vmask & ((1ull << q) - 1ull))) : 0u;
}

// Gather of the bits of zb on the QPU's variables (wave-uniform), without a loop over the
// variables (a data-dependent loop here would split the tile body and raise its register demand):
// the compress method of Hacker's Delight (sec. 7-4), six fixed steps that move each selected bit
// right by the number of unselected mask positions below it, one bit of that count per step.
__device__ __forceinline__ uint32_t part_gather(uint64_t zb, uint64_t vmask)
{
    uint64_t x = zb & vmask, m = vmask;
    uint64_t mk = ~m << 1;  // positions whose count of zeros below them is still to be moved
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        uint64_t mp = mk ^ (mk << 1);  // prefix parity of mk: odd count of mk bits at or below
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        mp ^= mp << 32;
        const uint64_t mv = mp & m;  // mask bits that move by 2^i in this step
        m = (m ^ mv) | (mv >> (1 << i));
        const uint64_t t = x & mv;
        x = (x ^ t) | (t >> (1 << i));
        mk &= ~mp;
    }
    return (uint32_t)x;
}

// The phase of the partitioned cost for this thread's 16 registers, as angles in revolutions:
// uf[r] = (gamma / 2 pi) times the FP64 sum over the local factors and the cross factor of C_m(z),
// reduced in FP64 to [-1/2, 1/2] and rounded to float (the product of the factors as one rotation).
// Layout: lanes hold qubits 0..3 (lane_lo) and qh, qh + 1 (lane_hi); registers hold qubits
// qr..qr+3; zb is the tile's wave-uniform first index, `tile` its index in the pass's table.  Every
// factor is quadratic in z, so its 16 register values follow from its value at register 0, its four
// single-bit increments and its pair sums among the register qubits (a.pcq, laid out
// [factor][run start][16], the cross factor last): five reads of a local table, or for the cross
// factor its per-tile table (as reg_cost_form).  The angles do not depend on the state, so a pass
// can form them before it loads any amplitude.
template <typename DT>
__device__ __forceinline__ void part_angles(float (&uf)[kRegs], const FastArgs &a, double g2pi, uint64_t zb,
                                            uint32_t lane_lo, uint32_t lane_hi, int qh, int qr, uint64_t tile, int t)
{
    // registers in two halves of 8, so the FP64 sums take 16 VGPRs, not 32
    constexpr int H = kRegs / 2;
    // opaque here, so the masks and lane tests derived from them are formed per tile instead of
    // hoisted out of the tile loop (where they would hold dozens of scalar registers throughout)
    asm volatile("" : "+s"(qh), "+s"(qr), "+v"(lane_lo), "+v"(lane_hi));
    const int M = a.part->nparts;
    const DT *tables = static_cast<const DT *>(a.tables);
    RegQ *pcq = (RegQ *)a.pcq;
    // the cross factor's table row and per-thread constants
    const double *xrow = a.xtab + tile * kCostRow;
    const double *xth = a.xthr + 8 * t;
    cdouble_t *xu = (cdouble_t *)xrow;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(t >> 6);
    // one factor's value at register 0 of half h (v0) and its four register increments k -> its 8
    // register values of half h, added to the FP64 sums u of the factors' values
    auto add_factor = [&](double v0, const double (&k)[4], RegQ *w, int h, double (&u)[H], bool first) {
        double v[H];
        v[0] = v0;
#pragma unroll
        for (int i = 1; i < H; ++i) {
            const int j = __builtin_ctz(i);
            v[i] = (v[i - (1 << j)] + k[j]) + w[h * H + i];
        }
#pragma unroll
        for (int i = 0; i < H; ++i) u[i] = first ? v[i] : u[i] + v[i];
    };
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double u[H];
        {
            double k[4];
            const double z0 = (xrow[t & 63] + xu[64 + wave]) + xth[0];
#pragma unroll
            for (int j = 0; j < 4; ++j) k[j] = xu[68 + j] + xth[1 + j];
            add_factor(h ? z0 + k[3] : z0, k, pcq + ((size_t)M * a.pcq_runs + qr) * kRegs, h, u, true);
        }
        for (int m = 0; m < M; ++m) {
            const uint64_t vm = a.part->vmask[m];
            const uint64_t tab = (uint64_t)(tables + a.part->table_off[m]);
            uint32_t L = part_gather(zb, vm);
#pragma unroll
            for (int j = 0; j < 4; ++j) L += ((lane_lo >> j) & 1u) ? part_contrib(vm, j) : 0u;
            L += (lane_hi & 1u) ? part_contrib(vm, qh) : 0u;
            L += (lane_hi & 2u) ? part_contrib(vm, qh + 1) : 0u;
            double e[5];
            e[0] = (double)gld<DT>(tab, L * (uint32_t)sizeof(DT));
#pragma unroll
            for (int j = 0; j < 4; ++j)
                e[j + 1] = (double)gld<DT>(tab, (L + part_contrib(vm, qr + j)) * (uint32_t)sizeof(DT));
            double k[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) k[j] = e[j + 1] - e[0];
            add_factor(h ? e[4] : e[0], k, pcq + ((size_t)m * a.pcq_runs + qr) * kRegs, h, u, false);
        }
        // one argument per amplitude: (gamma / 2 pi) times the sum of the factors' values, reduced
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double x = g2pi * u[i];
            uf[h * H + i] = (float)(x - rint(x));
        }
    }
}

// Multiply the states ST (bit 0 psi, bit 1 lambda) by exp(-+ 2 pi i uf[r]) (INV: the inverse).
template <int NS, int ST, bool INV>
__device__ __forceinline__ void apply_angles(float2 (&v)[NS][kRegs], const float (&uf)[kRegs])
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const float c = __builtin_amdgcn_cosf(uf[r]);
        const float s = INV ? -__builtin_amdgcn_sinf(uf[r]) : __builtin_amdgcn_sinf(uf[r]);
        if constexpr (ST & 1) rot_phase<float>(v[0][r], c, s);
        if constexpr (NS > 1 && (ST & 2)) rot_phase<float>(v[NS - 1][r], c, s);
    }
}

template <int KIND>
constexpr int kind_states()
{
    return KIND >= FK_LASTG ? 2 : 1;
}
template <int KIND>
constexpr int kind_slots()
{
    return KIND == FK_LAST ? 1 : KIND == FK_LASTG ? 2 : KIND == FK_BMID ? 1 : KIND == FK_BTURN ? 3
           : KIND == FK_BLAST ? 2 : 0;
}

// The tile loop of one pass kind.  FB1 / FB2: form of the first / second mixer coefficient.
template <int KIND, bool HIGH, bool FULL, typename DT, bool PART, bool WIDE, bool FB1, bool FB2, bool CT, bool PR>
__device__ __forceinline__ void pass_body(const FastArgs &a, float2 *lds, double (&acc)[3], int t, int b, int g,
                                          const MixCoef &c1, const MixCoef &c2, double g2pi)
{
    constexpr int NS = kind_states<KIND>();
    // CT: cost values from the per-tile tables (passes that read the cost, non-partitioned phases)
    constexpr bool TAB = CT && !PART && KIND != FK_MID && KIND != FK_BMID;
    // Global addressing.  Tile-local bits 0..3 and the two lane bits above them
    // vary per thread (a 32-bit byte offset); the two wave bits and the four
    // register bits are wave-uniform and go into a 64-bit scalar base per register.
    //   layout 2: lanes -> qubits 0..3, pos4, pos4+1; waves -> pos4+2, pos4+3; registers -> pos8..pos8+3
    //   layout 1: lanes -> qubits 0..3, pos8, pos8+1; waves -> pos8+2, pos8+3; registers -> pos4..pos4+3
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(t >> 6);
    const uint32_t lane_lo = t & 15, lane_hi = (t >> 4) & 3;
    // WIDE: the layout-1 lane offsets (lane bits on qubits pos8, pos8 + 1) need 64 bits
    using O1 = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    // index offsets (the cost diagonal, the partitioned gathers) and state address offsets: with
    // interleaved psi / lambda blocks (a.ilv = K) a run of four qubits at q >= K sits at q + 1 (no run
    // straddles K)
    const int K = a.ilv;
    const int s4 = a.pos4 + (K && a.pos4 >= K), s8 = a.pos8 + (K && a.pos8 >= K);
    const uint32_t e2 = lane_lo + (lane_hi << a.pos4);
    const O1 e1 = (O1)lane_lo + ((O1)lane_hi << a.pos8);
    const uint32_t vs2 = (lane_lo + (lane_hi << s4)) * (uint32_t)sizeof(float2), vd2 = e2 * (uint32_t)sizeof(DT);
    const O1 vs1 = ((O1)lane_lo + ((O1)lane_hi << s8)) * (O1)sizeof(float2), vd1 = e1 * (O1)sizeof(DT);
    const uint64_t w2 = (uint64_t)wave << (a.pos4 + 2), w1 = (uint64_t)wave << (a.pos8 + 2);
    const uint64_t sw2 = (uint64_t)wave << (s4 + 2), sw1 = (uint64_t)wave << (s8 + 2);
    // PAIR: state accesses by register pairs (gld_pair / gst_pair); the odd lane's offset is the even
    // lane's plus one register stride (layout 2: registers at s8, layout 1: at s4), within 32 bits
    // wherever the lane offsets are (not WIDE).  Measured at n = 28, B = 64: mid 45.2 -> 43.7 ms,
    // adjoint mid 90.7 -> 87.8, last with the seed 52.0 -> 50.5, but the adjoint turn on the high sets
    // 94.0 / 95.4 -> 99 / 102.5 and the turn mixed (one set faster, one slower): so the 12-qubit set's
    // passes and the last pass take them, the other high-set passes keep 8-byte accesses.  PR = false:
    // never (the persistent launch: 22.0 -> 23.2 ms on the uneven batch with them)
    constexpr bool PAIR = PR && !WIDE && !PART && (!HIGH || KIND == FK_LASTG);
    const uint32_t odd = PAIR ? lane_lo & 1u : 0u;
    const uint32_t pv2 = PAIR ? vs2 - 8u * odd + odd * (uint32_t)(8ull << s8) : 0u;
    const O1 pv1 = PAIR ? vs1 - (O1)(8u * odd) + (O1)odd * (O1)(8ull << s4) : (O1)0;
    const uint64_t psi_a = (uint64_t)(a.psi + (size_t)b * a.state_stride);
    const uint64_t lam_a = (uint64_t)(a.lam + (size_t)b * a.state_stride);
    const uint64_t diag_a = (uint64_t)a.diag;
    float2 v[NS][kRegs];

    // tile order: strided (workgroups that run together take neighbouring tiles) or blocked
    // (each workgroup takes a contiguous range, so concurrently running ones are far apart)
    uint64_t t_begin = (uint64_t)g, t_end = a.tiles, t_step = (uint64_t)a.G;
    if (a.blocked) {
        const uint64_t per = a.tiles / (uint64_t)a.G;
        t_begin = (uint64_t)g * per;
        t_end = t_begin + per;
        t_step = 1;
    }
    for (uint64_t tile = t_begin; tile < t_end; tile += t_step) {
        uint64_t base;
        if constexpr (HIGH) base = tile_base(tile, a.pos4, a.pos8, a.w1, a.w2);
        else base = tile << kTileBits;
        // register strides, opaque per tile so their multiples are formed in scalar
        // registers at each use rather than hoisted out of the loop (rs: index, ss: state address)
        const uint64_t rs2 = opaque_u64(1ull << a.pos8), rs1 = opaque_u64(1ull << a.pos4);
        const uint64_t b2 = base + w2, b1 = base + w1;
        const uint64_t sbase = K ? (base & ((1ull << K) - 1)) | ((base >> K) << (K + 1)) : base;
        const uint64_t ss2 = opaque_u64(1ull << s8), ss1 = opaque_u64(1ull << s4);
        const uint64_t sb2 = sbase + sw2, sb1 = sbase + sw1;
        RegQ *cq = (RegQ *)a.cq;
        // cost values of the thread's registers in layout 2 / layout 1: five loads of the diagonal, or
        // (TAB) the load of the tile's table row, with the values formed by cz_ready before their use
        TabVals tv;
        auto tab_issue = [&]() { tab_load(tv, a.ctab + tile * kCostRow, a.cthr + 8 * t, t, wave); };
        auto cz2 = [&](RegCost &rc) {
            if constexpr (TAB) tab_issue();
            else reg_cost_load<DT>(rc, diag_a, b2, rs2, vd2);
        };
        auto cz1 = [&](RegCost &rc) {
            if constexpr (TAB) tab_issue();
            else reg_cost_load<DT>(rc, diag_a, b1, rs1, vd1);
        };
        auto cz_ready = [&](RegCost &rc) {
            if constexpr (TAB) reg_cost_form(rc, tv);
        };
        auto ld2 = [&](uint64_t arr, int r) { return gld<float2>(arr + (sb2 + r * ss2) * 8, vs2); };
        // stores take their own opaque copy of the stride: sharing the load addresses
        // would keep 16-32 scalar address pairs live across the whole tile
        auto st2f = [&](uint64_t arr, int r, float2 x, uint64_t ss) { gst(arr + (sb2 + r * ss) * 8, vs2, x); };
        auto st1f = [&](uint64_t arr, int r, float2 x, uint64_t ss) { gst(arr + (sb1 + r * ss) * 8, vs1, x); };
        // all 16 registers of one state: loads in layout 2, stores in layout 2 / layout 1
        auto ld2all = [&](uint64_t arr, float2 (&x)[kRegs]) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) gld_pair(arr + (sb2 + q * ss2) * 8, pv2, odd, x[q], x[q + 1]);
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) x[r] = ld2(arr, r);
            }
        };
        auto st2all = [&](uint64_t arr, const float2 (&x)[kRegs], uint64_t ss) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) gst_pair(arr + (sb2 + q * ss) * 8, pv2, odd, x[q], x[q + 1]);
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) st2f(arr, r, x[r], ss);
            }
        };
        // psi and lambda together, register by register (pairs of registers with PAIR)
        auto ld2both = [&](float2 (&x)[kRegs], float2 (&y)[kRegs]) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) {
                    gld_pair(psi_a + (sb2 + q * ss2) * 8, pv2, odd, x[q], x[q + 1]);
                    gld_pair(lam_a + (sb2 + q * ss2) * 8, pv2, odd, y[q], y[q + 1]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    x[r] = ld2(psi_a, r);
                    y[r] = ld2(lam_a, r);
                }
            }
        };
        auto st2both = [&](const float2 (&x)[kRegs], const float2 (&y)[kRegs], uint64_t ss) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) {
                    gst_pair(psi_a + (sb2 + q * ss) * 8, pv2, odd, x[q], x[q + 1]);
                    gst_pair(lam_a + (sb2 + q * ss) * 8, pv2, odd, y[q], y[q + 1]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    st2f(psi_a, r, x[r], ss);
                    st2f(lam_a, r, y[r], ss);
                }
            }
        };
        auto st1both = [&](const float2 (&x)[kRegs], const float2 (&y)[kRegs], uint64_t ss) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) {
                    gst_pair(psi_a + (sb1 + q * ss) * 8, pv1, odd, x[q], x[q + 1]);
                    gst_pair(lam_a + (sb1 + q * ss) * 8, pv1, odd, y[q], y[q + 1]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    st1f(psi_a, r, x[r], ss);
                    st1f(lam_a, r, y[r], ss);
                }
            }
        };
        auto st1all = [&](uint64_t arr, const float2 (&x)[kRegs], uint64_t ss) {
            if constexpr (PAIR) {
#pragma unroll
                for (int q = 0; q < kRegs; q += 2) gst_pair(arr + (sb1 + q * ss) * 8, pv1, odd, x[q], x[q + 1]);
            } else {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) st1f(arr, r, x[r], ss);
            }
        };

        // passes that read the cost after a mixer issue those reads with the state loads, so they
        // are in flight during the mixer (the partitioned adjoint turn, at its register limit, and
        // the first pass, which starts with the phase, read where they use them)
        constexpr bool EARLY = KIND == FK_LAST || KIND == FK_LASTG || KIND == FK_BLAST ||
                               ((KIND == FK_TURN || KIND == FK_BTURN) && !PART);
        RegCost rc;
        if constexpr (KIND == FK_FIRST) {
            if constexpr (PART) {
                float uf[kRegs];
                part_angles<DT>(uf, a, g2pi, b2, lane_lo, lane_hi, a.pos4, a.pos8, tile, t);
#pragma unroll
                for (int r = 0; r < kRegs; ++r) v[0][r] = make_float2((float)a.amp0, 0.0f);
                apply_angles<NS, 1, false>(v, uf);
            } else {
                cz2(rc);
                cz_ready(rc);
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    float c, s;
                    phase_rev(g2pi, reg_cost(rc, cq, r), c, s);
                    v[0][r] = make_float2((float)a.amp0 * c, -(float)a.amp0 * s);
                    QQ_CHUNK_FENCE(r);
                }
            }
            double unused = 0.0;
            mix_op<HIGH, FULL, 2, 1, 1, false, FB1>(lds, v, t, a.active, c1, unused);
            const uint64_t rss = opaque_u64(ss1);
            st1all(psi_a, v[0], rss);
        } else if constexpr (KIND == FK_MID || KIND == FK_TURN || KIND == FK_LAST) {
            ld2all(psi_a, v[0]);
            if constexpr (EARLY) cz1(rc);
            double unused = 0.0;
            mix_op<HIGH, FULL, 2, 1, 1, false, FB1>(lds, v, t, a.active, c1, unused);
            if constexpr (KIND == FK_MID) {
                const uint64_t rss = opaque_u64(ss1);
                st1all(psi_a, v[0], rss);
            } else if constexpr (KIND == FK_TURN) {
                if constexpr (PART) {
                    float uf[kRegs];
                    part_angles<DT>(uf, a, g2pi, b1, lane_lo, lane_hi, a.pos8, a.pos4, tile, t);
                    apply_angles<NS, 1, false>(v, uf);
                } else {
                    if constexpr (!EARLY) cz1(rc);
                    cz_ready(rc);
#pragma unroll
                    for (int r = 0; r < kRegs; ++r) {
                        float c, s;
                        phase_rev(g2pi, reg_cost(rc, cq, r), c, s);
                        rot_phase<float>(v[0][r], c, s);
                        QQ_CHUNK_FENCE(r);
                    }
                }
                mix_op<HIGH, FULL, 1, 1, 1, false, FB2>(lds, v, t, a.active, c2, unused);
                const uint64_t rss = opaque_u64(ss2);
                st2all(psi_a, v[0], rss);
            } else {
                double e = 0.0;
                if constexpr (!EARLY) cz1(rc);
                cz_ready(rc);
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    const float pz = fmaf(v[0][r].x, v[0][r].x, v[0][r].y * v[0][r].y);
                    e = fma((double)pz, reg_cost(rc, cq, r) - a.shift, e);
                    QQ_CHUNK_FENCE(r);
                }
                acc[0] += e;
                if (a.store_psi) {
                    const uint64_t rss = opaque_u64(ss1);
                    st1all(psi_a, v[0], rss);
                }
            }
        } else if constexpr (KIND == FK_LASTG) {
            ld2all(psi_a, v[0]);
            if constexpr (EARLY) cz1(rc);
            double gb = 0.0;
            mix_op<HIGH, FULL, 2, 2, 1, false, FB1>(lds, v, t, a.active, c1, gb);
            cz_ready(rc);
            double e = 0.0;
#pragma unroll
            for (int r = 0; r < kRegs; ++r) {
                const double cz = reg_cost(rc, cq, r) - a.shift;
                const float pz = fmaf(v[0][r].x, v[0][r].x, v[0][r].y * v[0][r].y);
                e = fma((double)pz, cz, e);
                const float cf = (float)cz;
                v[1][r] = make_float2(cf * v[0][r].x, cf * v[0][r].y);
                QQ_CHUNK_FENCE(r);
            }
            acc[0] += e;
            mix_op<HIGH, FULL, 1, 2, 3, true, FB2>(lds, v, t, a.active, c2, gb);
            acc[1] += gb;
            const uint64_t rss = opaque_u64(ss2);
            st2all(lam_a, v[1], rss);
        } else {
            // partitioned adjoint turn: the un-phase angles (layout 1) before any amplitude is live
            float uf_b[kRegs];
            if constexpr (KIND == FK_BTURN && PART)
                part_angles<DT>(uf_b, a, g2pi, b1, lane_lo, lane_hi, a.pos8, a.pos4, tile, t);
            ld2both(v[0], v[1]);
            if constexpr (EARLY) cz1(rc);
            double gb = 0.0;
            mix_op<HIGH, FULL, 2, 2, 3, true, FB1>(lds, v, t, a.active, c1, gb);
            acc[0] += gb;
            if constexpr (KIND == FK_BMID) {
                const uint64_t rss = opaque_u64(ss1);
                st1both(v[0], v[1], rss);
            } else {
                double gg = 0.0;
                if constexpr (!EARLY) cz1(rc);
                cz_ready(rc);
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    const double cz = reg_cost(rc, cq, r);
                    const float2 ps = v[0][r], la = v[1][r];
                    const float im = fmaf(la.x, ps.y, -la.y * ps.x);
                    gg = fma(cz - a.shift, (double)im, gg);
                    if constexpr (KIND == FK_BTURN && !PART) {
                        float c, s;
                        phase_rev(g2pi, cz, c, s);
                        rot_phase<float>(v[0][r], c, -s);
                        rot_phase<float>(v[1][r], c, -s);
                    }
                    QQ_CHUNK_FENCE(r);
                }
                acc[1] += gg;
                if constexpr (KIND == FK_BTURN && PART) apply_angles<NS, 3, true>(v, uf_b);
                if constexpr (KIND == FK_BTURN) {
                    double gb2 = 0.0;
                    mix_op<HIGH, FULL, 1, 2, 3, true, FB2>(lds, v, t, a.active, c2, gb2);
                    acc[2] += gb2;
                    const uint64_t rss = opaque_u64(ss2);
                    st2both(v[0], v[1], rss);
                }
            }
        }
    }
}

// Layer constants of one pass for parameter set x, then one uniform dispatch on
// the forms of the (up to two) mixer coefficients, so the butterfly code of each
// path has no form branch.  Tiles g, g + a.G, ... below a.tiles.
template <int KIND, bool HIGH, bool FULL, typename DT, bool PART = false, bool WIDE = false, bool CT = false,
          bool PR = true>
__device__ __forceinline__ void run_pass(const FastArgs &a, float2 *lds, double (&acc)[3], int t, int b, int g)
{
    const double *x = a.params + (size_t)b * 2 * a.p;
    MixCoef c1{}, c2{};
    double gam = 0.0;
    if constexpr (KIND == FK_FIRST) {
        gam = x[0];
        c1 = mix_coef(x[1], false, a.nact);
    } else if constexpr (KIND == FK_MID || KIND == FK_LAST) {
        c1 = mix_coef(x[2 * a.k + 1], false, a.nact);
    } else if constexpr (KIND == FK_TURN) {
        c1 = mix_coef(x[2 * a.k + 1], false, a.nact);
        gam = x[2 * (a.k + 1)];
        c2 = mix_coef(x[2 * (a.k + 1) + 1], false, a.nact);
    } else if constexpr (KIND == FK_LASTG) {
        c1 = mix_coef(x[2 * a.k + 1], false, a.nact);
        c2 = mix_coef(x[2 * a.k + 1], true, a.nact);
    } else if constexpr (KIND == FK_BMID || KIND == FK_BLAST) {
        c1 = mix_coef(x[2 * a.k + 1], true, a.nact);
    } else if constexpr (KIND == FK_BTURN) {
        c1 = mix_coef(x[2 * a.k + 1], true, a.nact);
        gam = x[2 * a.k];
        c2 = mix_coef(x[2 * (a.k - 1) + 1], true, a.nact);
    }
    const double g2pi = gam * QQ_INV_TWO_PI;
    constexpr bool TWO = KIND == FK_TURN || KIND == FK_LASTG || KIND == FK_BTURN;
    if constexpr (!FULL) {
        // general butterflies: one body serves both forms
        pass_body<KIND, HIGH, FULL, DT, PART, WIDE, false, false, CT, PR>(a, lds, acc, t, b, g, c1, c2, g2pi);
        return;
    }
    const int sel = (c1.formB ? 1 : 0) | (TWO && c2.formB ? 2 : 0);
    if (sel == 0) pass_body<KIND, HIGH, FULL, DT, PART, WIDE, false, false, CT, PR>(a, lds, acc, t, b, g, c1, c2, g2pi);
    else if (sel == 1) pass_body<KIND, HIGH, FULL, DT, PART, WIDE, true, false, CT, PR>(a, lds, acc, t, b, g, c1, c2, g2pi);
    else if constexpr (TWO) {
        if (sel == 2) pass_body<KIND, HIGH, FULL, DT, PART, WIDE, false, true, CT, PR>(a, lds, acc, t, b, g, c1, c2, g2pi);
        else pass_body<KIND, HIGH, FULL, DT, PART, WIDE, true, true, CT, PR>(a, lds, acc, t, b, g, c1, c2, g2pi);
    }
}

// Fixed-order workgroup sum of one FP64 value per thread (all threads get the result).
// s_red holds one double per wave; the caller's next use of s_red must follow a barrier.
__device__ __forceinline__ double wg_sum(double x, double *s_red, int t)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if ((t & 63) == 0) s_red[t >> 6] = x;
    __syncthreads();
    const double r = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    __syncthreads();
    return r;
}

}  // namespace passes
}  // namespace qq
