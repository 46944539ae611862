// qq_generic.h -- the general pass body: one pass's list of operations (mixer on any subset of the
// tile bits, phase, energy, adjoint seed, gamma-derivative with un-phase) applied to tiles of one
// state in complex64 or complex128, shared by the per-pass kernel and the persistent launch.
//
// The operations follow the QAOA state eq. (11): cost unitary eq. (10), mixer eq. (12)-(13); the
// energy is eq. (15) and the adjoint sweep gives the gradient of eq. (17).
#pragma once

#include <type_traits>

#include "qq_device.h"

namespace qq {
namespace gen {

using namespace dev;

// Workgroup scratch of the general pass bodies: the LDS transpose buffer (FP32 pairs or FP64
// words), the layer constants of the workgroup's parameter set and the slot reductions.
template <typename R>
struct GenShared {
    typename std::conditional<sizeof(R) == 4, float2, double>::type lds[kLdsSlots];
    R cb[QQ_MAX_P], sb[QQ_MAX_P];  // cos, sin of beta_k
    double gam[QQ_MAX_P];          // gamma_k
    double red[kThreads / 64][kMaxLocalSlots];
    double imm[kMaxImmSlots];  // slots reduced tile by tile (single-pass plans)
    double wsum[kThreads / 64];
};

// Layer constants of the parameter set x (2p values, gamma_k and beta_k interleaved) and cleared
// immediate slots; ends with a barrier.  The caller orders any earlier use of sh before it.
template <typename R>
__device__ __forceinline__ void gen_setup(GenShared<R> &sh, const double *x, int p, int t)
{
    for (int k = t; k < kMaxImmSlots; k += kThreads) sh.imm[k] = 0.0;
    if (t < p) {
        double sb, cb;
        sincos(x[2 * t + 1], &sb, &cb);
        sh.cb[t] = (R)cb;
        sh.sb[t] = (R)sb;
        sh.gam[t] = x[2 * t];
    }
    __syncthreads();
}

// Tiles t_begin, t_begin + t_step, ... below t_end of state b: pass a's operations; FP64 partial
// sums of slots below kMaxLocalSlots accumulate in acc (per thread), higher slots in sh.imm.
template <typename R, int NS, typename DT>
__device__ __forceinline__ void gen_tiles(const PassArgs &a, GenShared<R> &sh, int t, int b, uint64_t t_begin,
                                          uint64_t t_end, uint64_t t_step, double (&acc)[kMaxLocalSlots])
{
    using C2 = typename Cx<R>::T;
    using W = typename std::conditional<sizeof(R) == 4, float2, double>::type;

    const uint64_t off2 = (uint64_t)(t & 15) | ((uint64_t)(t >> 4) << a.pos4);
    const uint64_t st2 = 1ull << a.pos8;
    const uint64_t off1 = (uint64_t)(t & 15) | ((uint64_t)(t >> 4) << a.pos8);
    const uint64_t st1 = 1ull << a.pos4;

    C2 *psi = static_cast<C2 *>(a.psi) + (size_t)b * a.state_stride;
    C2 *lam = NS > 1 ? static_cast<C2 *>(a.lam) + (size_t)b * a.state_stride : nullptr;

    C2 v[NS][kRegs];

    for (uint64_t tile = t_begin; tile < t_end; tile += t_step) {
        uint64_t base;
        if (a.high) base = tile_base(tile, a.pos4, a.pos8, a.w1, a.w2);
        else base = tile << kTileBits;

        int live = 0;
        if (a.flags & PF_INIT) {
#pragma unroll
            for (int r = 0; r < kRegs; ++r) v[0][r] = mk<C2, R>((R)a.amp0, (R)0);
            live |= 1;
        }
        if (a.flags & PF_LOAD_PSI) {
#pragma unroll
            for (int r = 0; r < kRegs; ++r) v[0][r] = psi[base + off2 + r * st2];
            live |= 1;
        }
        if constexpr (NS > 1) {
            if (a.flags & PF_LOAD_LAM) {
#pragma unroll
                for (int r = 0; r < kRegs; ++r) v[1][r] = lam[base + off2 + r * st2];
                live |= 2;
            }
        }
        int cur = 2;

        auto to_layout = [&](int to) {
            if (to == cur) return;
            if (live & 1) transpose1<W>(sh.lds, v[0], t, cur, to);
            if constexpr (NS > 1)
                if (live & 2) transpose1<W>(sh.lds, v[1], t, cur, to);
            cur = to;
        };
        auto coalesced = [&]() {
            if (cur == 0) to_layout(1);
        };
        // Slots 0..3 accumulate in registers across tiles; higher slots (only in
        // single-pass plans) are reduced over the workgroup at once into LDS.
        auto accumulate = [&](int slot, double val) {
            if (slot < kMaxLocalSlots) {
                add_slot(acc, slot, val);
                return;
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) val += __shfl_xor(val, d, 64);
            if ((t & 63) == 0) sh.wsum[t >> 6] = val;
            __syncthreads();
            if (t == 0) sh.imm[slot] += (sh.wsum[0] + sh.wsum[1]) + (sh.wsum[2] + sh.wsum[3]);
            __syncthreads();
        };

        for (int o = 0; o < a.nops; ++o) {
            const Op op = a.ops[o];
            if (op.kind == OP_MIX) {
                const R cb = sh.cb[op.layer];
                const R sb = (op.flags & OPF_INVERSE) ? -sh.sb[op.layer] : sh.sb[op.layer];
                int seq[3], ns = 0;
                const int need = (((op.active & 0x00f) != 0) << 0) | (((op.active & 0x0f0) != 0) << 1) |
                                 (((op.active & 0xf00) != 0) << 2);
                if (need & (1 << cur)) seq[ns++] = cur;
                if ((need & 1) && cur != 0) seq[ns++] = 0;
                if ((need & 2) && cur != 1) seq[ns++] = 1;
                if ((need & 4) && cur != 2) seq[ns++] = 2;
                for (int k = 0; k < ns; ++k) {
                    const int gi = seq[k];
                    to_layout(gi);
                    const int m = (op.active >> (4 * gi)) & 15;
                    double gacc = 0.0;
#define QQ_BIT(K)                                                                   \
    if (m & (1 << K)) {                                                             \
        if constexpr (NS > 1)                                                       \
            if (op.slot != kNoSlot) gacc += xexp_bit<K>(v[0], v[1]);                      \
        if (op.states & 1) rx_bit<K>(v[0], cb, sb);                                 \
        if constexpr (NS > 1)                                                       \
            if (op.states & 2) rx_bit<K>(v[1], cb, sb);                             \
    }
                    QQ_BIT(0)
                    QQ_BIT(1)
                    QQ_BIT(2)
                    QQ_BIT(3)
#undef QQ_BIT
                    if (op.slot != kNoSlot) accumulate(op.slot, gacc);
                }
            } else {
                coalesced();
                const uint64_t off = cur == 2 ? off2 : off1;
                const uint64_t st = cur == 2 ? st2 : st1;
                const double gam = sh.gam[op.layer];
                double tacc = 0.0;
                if (op.kind == OP_PHASE) {
                    const bool inv = op.flags & OPF_INVERSE;
#pragma unroll
                    for (int r = 0; r < kRegs; ++r) {
                        const uint64_t gi = (base + off + r * st) & a.dim_mask;
                        if (op.flags & OPF_PARTITIONED) {
                            for (int m = 0; m < a.part->nparts + 1; ++m) {
                                double cm;
                                if (m < a.part->nparts)
                                    cm = ldc<DT>(a.part_tables, a.part->table_off[m] +
                                                                    compress_bits(gi, a.part->vars[m], a.part->nvars[m]));
                                else cm = ldc<DT>(a.cross_diag, gi);
                                R c, s;
                                phase_cs(gam * cm, c, s);
                                if (inv) s = -s;
                                if (op.states & 1) rot_phase<R>(v[0][r], c, s);
                                if constexpr (NS > 1)
                                    if (op.states & 2) rot_phase<R>(v[1][r], c, s);
                            }
                        } else {
                            R c, s;
                            phase_cs(gam * ldc<DT>(a.diag, gi), c, s);
                            if (inv) s = -s;
                            if (op.states & 1) rot_phase<R>(v[0][r], c, s);
                            if constexpr (NS > 1)
                                if (op.states & 2) rot_phase<R>(v[1][r], c, s);
                        }
                    }
                } else if (op.kind == OP_ENERGY || op.kind == OP_ENERGY_LAMBDA) {
#pragma unroll
                    for (int r = 0; r < kRegs; ++r) {
                        const uint64_t gi = (base + off + r * st) & a.dim_mask;
                        const double cz = ldc<DT>(a.diag, gi);
                        const double re = (double)v[0][r].x, im = (double)v[0][r].y;
                        tacc = fma(fma(re, re, im * im), cz, tacc);
                        if constexpr (NS > 1)
                            if (op.kind == OP_ENERGY_LAMBDA) v[1][r] = mk<C2, R>((R)(cz * re), (R)(cz * im));
                    }
                    if (op.kind == OP_ENERGY_LAMBDA) live |= 2;
                } else if (op.kind == OP_GGAMMA) {
                    if constexpr (NS > 1) {
                        const bool unph = op.flags & OPF_UNPHASE;
#pragma unroll
                        for (int r = 0; r < kRegs; ++r) {
                            const uint64_t gi = (base + off + r * st) & a.dim_mask;
                            const double cz = ldc<DT>(a.diag, gi);
                            const C2 ps = v[0][r], la = v[1][r];
                            const double im = fma((double)la.x, (double)ps.y, -(double)la.y * (double)ps.x);
                            tacc = fma(cz, im, tacc);
                            if (unph) {
                                if (op.flags & OPF_PARTITIONED) {
                                    for (int m = 0; m < a.part->nparts + 1; ++m) {
                                        double cm;
                                        if (m < a.part->nparts)
                                            cm = ldc<DT>(a.part_tables,
                                                         a.part->table_off[m] +
                                                             compress_bits(gi, a.part->vars[m], a.part->nvars[m]));
                                        else cm = ldc<DT>(a.cross_diag, gi);
                                        R c, s;
                                        phase_cs(gam * cm, c, s);
                                        rot_phase<R>(v[0][r], c, -s);
                                        rot_phase<R>(v[1][r], c, -s);
                                    }
                                } else {
                                    R c, s;
                                    phase_cs(gam * cz, c, s);
                                    rot_phase<R>(v[0][r], c, -s);
                                    rot_phase<R>(v[1][r], c, -s);
                                }
                            }
                        }
                    }
                }
                if (op.slot != kNoSlot) accumulate(op.slot, tacc);
            }
        }

        if (a.flags & (PF_STORE_PSI | PF_STORE_LAM)) {
            coalesced();
            const uint64_t off = cur == 2 ? off2 : off1;
            const uint64_t st = cur == 2 ? st2 : st1;
#pragma unroll
            for (int r = 0; r < kRegs; ++r) {
                const uint64_t gi = base + off + r * st;
                if (gi & ~a.dim_mask) continue;  // replicated copies of a state smaller than a tile
                if (a.flags & PF_STORE_PSI) psi[gi] = v[0][r];
                if constexpr (NS > 1)
                    if (a.flags & PF_STORE_LAM) lam[gi] = v[1][r];
            }
        }
    }

}

// Workgroup totals of a pass's slots: write(s, total) for every slot s < nslots (thread s, then
// s + kThreads, ...), each total a fixed-order sum.
template <typename R, typename F>
__device__ __forceinline__ void gen_slot_totals(int nslots, const double (&acc)[kMaxLocalSlots], GenShared<R> &sh,
                                                int t, F write)
{
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int s = 0; s < kMaxLocalSlots; ++s) {
        if (s >= nslots) break;
        double x = acc[s];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
        if (lane == 0) sh.red[wave][s] = x;
    }
    __syncthreads();
    for (int s = t; s < nslots; s += kThreads) {
        const double sum =
            s < kMaxLocalSlots ? ((sh.red[0][s] + sh.red[1][s]) + (sh.red[2][s] + sh.red[3][s])) : sh.imm[s];
        write(s, sum);
    }
}

}  // namespace gen
}  // namespace qq
