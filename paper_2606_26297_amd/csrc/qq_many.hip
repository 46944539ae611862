// qq_many.hip -- one persistent launch evaluating many problems of uneven n and p.
//
// The launch drains a queue of work items (problem, parameter set, pass, tile
// chunk).  A multi-pass problem (n > 12) runs the same complex64 pass bodies as
// the per-pass kernels, one chunk of tiles per item; its pass j + 1 may start
// on a state once every chunk of pass j on that state has completed.  A problem
// with n <= 12 is a single item: one workgroup runs the whole evaluation (all p
// layers, the energy and the adjoint sweep) on one register-resident tile.
// The complex128 launch (many128_kernel) runs the general pass bodies on
// complex128 states instead, one chunk of tiles per item for every problem
// (a problem with n <= 12 has one pass of one tile).
//
// Ordering and progress.  Tickets are handed out in increasing order from one
// atomic counter, and items are numbered so that every pass of a state comes
// after its earlier passes (the host orders them by the fraction of each
// problem's pass chain done), so every item an item waits for has a smaller
// ticket and is held by a workgroup that is already running.  Hence the queue drains with
// any number of resident workgroups.  Every wait is bounded in wall-clock time;
// a wait that runs out sets an error flag, after which every workgroup stops
// taking items and the launch ends (the host reports the error).
//
// Memory ordering.  Each XCD has its own L2, so an item is published with an
// agent-scope release (L2 write-back) before its counter increment, and a waiting
// workgroup takes an agent-scope acquire (L2 and vector-cache invalidate) once the
// counter is reached.  Both are XCD-wide cache operations, so each is issued once
// per item by thread 0, the other waves being ordered through the workgroup barrier
// after their own stores have completed.
//
// Reductions.  Each item writes its workgroup's FP64 partial sums to a slot of
// its own; the workgroup that completes the last item of a state sums the
// partials in a fixed order (slots ascending, chunks ascending), so results are
// reproducible run to run.
#include "qq_generic.h"
#include "qq_passes.h"

namespace qq {
namespace {

using namespace dev;
using namespace passes;

// ---- problems with n <= 12: the whole evaluation in one tile ----------------------------------
// The tile holds 2^(12-n) identical copies of the state (tile bits n..11 are
// spectators: the cost diagonal is read at z & (2^n - 1) and those bits are never
// mixed), so tile sums are 2^(12-n) times the state's sums.

template <int L, typename DT>
__device__ __forceinline__ double cz_tile(const DT *diag, uint32_t mask, int t, int r)
{
    return (double)diag[(uint32_t)lidx<L>(t, r) & mask];
}

// psi *= exp(-i gamma C) in layout L.
template <int L, typename DT>
__device__ __forceinline__ void single_phase(float2 (&v)[kRegs], const DT *diag, uint32_t mask, int t, double g2pi)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        float c, s;
        phase_rev(g2pi, cz_tile<L>(diag, mask, t, r), c, s);
        rot_phase<float>(v[r], c, s);
        QQ_CHUNK_FENCE(r);
    }
}

// sum |psi|^2 C; with GRAD also lambda = C psi.  The state is in layout 1 when
// L1 is set and in layout 2 otherwise (a uniform select of the register's index).
template <typename DT, bool GRAD>
__device__ __forceinline__ double single_energy(float2 (&v)[2][kRegs], const DT *diag, uint32_t mask, int t, bool L1)
{
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const uint32_t z = (uint32_t)(L1 ? lidx<1>(t, r) : lidx<2>(t, r)) & mask;
        const double cz = (double)diag[z];
        const float pz = fmaf(v[0][r].x, v[0][r].x, v[0][r].y * v[0][r].y);
        e = fma((double)pz, cz, e);
        if constexpr (GRAD) {
            const float cf = (float)cz;
            v[1][r] = make_float2(cf * v[0][r].x, cf * v[0][r].y);
        }
        QQ_CHUNK_FENCE(r);
    }
    return e;
}

// sum C Im(conj(lambda) psi) in layout L, then both states un-phased.
template <int L, typename DT>
__device__ __forceinline__ double single_ggamma(float2 (&v)[2][kRegs], const DT *diag, uint32_t mask, int t,
                                                double g2pi)
{
    double gg = 0.0;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const double cz = cz_tile<L>(diag, mask, t, r);
        const float2 ps = v[0][r], la = v[1][r];
        gg = fma(cz, (double)fmaf(la.x, ps.y, -la.y * ps.x), gg);
        float c, s;
        phase_rev(g2pi, cz, c, s);
        rot_phase<float>(v[0][r], c, -s);
        rot_phase<float>(v[1][r], c, -s);
        QQ_CHUNK_FENCE(r);
    }
    return gg;
}

// The thread index made opaque: per-register diagonal addresses and LDS slots are
// then formed where they are used rather than hoisted out of the layer loops
// (where 16 addresses per layout would stay live throughout).
__device__ __forceinline__ int fresh_index(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}

// Forward layer k of a single-tile evaluation: phase, then the mixer from layout
// L (2 for even k, 1 for odd k) to the other layout.
template <int L, typename DT>
__device__ __forceinline__ void single_layer(float2 *lds, float2 (&v)[2][kRegs], const DT *diag, uint32_t mask,
                                             int t, int active, double g2pi, const MixCoef &c)
{
    const int tk = fresh_index(t);
    single_phase<L>(v[0], diag, mask, tk, g2pi);
    double unused = 0.0;
    mix_op<false, false, L, 2, 1, false, false>(lds, v, tk, active, c, unused);
}

// Adjoint step of layer k: inverse mixer with the beta-derivative, from the layout
// the forward layer ended in (1 for even k, 2 for odd k) back to L; then the
// gamma-derivative and the un-phase in L.  The un-phase after layer 0 is not needed
// and is harmless.  Returns (d/d beta_k, d/d gamma_k) partials of this thread.
template <int L, typename DT>
__device__ __forceinline__ void single_back(float2 *lds, float2 (&v)[2][kRegs], const DT *diag, uint32_t mask, int t,
                                            int active, double g2pi, const MixCoef &c, double &gb, double &gg)
{
    const int tk = fresh_index(t);
    gb = 0.0;
    mix_op<false, false, 3 - L, 2, 3, true, false>(lds, v, tk, active, c, gb);
    gg = single_ggamma<L>(v, diag, mask, tk, g2pi);
}

// Whole evaluation of parameter set b of a problem with n <= 12.  Output o of the
// problem (0: energy, 1 + 2k: d/d gamma_k, 2 + 2k: d/d beta_k, before the final
// scaling) is written to accumulator slot o, chunk 0.  Layer k's mixer runs 2 -> 1
// for even k and 1 -> 2 for odd k; the layers are taken in pairs so that every
// layout is fixed at compile time (the mixers use general butterflies, which serve
// both coefficient forms and the partial masks of n < 12).
template <typename DT, bool GRAD>
__device__ void single_eval(const ManyInst &I, double *partial, float2 *lds, double *s_red, MixCoef *s_coef, int t,
                            int b)
{
    const DT *diag = static_cast<const DT *>(I.diag);
    const uint32_t mask = (uint32_t)I.dim_mask;
    const int n = I.n, p = I.p;
    const int active = (1 << n) - 1;
    const double *x = I.params + (size_t)b * 2 * p;
    double *out = partial + I.partial_off + b;  // slot o at out[o * B]
    const size_t ostride = (size_t)I.B;
    // mixer coefficients of every layer (forward, then inverse), one thread per layer
    if (t < p) {
        s_coef[t] = mix_coef(x[2 * t + 1], false, n);
        s_coef[QQ_MAX_P + t] = mix_coef(x[2 * t + 1], true, n);
    }
    __syncthreads();
    float2 v[2][kRegs];
#pragma unroll
    for (int r = 0; r < kRegs; ++r) v[0][r] = make_float2((float)I.amp0, 0.0f);

    int k = 0;
    for (; k + 1 < p; k += 2) {
        single_layer<2>(lds, v, diag, mask, t, active, x[2 * k] * QQ_INV_TWO_PI, s_coef[k]);
        single_layer<1>(lds, v, diag, mask, t, active, x[2 * k + 2] * QQ_INV_TWO_PI, s_coef[k + 1]);
    }
    if (k < p) single_layer<2>(lds, v, diag, mask, t, active, x[2 * k] * QQ_INV_TWO_PI, s_coef[k]);
    // after layer p - 1 the state is in layout 1 (p odd) or 2 (p even)
    const int te = fresh_index(t);
    const double e = wg_sum(single_energy<DT, GRAD>(v, diag, mask, te, (p & 1) != 0), s_red, te);
    if (te == 0) out[0] = e;
    if constexpr (GRAD) {
        auto put = [&](int kk, double gb, double gg) {
            gb = wg_sum(gb, s_red, t);
            gg = wg_sum(gg, s_red, t);
            if (t == 0) {
                out[(size_t)(2 + 2 * kk) * ostride] = gb;
                out[(size_t)(1 + 2 * kk) * ostride] = gg;
            }
        };
        k = p - 1;
        double gb, gg;
        if ((k & 1) == 0) {  // p odd: the top layer is even and goes alone
            single_back<2>(lds, v, diag, mask, t, active, x[2 * k] * QQ_INV_TWO_PI, s_coef[QQ_MAX_P + k], gb, gg);
            put(k, gb, gg);
            --k;
        }
        for (; k >= 1; k -= 2) {
            single_back<1>(lds, v, diag, mask, t, active, x[2 * k] * QQ_INV_TWO_PI, s_coef[QQ_MAX_P + k], gb, gg);
            put(k, gb, gg);
            single_back<2>(lds, v, diag, mask, t, active, x[2 * k - 2] * QQ_INV_TWO_PI, s_coef[QQ_MAX_P + k - 1], gb,
                           gg);
            put(k - 1, gb, gg);
        }
    }
}

// ---- multi-pass problems: one chunk of one pass ---------------------------------------------
template <int KIND, typename DT>
__device__ __forceinline__ void run_geom(int geom, const FastArgs &a, float2 *lds, double (&acc)[3], int t, int b,
                                         int g)
{
    if (geom == 0) {
        run_pass<KIND, false, true, DT, false, false, true, false>(a, lds, acc, t, b, g);
    } else if constexpr (KIND != FK_FIRST) {  // the persistent plans take the qubit-0..11 set first
        if (geom == 1) run_pass<KIND, true, true, DT, false, false, true, false>(a, lds, acc, t, b, g);
        else run_pass<KIND, true, false, DT, false, false, true, false>(a, lds, acc, t, b, g);
    }
}

template <typename DT>
__device__ __forceinline__ void run_chunk(const ManyInst &I, const ManyPass &P, double *partial, float2 *lds,
                                          double *s_red, int t, int b, int chunk)
{
    FastArgs a;
    a.B = I.B;
    a.G = 1;  // consecutive tiles
    a.p = I.p;
    a.k = P.k;
    const uint64_t t0 = (uint64_t)chunk * (uint64_t)I.tpc;
    a.tiles = min(I.tiles, t0 + (uint64_t)I.tpc);
    a.dim_mask = I.dim_mask;
    a.pos4 = P.pos4;
    a.pos8 = P.pos8;
    a.w1 = P.w1;
    a.w2 = P.w2;
    a.active = P.active;
    a.nact = P.nact;
    a.store_psi = P.store_psi;
    a.slot_base = 0;
    a.slot_stride = 0;
    a.amp0 = I.amp0;
    a.params = I.params;
    a.diag = I.diag;
    a.psi = static_cast<float2 *>(I.psi);
    a.lam = static_cast<float2 *>(I.lam);
    a.state_stride = I.dim_mask + 1;
    a.partial = nullptr;
    a.blocked = 0;
    a.part = nullptr;
    a.tables = nullptr;
    a.cq = I.regq + 16 * (P.kind == FK_FIRST ? P.pos8 : P.pos4);
    a.pcq = nullptr;  // the persistent launch takes no partitioned phases
    a.pcq_runs = 0;
    a.shift = I.shift;
    a.ctab = P.ctab;
    a.cthr = P.cthr;
    a.xtab = a.xthr = nullptr;  // no partitioned phases here
    a.ilv = 0;                  // separate psi and lambda arrays
    double acc[3] = {0.0, 0.0, 0.0};
    const int g = (int)t0;
    switch (P.kind) {
    case FK_FIRST: run_geom<FK_FIRST, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_MID: run_geom<FK_MID, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_TURN: run_geom<FK_TURN, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_LAST: run_geom<FK_LAST, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_LASTG: run_geom<FK_LASTG, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_BMID: run_geom<FK_BMID, DT>(P.geom, a, lds, acc, t, b, g); break;
    case FK_BTURN: run_geom<FK_BTURN, DT>(P.geom, a, lds, acc, t, b, g); break;
    default: run_geom<FK_BLAST, DT>(P.geom, a, lds, acc, t, b, g); break;
    }
    // partial sums: slot (P.slot_base + s), state b, chunk
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        if (s >= P.nslots) break;
        const double v = wg_sum(acc[s], s_red, t);
        if (t == 0) partial[I.partial_off + ((size_t)(P.slot_base + s) * I.B + b) * I.nchunks + chunk] = v;
    }
}

// Final results of state b: fixed-order sums of its partials.
__device__ void finish_state(const ManyArgs &A, const ManyInst &I, int b, int t)
{
    const int nout = A.grad ? 1 + 2 * I.p : 1;
    for (int o = t; o < nout; o += kThreads) {
        double tot = 0.0;
        for (int s = 0; s < I.nslots; ++s) {
            if ((int)A.slot_out[I.slot_off + s] != o) continue;
            const double *src = A.partial + I.partial_off + ((size_t)s * I.B + b) * I.nchunks;
            double x = 0.0;
            for (int c = 0; c < I.nchunks; ++c) x += src[c];
            tot += x;
        }
        const double v = o == 0 ? tot * I.escale + I.shift : tot * (2.0 * I.escale);
        if (I.energy_out) {
            if (o == 0) I.energy_out[b] = v;
            else I.grad_out[(size_t)b * 2 * I.p + (o - 1)] = v;
        } else {
            I.out_ws[(size_t)b * (1 + 2 * I.p) + o] = v;
        }
    }
}

// The queue of a persistent launch: take tickets until every item is taken or an error is flagged;
// wait until the item's state has completed its earlier passes, run(I, pass, b, chunk), publish
// the item, and let the workgroup that completes a state's last item finish that state.  The item
// bodies are lambdas marked always_inline: called out of line, they spill registers across the call.
template <typename Run>
__device__ __forceinline__ void drain_queue(const ManyArgs &A, uint32_t *s_msg, int t, Run run)
{
    uint32_t *head = A.ctl, *err = A.ctl + 1, *cnt = A.ctl + 2;

    for (;;) {
        if (t == 0) {
            s_msg[0] = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_msg[1] = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const uint32_t ticket = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_msg[0]);
        const uint32_t failed = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_msg[1]);
        __syncthreads();
        if (ticket >= A.total || failed) break;

        // the segment holding this ticket: the last one with first <= ticket
        int lo = 0, hi = A.nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.seg[mid].first <= ticket) lo = mid;
            else hi = mid - 1;
        }
        const ManySeg sg = A.seg[lo];
        const ManyInst &I = A.inst[sg.inst];
        const int b = (int)sg.b;
        const int chunk = (int)(ticket - sg.first);
        const uint32_t state = (uint32_t)I.state0 + sg.b;

        if (sg.pass > 0) {
            // wait until every chunk of the previous passes on this state has completed
            const uint32_t need = sg.pass * (uint32_t)I.nchunks;
            if (t == 0) {
                uint32_t ok = 1;
                const uint64_t start = wall_clock64();
                // relaxed polling (an acquire per poll would invalidate this XCD's L2 each
                // time); the acquire fence follows once the count is reached
                while (__hip_atomic_load(cnt + state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        ok = 0;
                        break;
                    }
                    if (wall_clock64() - start > A.spin_ticks) {
                        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                // acquire for the whole workgroup: the invalidate covers the CU's vector
                // cache, which the other waves share, and they load only after the barrier
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_msg[1] = ok;
            }
            __syncthreads();
            const uint32_t ok = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_msg[1]);
            __syncthreads();
            if (!ok) break;
        }

        run(I, (int)sg.pass, b, chunk);

        // publish: every wave waits for its own stores to complete (to the XCD's L2), the
        // barrier orders them before thread 0, whose agent-scope release writes the L2
        // back before the counter increment; one release per item instead of one per wave
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t == 0) {
            const uint32_t done = __hip_atomic_fetch_add(cnt + state, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
            s_msg[0] = done == (uint32_t)(I.npasses * I.nchunks) ? 1u : 0u;
        }
        __syncthreads();
        const uint32_t last = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_msg[0]);
        __syncthreads();
        if (last) finish_state(A, I, b, t);  // thread 0's acq_rel increment acquired for the CU
    }
}

template <typename DT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) many_kernel(const ManyArgs A)
{
    __shared__ float2 lds[kLdsSlots];
    __shared__ double s_red[kThreads / 64];
    __shared__ uint32_t s_msg[2];
    __shared__ MixCoef s_coef[2 * QQ_MAX_P];
    const int t = threadIdx.x;
    drain_queue(A, s_msg, t, [&](const ManyInst &I, int pass, int b, int chunk) __attribute__((always_inline)) {
        const ManyPass &P = A.pass[I.pass_off + pass];
        // The thread index, opaque per item: keeps each body's index arithmetic
        // inside its own branch instead of hoisted out of the item loop (where
        // the values of every body would stay live at once).
        int ti = t;
        asm volatile("" : "+v"(ti));
        if (P.kind == FK_SINGLE) {
            if (A.grad) single_eval<DT, true>(I, A.partial, lds, s_red, s_coef, ti, b);
            else single_eval<DT, false>(I, A.partial, lds, s_red, s_coef, ti, b);
        } else {
            run_chunk<DT>(I, P, A.partial, lds, s_red, ti, b, chunk);
        }
    });
}

// Complex128 states: the general pass body of item (problem, parameter set b, pass, chunk) over the
// chunk's consecutive tiles, its slot totals into the item's partial sums.
template <typename DT>
__global__ void __launch_bounds__(kThreads) many128_kernel(const ManyArgs A)
{
    __shared__ gen::GenShared<double> sh;
    __shared__ uint32_t s_msg[2];
    const int t = threadIdx.x;
    drain_queue(A, s_msg, t, [&](const ManyInst &I, int pass, int b, int chunk) __attribute__((always_inline)) {
        const ManyPass &P = A.pass[I.pass_off + pass];
        const PassArgs &a = A.gpass[I.pass_off + pass];
        gen::gen_setup<double>(sh, I.params + (size_t)b * 2 * I.p, I.p, t);
        double acc[kMaxLocalSlots] = {0.0, 0.0, 0.0, 0.0};
        const uint64_t t0 = (uint64_t)chunk * (uint64_t)I.tpc, t1 = min(I.tiles, t0 + (uint64_t)I.tpc);
        if (P.geom > 1) gen::gen_tiles<double, 2, DT>(a, sh, t, b, t0, t1, 1, acc);
        else gen::gen_tiles<double, 1, DT>(a, sh, t, b, t0, t1, 1, acc);
        gen::gen_slot_totals<double>(P.nslots, acc, sh, t, [&](int s, double sum) __attribute__((always_inline)) {
            A.partial[I.partial_off + ((size_t)(P.slot_base + s) * I.B + b) * I.nchunks + chunk] = sum;
        });
    });
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// As many workgroups as can be resident at once (every one of them then runs until the queue is
// drained), at most max_grid (> 0) and at most one per item.
template <typename K>
hipError_t launch_resident(K kernel, const ManyArgs &a, int max_grid, hipStream_t s, int *grid_out)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0)) != hipSuccess) return e;
    long grid = (long)std::max(1, per_cu) * std::max(1, cus);
    if (max_grid > 0) grid = std::min<long>(grid, max_grid);
    grid = std::max(1L, std::min<long>(grid, (long)a.total));
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <typename DT>
hipError_t launch_many_t(const ManyArgs &a, bool c128, int max_grid, hipStream_t s, int *grid_out)
{
    return c128 ? launch_resident(many128_kernel<DT>, a, max_grid, s, grid_out)
                : launch_resident(many_kernel<DT>, a, max_grid, s, grid_out);
}

}  // namespace

hipError_t launch_many(const ManyArgs &a, bool c128, int diag_type, int max_grid, hipStream_t s, int *grid_out)
{
    switch (diag_type) {
    case DIAG_F64: return launch_many_t<double>(a, c128, max_grid, s, grid_out);
    case DIAG_I32: return launch_many_t<int32_t>(a, c128, max_grid, s, grid_out);
    default: return launch_many_t<int16_t>(a, c128, max_grid, s, grid_out);
    }
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace qq
