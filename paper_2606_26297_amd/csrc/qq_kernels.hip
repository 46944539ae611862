// qq_kernels.hip -- gfx950 kernels of the exact QAOA-for-QUBO statevector engine.
//
// The method (cost unitary eq. (10), mixer eq. (12)-(13), state eq. (11),
// objective eq. (15)/(17)) is executed as a sequence of "passes".  A pass
// streams every amplitude of the state(s) once through registers in tiles of
// 2^12 amplitudes and applies, in registers, a short program of operations:
//   MIX      RX(+-2 beta_k) on a subset of the tile's qubits (butterflies on
//            register-resident bits; LDS transposes rotate which 4 tile bits
//            are register bits),
//   PHASE    multiplication by exp(-+ i gamma_k C(z)) (FP64 argument, FP64
//            reduction modulo 2 pi, then the rotation in the state precision),
//   ENERGY   FP64 accumulation of |psi|^2 C,
//   ENERGY_LAMBDA / GGAMMA   the seeds and gamma-derivatives of the adjoint sweep.
// The beta-derivative sum_q Im<lambda|X_q|psi> is accumulated inside the
// MIX butterflies of the backward sweep.  All accumulations are FP64 and are
// reduced in a fixed order (no floating-point atomics), so results are
// bit-reproducible.
#include <type_traits>

#include "qq_device.h"
#include "qq_generic.h"

namespace qq {
namespace {

using namespace dev;

template <typename R, int NS, typename DT>
__global__ void __launch_bounds__(kThreads) pass_kernel(const PassArgs a)
{
    __shared__ gen::GenShared<R> sh;
    const int t = threadIdx.x;
    int b, g;
    block_coords(a.B, a.G, b, g);
    gen::gen_setup<R>(sh, a.params + (size_t)b * 2 * a.p, a.p, t);
    double acc[kMaxLocalSlots] = {0.0, 0.0, 0.0, 0.0};
    gen::gen_tiles<R, NS, DT>(a, sh, t, b, (uint64_t)g, a.tiles, (uint64_t)a.G, acc);
    // fixed-order workgroup reduction of the FP64 accumulators
    gen::gen_slot_totals<R>(a.nslots, acc, sh, t, [&](int s, double sum) __attribute__((always_inline)) {
        a.partial[(size_t)(a.slot_base + s) * a.slot_stride + (size_t)b * a.G + g] = sum;
    });
}

// out[b][o] = scale_o * sum over the slots mapped to o of sum_g partial[slot][b][g].
__global__ void __launch_bounds__(256) finalize_kernel(const FinalizeArgs a)
{
    const int nout = 1 + 2 * a.p;
    const int b = blockIdx.x / nout;
    const int o = blockIdx.x % nout;
    const int t = threadIdx.x;
    __shared__ double red[256];
    double total = 0.0;
    for (int s = 0; s < a.nslots; ++s) {
        if (a.slot_out[s] != o) continue;
        const double *src = a.partial + (size_t)s * a.B * a.G + (size_t)b * a.G;
        double x = 0.0;
        for (int gg = t; gg < a.G; gg += 256) x += src[gg];
        red[t] = x;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        total += red[0];
        __syncthreads();
    }
    if (t == 0) a.out[(size_t)b * nout + o] = o == 0 ? total * a.escale + a.shift : total * (2.0 * a.escale);
}

// ---- cost diagonal (eq. (6)) ---------------------------------------------------------------
// Four basis indices per thread.  Real problems: FP64 sum in the canonical order (c0, then l_i for
// ascending i, then b_ij row-major) over the set bits of z; integer problems: exact int32 sum of the
// same terms.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};

template <bool INT, typename DT>
__global__ void __launch_bounds__(256) cost_diag_kernel(int n, uint64_t dim, const double *ell, const int32_t *ell_i,
                                                         int npairs, const int32_t *pij, const double *pb,
                                                         const int32_t *pbi, double c0, int32_t c0_i, DT *out)
{
    // A wave takes 256 consecutive indices z = zb + 4 l + u (lane l, u = 0..3): bits 0..7 vary inside the
    // wave, bits 8 and up are those of zb, the same for the whole wave.  A coupling row i >= 8 whose
    // bit is clear in zb is skipped by the whole wave; a term whose other bits are all >= 8 adds its
    // coefficient or the neutral element chosen once for the wave (-0.0 in FP64: x + (-0.0) == x for
    // every x, so an absent term leaves the sum's bits unchanged); a term with bits below 8 is added
    // where the index's bits are set.  The coefficients are wave-uniform (scalar cache).  Each index
    // adds its present terms in the canonical order, so the FP64 entries equal the one-index sums bit
    // for bit.  The pairs are in row-major order with i < j (the canonical form's order).
    using Acc = typename std::conditional<INT, int32_t, double>::type;
    constexpr int kLow = 8;
    const Acc neutral = INT ? (Acc)0 : (Acc)-0.0;
    // first pair of every row (s_rows[n] = npairs), from the row-major pair list
    __shared__ int s_rows[QQ_MAX_N + 1];
    if ((int)threadIdx.x <= n) s_rows[threadIdx.x] = npairs;
    __syncthreads();
    for (int k = threadIdx.x; k < npairs; k += blockDim.x) {
        const int r = pij[2 * k];
        if (k == 0 || pij[2 * k - 2] != r) s_rows[r] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int r = n - 1; r >= 0; --r) s_rows[r] = min(s_rows[r], s_rows[r + 1]);
    __syncthreads();
    // lane r holds the first pair of row r; read with readlane (no memory latency in the row loop)
    const int vrows = s_rows[min((int)(threadIdx.x & 63), n)];

    const uint32_t lo = 4u * (uint32_t)(threadIdx.x & 63);
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t w = uni64((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); (w << kLow) < dim;
         w += nw) {
        const uint64_t zb = w << kLow;
        Acc acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = INT ? (Acc)c0_i : (Acc)c0;
        for (int i = 0; i < n; ++i) {
            const int iu = __builtin_amdgcn_readfirstlane(i);
            const Acc l = INT ? (Acc)ell_i[iu] : (Acc)ell[iu];
            if (iu < kLow) {
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = (((lo + u) >> iu) & 1u) ? acc[u] + l : acc[u];
            } else {
                const Acc lu = ((zb >> iu) & 1ull) ? l : neutral;
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] += lu;
            }
        }
        for (int r = 0; r < n; ++r) {
            const int ru = __builtin_amdgcn_readfirstlane(r);
            if (ru >= kLow && !((zb >> ru) & 1ull)) continue;  // the row is absent for the whole wave
            const int k0 = __builtin_amdgcn_readlane(vrows, ru);
            const int k1 = __builtin_amdgcn_readlane(vrows, ru + 1);
            if (ru >= kLow) {
                // both bits are wave-uniform: the coefficient or the neutral element, added everywhere

                for (int k = k0; k < k1; ++k) {
                    const int ku = __builtin_amdgcn_readfirstlane(k);
                    const int j = pij[2 * ku + 1];
                    const Acc wv = INT ? (Acc)pbi[ku] : (Acc)pb[ku];
                    const Acc wu = ((zb >> j) & 1ull) ? wv : neutral;
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] += wu;
                }
            } else {
                // bit r varies inside the wave; bit j does below 8, is wave-uniform from 8 on

                for (int k = k0; k < k1; ++k) {
                    const int ku = __builtin_amdgcn_readfirstlane(k);
                    const int j = pij[2 * ku + 1];
                    const Acc wv = INT ? (Acc)pbi[ku] : (Acc)pb[ku];
                    const uint32_t hj = (uint32_t)((zb >> j) & 1ull);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t bj = j < kLow ? ((lo + u) >> j) & 1u : hj;
                        acc[u] = (((lo + u) >> ru) & bj & 1u) ? acc[u] + wv : acc[u];
                    }
                }
            }
        }
        const uint64_t z = zb + lo;
        if (z + 4 <= dim) {
            Quad<DT> q;
#pragma unroll
            for (int u = 0; u < 4; ++u) q.v[u] = (DT)acc[u];
            *reinterpret_cast<Quad<DT> *>(out + z) = q;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (z + u < dim) out[z + u] = (DT)acc[u];
        }
    }
}

// Per-block (min, argmin, max) of the diagonal; ties of the minimum go to the lowest index.
template <typename DT>
__global__ void __launch_bounds__(256) minmax_kernel(const DT *d, uint64_t dim, double *part, uint64_t *pidx)
{
    __shared__ double smin[256], smax[256];
    __shared__ uint64_t sidx[256];
    double mn = INFINITY, mx = -INFINITY;
    uint64_t mi = ~0ull;
    // kUnroll coalesced loads in flight per thread, then the comparisons in increasing z (so the
    // first index of a tie within the thread is kept)
    constexpr int kUnroll = 8;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z0 < dim; z0 += stride * kUnroll) {
        double c[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t z = z0 + u * stride;
            c[u] = z < dim ? (double)d[z] : INFINITY;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t z = z0 + u * stride;
            if (z < dim) {
                if (c[u] < mn) {
                    mn = c[u];
                    mi = z;
                }
                mx = fmax(mx, c[u]);
            }
        }
    }
    const int t = threadIdx.x;
    smin[t] = mn;
    smax[t] = mx;
    sidx[t] = mi;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) {
            const double m2 = smin[t + w];
            const uint64_t i2 = sidx[t + w];
            if (m2 < smin[t] || (m2 == smin[t] && i2 < sidx[t])) {
                smin[t] = m2;
                sidx[t] = i2;
            }
            smax[t] = fmax(smax[t], smax[t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        part[2 * blockIdx.x] = smin[0];
        part[2 * blockIdx.x + 1] = smax[0];
        pidx[blockIdx.x] = sidx[0];
    }
}

template <typename DT, typename OT>
__global__ void widen_kernel(const DT *d, uint64_t dim, OT *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) out[z] = (OT)d[z];
}

// Per-QPU local cost tables: entry u of table m is the cost of the QPU's own
// terms with its variables set from the bits of u (ascending variable order);
// c0 belongs to QPU 0.  Same canonical term order as the full diagonal.
template <bool INT, typename DT>
__global__ void __launch_bounds__(256) local_tables_kernel(int n, const PartDesc *pd, const double *ell,
                                                            const int32_t *ell_i, int npairs, const int32_t *pij,
                                                            const double *pb, const int32_t *pbi, const int32_t *qpu,
                                                            double c0, int32_t c0_i, DT *out, uint64_t total)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        int m = 0;
        while (m + 1 < pd->nparts && e >= pd->table_off[m + 1]) ++m;
        const uint64_t u = e - pd->table_off[m];
        uint64_t z = 0;
        for (int j = 0; j < pd->nvars[m]; ++j) z |= ((u >> j) & 1ull) << pd->vars[m][j];
        if constexpr (INT) {
            int32_t acc = m == 0 ? c0_i : 0;
            for (int i = 0; i < n; ++i)
                if (qpu[i] == m && ((z >> i) & 1)) acc += ell_i[i];
            for (int k = 0; k < npairs; ++k) {
                const int i = pij[2 * k], j = pij[2 * k + 1];
                if (qpu[i] == m && qpu[j] == m && ((z >> i) & (z >> j) & 1)) acc += pbi[k];
            }
            out[e] = (DT)acc;
        } else {
            double acc = m == 0 ? c0 : 0.0;
            for (int i = 0; i < n; ++i)
                if (qpu[i] == m && ((z >> i) & 1)) acc += ell[i];
            for (int k = 0; k < npairs; ++k) {
                const int i = pij[2 * k], j = pij[2 * k + 1];
                if (qpu[i] == m && qpu[j] == m && ((z >> i) & (z >> j) & 1)) acc += pb[k];
            }
            out[e] = (DT)acc;
        }
    }
}

template <typename C2>
__global__ void prob_kernel(const C2 *psi, uint64_t dim, double *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const double re = (double)psi[z].x, im = (double)psi[z].y;
        out[z] = fma(re, re, im * im);
    }
}

// ---- top-k of |psi|^2 ------------------------------------------------------------------------
// Order: larger probability first, equal probabilities by lower index.
constexpr int kTopK = QQ_MAX_TOPK;

__device__ __forceinline__ bool better(double p1, uint64_t i1, double p2, uint64_t i2)
{
    return p1 > p2 || (p1 == p2 && i1 < i2);
}

struct TopList {
    double p[kTopK];
    uint64_t i[kTopK];
    __device__ void init()
    {
#pragma unroll
        for (int k = 0; k < kTopK; ++k) {
            p[k] = -1.0;
            i[k] = ~0ull;
        }
    }
    __device__ void insert(double pp, uint64_t ii)
    {
        if (!better(pp, ii, p[kTopK - 1], i[kTopK - 1])) return;
        p[kTopK - 1] = pp;
        i[kTopK - 1] = ii;
#pragma unroll
        for (int k = kTopK - 1; k > 0; --k) {
            if (better(p[k], i[k], p[k - 1], i[k - 1])) {
                const double tp = p[k];
                p[k] = p[k - 1];
                p[k - 1] = tp;
                const uint64_t ti = i[k];
                i[k] = i[k - 1];
                i[k - 1] = ti;
            }
        }
    }
};

// k rounds of a workgroup tournament over the per-thread sorted lists.
__device__ void tournament(TopList &L, int k, double *outp, uint64_t *outi)
{
    __shared__ double sp[256];
    __shared__ uint64_t si[256];
    __shared__ int sw[256];
    const int t = threadIdx.x;
    int head = 0;
    for (int round = 0; round < k; ++round) {
        double hp = -1.0;
        uint64_t hi = ~0ull;
#pragma unroll
        for (int q = 0; q < kTopK; ++q)
            if (q == head) {
                hp = L.p[q];
                hi = L.i[q];
            }
        sp[t] = hp;
        si[t] = hi;
        sw[t] = t;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w && better(sp[t + w], si[t + w], sp[t], si[t])) {
                sp[t] = sp[t + w];
                si[t] = si[t + w];
                sw[t] = sw[t + w];
            }
            __syncthreads();
        }
        if (t == 0) {
            outp[round] = sp[0];
            outi[round] = si[0];
        }
        if (sw[0] == t) ++head;
        __syncthreads();
    }
}

// Stage 1 of the top-k: the best k (probability, index) pairs of each workgroup's amplitudes.  Each
// wave keeps its own best k in registers spread over its lanes (lane j holds the j-th best, in the
// order of `better`), and an amplitude is a candidate only if it beats the wave's current k-th best.
// A wave sees its amplitudes in an order unrelated to their probabilities, so after the first few
// chunks candidates are rare: most of the sweep is a load, |psi|^2 and one comparison per amplitude,
// and the insertions (a wave-uniform loop over the ballot of candidates) are taken one at a time.
template <typename C2>
__global__ void __launch_bounds__(256) topk_stage1(const C2 *psi, uint64_t dim, int k, double *cp, uint64_t *ci)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double lp = -1.0;      // this lane's entry of the wave's list (j-th best for lane j < k)
    uint64_t li = ~0ull;
    double tp = -1.0;      // the wave's current k-th best (wave-uniform)
    uint64_t ti = ~0ull;
    constexpr int kUnroll = 8;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the loop runs over wave-uniform bases so that every lane takes part in the ballots and shuffles
    for (uint64_t zb = (uint64_t)blockIdx.x * blockDim.x + (uint64_t)wave * 64; zb < dim; zb += stride * kUnroll) {
        C2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t z = zb + lane + u * stride;
            if (z < dim) v[u] = psi[z];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t z = zb + lane + u * stride;
            const bool valid = z < dim;
            const double re = valid ? (double)v[u].x : 0.0, im = valid ? (double)v[u].y : 0.0;
            const double pz = valid ? fma(re, re, im * im) : -1.0;
            uint64_t m = __ballot(valid && better(pz, z, tp, ti));
            while (m) {
                const int src = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const double xp = __shfl(pz, src);
                const uint64_t xi = __shfl(z, src);
                if (!better(xp, xi, tp, ti)) continue;  // overtaken by an insertion of this chunk
                const int pos = __popcll(__ballot(lane < k && better(lp, li, xp, xi)));
                const double up = __shfl_up(lp, 1);
                const uint64_t ui = __shfl_up(li, 1);
                if (lane == pos) {
                    lp = xp;
                    li = xi;
                } else if (lane > pos) {
                    lp = up;
                    li = ui;
                }
                tp = __shfl(lp, k - 1);
                ti = __shfl(li, k - 1);
            }
        }
    }
    // the workgroup's best k from the four wave lists: each candidate's rank is the number of
    // candidates better than it (ties between empty entries broken by position, so ranks are distinct)
    __shared__ double sp[4 * kTopK];
    __shared__ uint64_t si[4 * kTopK];
    if (lane < k) {
        sp[wave * k + lane] = lp;
        si[wave * k + lane] = li;
    }
    __syncthreads();
    if (wave == 0 && lane < 4 * k) {
        const double mp = sp[lane];
        const uint64_t mi = si[lane];
        int rank = 0;
        for (int j = 0; j < 4 * k; ++j)
            rank += (better(sp[j], si[j], mp, mi) || (j < lane && sp[j] == mp && si[j] == mi)) ? 1 : 0;
        if (rank < k) {
            cp[(size_t)blockIdx.x * k + rank] = mp;
            ci[(size_t)blockIdx.x * k + rank] = mi;
        }
    }
}

template <typename DT>
__global__ void __launch_bounds__(256) topk_stage2(const double *cp, const uint64_t *ci, int ncand, int k,
                                                    const DT *diag, uint64_t *oi, double *op, double *oc)
{
    __shared__ double fp[kTopK];
    __shared__ uint64_t fi[kTopK];
    TopList L;
    L.init();
    for (int e = threadIdx.x; e < ncand; e += blockDim.x) L.insert(cp[e], ci[e]);
    tournament(L, k, fp, fi);
    __syncthreads();
    if (threadIdx.x < k) {
        oi[threadIdx.x] = fi[threadIdx.x];
        op[threadIdx.x] = fp[threadIdx.x];
        oc[threadIdx.x] = (double)diag[fi[threadIdx.x]];
    }
}

template <typename R, int NS>
hipError_t launch_pass_t(const PassArgs &a, int diag_type, hipStream_t s)
{
    const dim3 grid((unsigned)(a.B * a.G)), block(kThreads);
    switch (diag_type) {
    case DIAG_F64: hipLaunchKernelGGL((pass_kernel<R, NS, double>), grid, block, 0, s, a); break;
    case DIAG_I32: hipLaunchKernelGGL((pass_kernel<R, NS, int32_t>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((pass_kernel<R, NS, int16_t>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

unsigned grid_for(uint64_t work, unsigned cap = 8192)
{
    uint64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_pass(const PassArgs &a, bool c128, int nstates, int diag_type, hipStream_t s)
{
    if (c128) return nstates > 1 ? launch_pass_t<double, 2>(a, diag_type, s) : launch_pass_t<double, 1>(a, diag_type, s);
    return nstates > 1 ? launch_pass_t<float, 2>(a, diag_type, s) : launch_pass_t<float, 1>(a, diag_type, s);
}

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)(a.B * (1 + 2 * a.p))), dim3(256), 0, s, a);
    return hipGetLastError();
}

namespace {

// One row per tile (layout with launch_cost_table's declaration): C(T) of the tile's base bits T
// (c0, the l_i over T and the couplings inside T) and G_q(T) = sum_{i in T} b_iq for the tile's 12
// qubits, combined into the per-lane, per-wave and per-register entries.  One wave per tile: lane k
// takes the linear terms and couplings k, k + 64, ..., the wave sums them with butterflies, then
// lane l writes entry l and lanes 0..7 the wave and register entries.
__global__ void __launch_bounds__(256) cost_table_kernel(int n, int high, int pos4, int pos8, int lane_q, int reg_q,
                                                          uint64_t tiles, const double *ell, int npairs,
                                                          const int32_t *pij, const double *pb, double c0,
                                                          double *out)
{
    const int lane = threadIdx.x & 63;
    const uint64_t tile = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles) return;  // whole waves
    const uint64_t T = high ? tile_base(tile, pos4, pos8, pos4 - 4, pos8 - pos4 - 4) : (tile << kTileBits);
    // slots 0..3: qubits 0..3, 4..7: lane_q .. lane_q + 3, 8..11: reg_q .. reg_q + 3
    auto slot = [&](int q) {
        if (q < 4) return q;
        if (q >= lane_q && q < lane_q + 4) return 4 + (q - lane_q);
        if (q >= reg_q && q < reg_q + 4) return 8 + (q - reg_q);
        return -1;
    };
    double C = 0.0;
    for (int i = lane; i < n; i += 64)
        if ((T >> i) & 1ull) C += ell[i];
    double G[12];
#pragma unroll
    for (int s = 0; s < 12; ++s) G[s] = 0.0;
    for (int k = lane; k < npairs; k += 64) {
        const int i = pij[2 * k], j = pij[2 * k + 1];
        const double w = pb[k];
        const int si = slot(i), sj = slot(j);
        const bool bi = (T >> i) & 1ull, bj = (T >> j) & 1ull;
        if (si < 0 && sj < 0) {
            if (bi && bj) C += w;
        } else if (si < 0 || sj < 0) {
            // one end on the tile, the other in the base bits
            const int s = si < 0 ? sj : si;
            const bool on = si < 0 ? bi : bj;
#pragma unroll
            for (int u = 0; u < 12; ++u)
                if (u == s && on) G[u] += w;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        C += __shfl_xor(C, off);
#pragma unroll
        for (int s = 0; s < 12; ++s) G[s] += __shfl_xor(G[s], off);
    }
    C += c0;
    double *row = out + tile * kCostRow;
    double z = C;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if ((lane >> q) & 1) z += G[q];
    row[lane] = z;
    if (lane < 4) row[64 + lane] = ((lane & 1) ? G[6] : 0.0) + ((lane & 2) ? G[7] : 0.0);
    else if (lane < 8) row[64 + lane] = lane == 4 ? G[8] : lane == 5 ? G[9] : lane == 6 ? G[10] : G[11];
}

}  // namespace

hipError_t launch_cost_table(int n, int high, int pos4, int pos8, int lane_q, int reg_q, uint64_t tiles,
                             const double *d_ell, int npairs, const int32_t *d_pair_ij, const double *d_pair_b,
                             double c0, double *out, hipStream_t s)
{
    const unsigned grid = (unsigned)((tiles + 3) / 4);
    hipLaunchKernelGGL(cost_table_kernel, dim3(grid), dim3(256), 0, s, n, high, pos4, pos8, lane_q, reg_q, tiles,
                       d_ell, npairs, d_pair_ij, d_pair_b, c0, out);
    return hipGetLastError();
}

hipError_t launch_cost_diag(int n, int diag_type, const double *d_ell, const int32_t *d_ell_i, int npairs,
                            const int32_t *d_pair_ij, const double *d_pair_b, const int32_t *d_pair_bi, double c0,
                            int32_t c0_i, void *d_out, uint64_t dim, hipStream_t s)
{
    // 256 indices per wave, 1024 per workgroup of four waves
    const dim3 grid(grid_for((dim + 3) / 4, 65536)), block(256);
#define QQ_COST_DIAG(INT, DT)                                                                                     \
    hipLaunchKernelGGL((cost_diag_kernel<INT, DT>), grid, block, 0, s, n, dim, d_ell, d_ell_i, npairs, d_pair_ij,   \
                       d_pair_b, d_pair_bi, c0, c0_i, static_cast<DT *>(d_out))
    switch (diag_type) {
    case DIAG_F64: QQ_COST_DIAG(false, double); break;
    case DIAG_I32: QQ_COST_DIAG(true, int32_t); break;
    default: QQ_COST_DIAG(true, int16_t); break;
    }
#undef QQ_COST_DIAG
    return hipGetLastError();
}

hipError_t launch_minmax(const void *d_diag, int diag_type, uint64_t dim, double *d_part, uint64_t *d_idx,
                         int nblocks, hipStream_t s)
{
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL(minmax_kernel<double>, dim3(nblocks), dim3(256), 0, s,
                           static_cast<const double *>(d_diag), dim, d_part, d_idx);
        break;
    case DIAG_I32:
        hipLaunchKernelGGL(minmax_kernel<int32_t>, dim3(nblocks), dim3(256), 0, s,
                           static_cast<const int32_t *>(d_diag), dim, d_part, d_idx);
        break;
    default:
        hipLaunchKernelGGL(minmax_kernel<int16_t>, dim3(nblocks), dim3(256), 0, s,
                           static_cast<const int16_t *>(d_diag), dim, d_part, d_idx);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_widen_diag(const void *d_diag, int diag_type, uint64_t dim, void *d_out, hipStream_t s)
{
    const dim3 grid(grid_for(dim)), block(256);
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL((widen_kernel<double, double>), grid, block, 0, s, static_cast<const double *>(d_diag),
                           dim, static_cast<double *>(d_out));
        break;
    case DIAG_I32:
        hipLaunchKernelGGL((widen_kernel<int32_t, int32_t>), grid, block, 0, s,
                           static_cast<const int32_t *>(d_diag), dim, static_cast<int32_t *>(d_out));
        break;
    default:
        hipLaunchKernelGGL((widen_kernel<int16_t, int32_t>), grid, block, 0, s,
                           static_cast<const int16_t *>(d_diag), dim, static_cast<int32_t *>(d_out));
        break;
    }
    return hipGetLastError();
}

hipError_t launch_probabilities(const void *psi, bool c128, uint64_t dim, double *out, hipStream_t s)
{
    const dim3 grid(grid_for(dim)), block(256);
    if (c128)
        hipLaunchKernelGGL(prob_kernel<double2>, grid, block, 0, s, static_cast<const double2 *>(psi), dim, out);
    else
        hipLaunchKernelGGL(prob_kernel<float2>, grid, block, 0, s, static_cast<const float2 *>(psi), dim, out);
    return hipGetLastError();
}

hipError_t launch_topk(const void *psi, bool c128, uint64_t dim, int k, const void *diag, int diag_type,
                       uint64_t *d_idx, double *d_prob, double *d_cost, void *scratch, int nblocks, hipStream_t s)
{
    double *cp = static_cast<double *>(scratch);
    uint64_t *ci = reinterpret_cast<uint64_t *>(cp + (size_t)nblocks * k);
    if (c128)
        hipLaunchKernelGGL(topk_stage1<double2>, dim3(nblocks), dim3(256), 0, s, static_cast<const double2 *>(psi),
                           dim, k, cp, ci);
    else
        hipLaunchKernelGGL(topk_stage1<float2>, dim3(nblocks), dim3(256), 0, s, static_cast<const float2 *>(psi),
                           dim, k, cp, ci);
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL(topk_stage2<double>, dim3(1), dim3(256), 0, s, cp, ci, nblocks * k, k,
                           static_cast<const double *>(diag), d_idx, d_prob, d_cost);
        break;
    case DIAG_I32:
        hipLaunchKernelGGL(topk_stage2<int32_t>, dim3(1), dim3(256), 0, s, cp, ci, nblocks * k, k,
                           static_cast<const int32_t *>(diag), d_idx, d_prob, d_cost);
        break;
    default:
        hipLaunchKernelGGL(topk_stage2<int16_t>, dim3(1), dim3(256), 0, s, cp, ci, nblocks * k, k,
                           static_cast<const int16_t *>(diag), d_idx, d_prob, d_cost);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_local_tables(int n, int diag_type, const PartDesc *d_pd, const double *d_ell,
                               const int32_t *d_ell_i, int npairs, const int32_t *d_pair_ij, const double *d_pair_b,
                               const int32_t *d_pair_bi, const int32_t *d_qpu, double c0, int32_t c0_i, void *d_tables,
                               uint64_t total, hipStream_t s)
{
    const dim3 grid(grid_for(total)), block(256);
    switch (diag_type) {
    case DIAG_F64:
        hipLaunchKernelGGL((local_tables_kernel<false, double>), grid, block, 0, s, n, d_pd, d_ell, d_ell_i, npairs,
                           d_pair_ij, d_pair_b, d_pair_bi, d_qpu, c0, c0_i, static_cast<double *>(d_tables), total);
        break;
    case DIAG_I32:
        hipLaunchKernelGGL((local_tables_kernel<true, int32_t>), grid, block, 0, s, n, d_pd, d_ell, d_ell_i, npairs,
                           d_pair_ij, d_pair_b, d_pair_bi, d_qpu, c0, c0_i, static_cast<int32_t *>(d_tables), total);
        break;
    default:
        hipLaunchKernelGGL((local_tables_kernel<true, int16_t>), grid, block, 0, s, n, d_pd, d_ell, d_ell_i, npairs,
                           d_pair_ij, d_pair_b, d_pair_bi, d_qpu, c0, c0_i, static_cast<int16_t *>(d_tables), total);
        break;
    }
    return hipGetLastError();
}

}  // namespace qq
