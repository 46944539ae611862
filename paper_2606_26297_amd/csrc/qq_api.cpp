// qq_api.cpp -- host side of the C ABI declared in include/qaoa_qubo.h.
//
// Responsibilities: argument validation (before any device work), the
// canonical form of eq. (4)-(5), integer classification, the Pauli
// coefficients of eq. (9), device buffers of the problem handle, the pass
// planner that turns (n, p, mode) into a sequence of fused tile passes, and
// the evaluation entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "qq_internal.h"

using namespace qq;

namespace {

thread_local std::string g_err;

qq_status fail(qq_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define QQ_HIP(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(QQ_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Opt-in debugging aids, read from the environment at each call:
//   QQ_POISON  (non-empty, not "0"): fill every evaluation workspace with all-ones words (a NaN in
//              float and double) before the evaluation's kernels run, so a read of a byte that the
//              call has not written first turns its results into NaN;
//   QQ_LOG     (non-empty, not "0"): one line per evaluation call on stderr (entry point, sizes,
//              flags, status, host wall time).
bool env_flag(const char *name)
{
    const char *v = std::getenv(name);
    return v && *v && std::strcmp(v, "0") != 0;
}

hipError_t poison(void *ws, size_t bytes, hipStream_t stream)
{
    if (!env_flag("QQ_POISON") || bytes < 4) return hipSuccess;
    return launch_fill_u32(static_cast<uint32_t *>(ws), 0xffffffffu, bytes / 4, stream);
}

struct CallLog {
    const char *name;
    int n, p, batch, flags;
    std::chrono::steady_clock::time_point t0;
    qq_status st = QQ_OK;
    CallLog(const char *nm, int n_, int p_, int b_, int f_)
        : name(nm), n(n_), p(p_), batch(b_), flags(f_), t0(std::chrono::steady_clock::now()) {}
    qq_status operator()(qq_status s) { st = s; return s; }
    ~CallLog()
    {
        if (!env_flag("QQ_LOG")) return;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[qq] %s n=%d p=%d batch=%d flags=0x%x status=%d %.3f ms%s%s\n", name, n, p, batch, flags,
                     (int)st, ms, st == QQ_OK ? "" : ": ", st == QQ_OK ? "" : g_err.c_str());
    }
};

constexpr int kTelegateMaxN = 26;  // n + 2 qubits of complex128: 4 GiB
constexpr double kTwo31 = 2147483648.0;
// The specialised kernels serve every n up to QQ_MAX_N: a lane's amplitudes are addressed with a
// 32-bit byte offset of at most (15 + 3 * 2^pos8) * 8 bytes while pos8 <= 27, and with a 64-bit one
// for the partial high set of n >= 32 (pos8 >= 28).  The persistent many-problem kernel keeps the
// 32-bit form only, so it serves n <= 31.
constexpr int kFastMaxN = QQ_MAX_N;
constexpr int kManyMaxN = 31;
constexpr double kTwo15 = 32768.0;

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

int diag_bytes_of(int t) { return t == DIAG_F64 ? 8 : t == DIAG_I32 ? 4 : 2; }

struct ProfRec {
    hipEvent_t start, stop;
    qq_launch_record meta;
};
bool g_prof = false;
std::vector<ProfRec> g_prof_log;

// Event-timed record of one auxiliary launch (cost diagonal, probabilities, top-k, ...) when
// profiling is on; `bytes` is the launch's algorithmic memory traffic.
template <typename F>
hipError_t prof_aux(int kind, int n, int diag_bytes, double bytes, hipStream_t stream, F launch)
{
    if (!g_prof) return launch();
    ProfRec rec{};
    hipError_t e;
    if ((e = hipEventCreate(&rec.start)) != hipSuccess || (e = hipEventCreate(&rec.stop)) != hipSuccess) return e;
    if ((e = hipEventRecord(rec.start, stream)) != hipSuccess) return e;
    if ((e = launch()) != hipSuccess) return e;
    if ((e = hipEventRecord(rec.stop, stream)) != hipSuccess) return e;
    rec.meta.kind = kind;
    rec.meta.pass_kind = -1;
    rec.meta.n = n;
    rec.meta.batch = 1;
    rec.meta.diag_bytes = diag_bytes;
    rec.meta.bytes = bytes;
    g_prof_log.push_back(rec);
    return hipSuccess;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

struct qq_problem {
    int n = 0;
    int device = 0;
    uint64_t dim = 0;
    std::vector<double> H, f;
    double c0 = 0.0;
    std::vector<double> ell;  // n
    std::vector<double> b;    // n*n, strict upper triangle
    bool is_integer = false;
    int diag_type = DIAG_F64;
    int32_t c0_i = 0;
    std::vector<int32_t> ell_i;
    // nonzero couplings in row-major order
    std::vector<int32_t> pair_ij;
    std::vector<double> pair_b;
    std::vector<int32_t> pair_bi;
    // device copies
    void *d_diag = nullptr;
    double *d_ell = nullptr;
    int32_t *d_ell_i = nullptr;
    int32_t *d_pair_ij = nullptr;
    double *d_pair_b = nullptr;
    int32_t *d_pair_bi = nullptr;
    // Couplings among four consecutive qubits R_j = q + j, for the register-cost reconstruction of
    // the pass kernels: regq[16 q + r] = sum over the bits k > j of r of b_{R_j R_k}, j the lowest
    // bit of r (0 for r = 0 and single bits); q = 0 .. n - 4.
    double *d_regq = nullptr;
    // The same sums per factor of the partitioned phase (set by qq_set_allocation): [factor][q][16],
    // factors 0 .. M-1 the QPU-local couplings, factor M the cross-QPU couplings.
    double *d_part_cq = nullptr;
    // summary
    double alpha = 0, sigma_c = 0, cmin = 0, cmax = 0;
    uint64_t argmin = 0;
    // allocation / partitioned phases
    int num_qpus = 0;
    std::vector<int32_t> qpu;
    int64_t cross_terms = -1;
    int32_t *d_qpu = nullptr;
    void *d_tables = nullptr;
    void *d_cross = nullptr;
    PartDesc *d_part = nullptr;
    // schedules pinned by qq_set_schedule / qq_autotune, keyed by (p, batch, planning flags)
    struct Sched {
        int p, batch, flags, G, pairing, blocked, set_order;
        double ms;
    };
    std::vector<Sched> sched;
    // graphs captured on this problem: they hold its device pointers, so the problem is not
    // destroyed and its allocation not replaced while any exists
    int graphs = 0;
    // Per-tile cost tables of the complex64 per-pass kernels (launch_cost_table), in one allocation: one
    // per tile geometry (high, pos4, pos8) of every set plan and per cost layout (the tile's lane and wave
    // qubits at lane_q, its register qubits at the other run); each is [tiles][kCostRow] rows followed
    // by the per-thread constants [256][8].  Built once at creation, so no evaluation allocates for them.
    struct CostTab {
        int high, pos4, pos8, lane_q;
        size_t off;  // in doubles from d_ctab
    };
    std::vector<CostTab> ctabs;
    double *d_ctab = nullptr;
    // the same tables of the cross-QPU couplings alone (qq_set_allocation), read by the partitioned phases
    std::vector<CostTab> xtabs;
    double *d_xtab = nullptr;

    ~qq_problem()
    {
        void *ptrs[] = {d_diag, d_ell, d_ell_i, d_pair_ij, d_pair_b, d_pair_bi, d_regq, d_part_cq, d_qpu, d_tables, d_cross,
                        d_part, d_ctab, d_xtab};
        if (dim) (void)hipSetDevice(device);
        for (void *q : ptrs)
            if (q) (void)hipFree(q);
    }
};

namespace {

// ---- pass planning -------------------------------------------------------------------------
// Qubit sets mixed by one pass.  Set 0 is qubits 0..11 (a contiguous tile);
// every further set is a high tile: qubits 0..3 (passive) plus two runs of
// four qubits, pos4..pos4+3 and pos8..pos8+3, of which the `active` tile bits
// are mixed.
struct SetDesc {
    int high;
    int pos4, pos8;
    uint16_t active;
};

// High-set layout.  When the qubits above 11 split into full sets (n - 12 a
// multiple of 8) they are cut into 4-qubit runs R_0..R_{m-1}, paired per
// `pairing`: 0 pairs run i with run m-1-i (the default, measured fastest on
// MI355X at n = 28: it spreads the qubits of the largest address strides over
// both high sets), 1 pairs adjacent runs (2i, 2i+1), 2 pairs run i with run
// i + m/2.  Otherwise each set is a contiguous 8-qubit window [h, h+8), the last
// one shifted down to end at n with its already-covered qubits inactive.
constexpr int kPairings = 3;

bool pairing_applies(int n) { return n > kTileBits && (n - kTileBits) % 8 == 0 && (n - kTileBits) / 4 >= 4; }

// Visiting order of the sets in a layer: set_order 0 takes the qubit-0..11 set first, 1 second.
// The zig-zag reverses the order every layer, so the first and last sets are where a pass mixes,
// applies the next phase and mixes again; with the 12-qubit set in the middle those passes mix at
// most 8 qubits (less arithmetic per byte).  Measured on MI355X (energy + gradient, 3-regular
// instances): equal or faster at every n tried, 22 to 32 (by up to 9%), so it is the default
// wherever there are three or more sets.  The persistent many-problem launch keeps order 0.
int num_sets(int n);
bool set_order_applies(int n) { return num_sets(n) >= 3; }
int default_set_order(int n) { return set_order_applies(n) ? 1 : 0; }

std::vector<SetDesc> make_sets(int n, int pairing = 0)
{
    std::vector<SetDesc> sets;
    if (n <= kTileBits) {
        sets.push_back({0, 4, 8, (uint16_t)((1u << n) - 1u)});
        return sets;
    }
    sets.push_back({0, 4, 8, 0x0fff});
    if ((n - kTileBits) % 8 == 0) {
        const int m = (n - kTileBits) / 4;
        for (int i = 0; i < m / 2; ++i) {
            const int a = pairing == 1 ? 2 * i : i;
            const int c = pairing == 1 ? 2 * i + 1 : pairing == 2 ? i + m / 2 : m - 1 - i;
            sets.push_back({1, kTileBits + 4 * a, kTileBits + 4 * c, 0x0ff0});
        }
        return sets;
    }
    for (int q0 = kTileBits; q0 < n; q0 += 8) {
        const int q1 = std::min(n, q0 + 8);
        const int h = std::min(q0, n - 8);
        uint16_t act = 0;
        for (int q = q0; q < q1; ++q) act |= (uint16_t)(1u << (4 + q - h));
        sets.push_back({1, h, h + 4, act});
    }
    return sets;
}

int num_sets(int n) { return (int)make_sets(n, 0).size(); }

struct PassPlan {
    int fkind = -1;  // FastPassKind of this pass (multi-pass plans)
    int fk = 0;      // its layer index
    int set = 0;
    uint32_t flags = 0;
    int nstates = 1;
    std::vector<Op> ops;
    std::vector<int> slot_out;  // local slot -> output index
};

struct Plan {
    std::vector<SetDesc> sets;
    std::vector<PassPlan> passes;
    int nslots = 0;
};

enum PlanMode { PM_ENERGY = 1, PM_GRAD = 2, PM_STORE = 4, PM_PART = 8 };

int out_energy() { return 0; }
int out_gamma(int k) { return 1 + 2 * k; }
int out_beta(int k) { return 2 + 2 * k; }

int local_slot(PassPlan &pp, int out)
{
    for (size_t s = 0; s < pp.slot_out.size(); ++s)
        if (pp.slot_out[s] == out) return (int)s;
    pp.slot_out.push_back(out);
    return (int)pp.slot_out.size() - 1;
}

Op op_mix(PassPlan &pp, int k, bool inverse, uint16_t active, int states, int out)
{
    Op o{};
    o.kind = OP_MIX;
    o.layer = (uint8_t)k;
    o.states = (uint8_t)states;
    o.flags = inverse ? OPF_INVERSE : 0;
    o.active = active;
    o.slot = (uint8_t)(out >= 0 ? local_slot(pp, out) : kNoSlot);
    return o;
}

Op op_phase(int k, bool inverse, int states, bool part)
{
    Op o{};
    o.kind = OP_PHASE;
    o.layer = (uint8_t)k;
    o.states = (uint8_t)states;
    o.flags = (uint8_t)((inverse ? OPF_INVERSE : 0) | (part ? OPF_PARTITIONED : 0));
    o.slot = kNoSlot;
    return o;
}

Op op_acc(PassPlan &pp, uint8_t kind, int k, int out, uint8_t flags)
{
    Op o{};
    o.kind = kind;
    o.layer = (uint8_t)k;
    o.states = 3;
    o.flags = flags;
    o.slot = (uint8_t)local_slot(pp, out);
    return o;
}

// Passes for one evaluation.  Layer k (0-based) visits the qubit sets in
// ascending order when k is even and descending when k is odd ("zig-zag"),
// so the last set of layer k is the first set of layer k+1: that pass mixes
// layer k on the set, applies phase k+1 and mixes layer k+1 on the same set.
// A forward evaluation with s sets takes 1 + p(s-1) passes.  The adjoint
// sweep runs the same zig-zag backwards over (psi, lambda).
Plan make_plan(int n, int p, int mode, int pairing = 0, int set_order = 0)
{
    Plan plan;
    plan.sets = make_sets(n, pairing);
    const int s = (int)plan.sets.size();
    std::vector<int> vis(s);
    for (int i = 0; i < s; ++i) vis[i] = i;
    if (set_order == 1 && s >= 3) std::swap(vis[0], vis[1]);
    const bool grad = mode & PM_GRAD, energy = mode & (PM_ENERGY | PM_GRAD), store = mode & PM_STORE,
               part = mode & PM_PART;
    auto order = [&](int k) {
        std::vector<int> o(s);
        for (int i = 0; i < s; ++i) o[i] = (k % 2 == 0) ? vis[i] : vis[s - 1 - i];
        return o;
    };
    auto act = [&](int set) { return plan.sets[set].active; };

    if (s == 1) {
        PassPlan pp;
        pp.set = 0;
        pp.flags = PF_INIT | (store ? PF_STORE_PSI : 0);
        pp.nstates = grad ? 2 : 1;
        for (int k = 0; k < p; ++k) {
            pp.ops.push_back(op_phase(k, false, 1, part));
            pp.ops.push_back(op_mix(pp, k, false, act(0), 1, -1));
        }
        if (grad) {
            pp.ops.push_back(op_acc(pp, OP_ENERGY_LAMBDA, p - 1, out_energy(), 0));
            for (int k = p - 1; k >= 0; --k) {
                pp.ops.push_back(op_mix(pp, k, true, act(0), 3, out_beta(k)));
                pp.ops.push_back(op_acc(pp, OP_GGAMMA, k, out_gamma(k),
                                        (uint8_t)((k > 0 ? OPF_UNPHASE : 0) | (part ? OPF_PARTITIONED : 0))));
            }
        } else if (energy) {
            pp.ops.push_back(op_acc(pp, OP_ENERGY, p - 1, out_energy(), 0));
        }
        plan.passes.push_back(pp);
    } else {
        {
            PassPlan pp;
            pp.fkind = FK_FIRST;
            pp.set = order(0)[0];
            pp.flags = PF_INIT | PF_STORE_PSI;
            pp.ops.push_back(op_phase(0, false, 1, part));
            pp.ops.push_back(op_mix(pp, 0, false, act(pp.set), 1, -1));
            plan.passes.push_back(pp);
        }
        for (int k = 0; k < p; ++k) {
            const auto o = order(k);
            for (int idx = 1; idx < s; ++idx) {
                const int set = o[idx];
                PassPlan pp;
                pp.set = set;
                pp.fk = k;
                if (idx < s - 1) {
                    pp.fkind = FK_MID;
                    pp.flags = PF_LOAD_PSI | PF_STORE_PSI;
                    pp.ops.push_back(op_mix(pp, k, false, act(set), 1, -1));
                } else if (k < p - 1) {
                    pp.fkind = FK_TURN;
                    pp.flags = PF_LOAD_PSI | PF_STORE_PSI;
                    pp.ops.push_back(op_mix(pp, k, false, act(set), 1, -1));
                    pp.ops.push_back(op_phase(k + 1, false, 1, part));
                    pp.ops.push_back(op_mix(pp, k + 1, false, act(set), 1, -1));
                } else if (grad) {
                    // psi in memory stays the state before this set's mixer; lambda is
                    // formed in registers and leaves with the set already un-mixed.
                    pp.fkind = FK_LASTG;
                    pp.flags = PF_LOAD_PSI | PF_STORE_LAM;
                    pp.nstates = 2;
                    pp.ops.push_back(op_mix(pp, k, false, act(set), 1, -1));
                    pp.ops.push_back(op_acc(pp, OP_ENERGY_LAMBDA, k, out_energy(), 0));
                    pp.ops.push_back(op_mix(pp, k, true, act(set), 3, out_beta(k)));
                } else {
                    pp.fkind = FK_LAST;
                    pp.flags = PF_LOAD_PSI | (store ? PF_STORE_PSI : 0);
                    pp.ops.push_back(op_mix(pp, k, false, act(set), 1, -1));
                    if (energy) pp.ops.push_back(op_acc(pp, OP_ENERGY, k, out_energy(), 0));
                }
                plan.passes.push_back(pp);
            }
        }
        if (grad) {
            for (int k = p - 1; k >= 0; --k) {
                auto r = order(k);
                std::reverse(r.begin(), r.end());
                for (int idx = 1; idx < s; ++idx) {
                    const int set = r[idx];
                    PassPlan pp;
                    pp.set = set;
                    pp.nstates = 2;
                    pp.fk = k;
                    if (idx < s - 1) {
                        pp.fkind = FK_BMID;
                        pp.flags = PF_LOAD_PSI | PF_LOAD_LAM | PF_STORE_PSI | PF_STORE_LAM;
                        pp.ops.push_back(op_mix(pp, k, true, act(set), 3, out_beta(k)));
                    } else if (k > 0) {
                        pp.fkind = FK_BTURN;
                        pp.flags = PF_LOAD_PSI | PF_LOAD_LAM | PF_STORE_PSI | PF_STORE_LAM;
                        pp.ops.push_back(op_mix(pp, k, true, act(set), 3, out_beta(k)));
                        pp.ops.push_back(op_acc(pp, OP_GGAMMA, k, out_gamma(k),
                                                (uint8_t)(OPF_UNPHASE | (part ? OPF_PARTITIONED : 0))));
                        pp.ops.push_back(op_mix(pp, k - 1, true, act(set), 3, out_beta(k - 1)));
                    } else {
                        pp.fkind = FK_BLAST;
                        pp.flags = PF_LOAD_PSI | PF_LOAD_LAM;
                        pp.ops.push_back(op_mix(pp, 0, true, act(set), 3, out_beta(0)));
                        pp.ops.push_back(op_acc(pp, OP_GGAMMA, 0, out_gamma(0), 0));
                    }
                    plan.passes.push_back(pp);
                }
            }
        }
    }
    for (auto &pp : plan.passes) plan.nslots += (int)pp.slot_out.size();
    return plan;
}

uint64_t tiles_per_state(int n) { return n <= kTileBits ? 1ull : (1ull << (n - kTileBits)); }

int choose_G(int n, int B)
{
    const uint64_t T = tiles_per_state(n);
    uint64_t target = std::max<uint64_t>(1, 4096 / (uint64_t)B);
    uint64_t G = 1;
    while (G * 2 <= target && G * 2 <= T) G *= 2;
    return (int)G;
}

// With gradients the complex64 per-pass kernels keep psi and lambda of a state in one region, in
// alternating blocks of 2^kIlvBit amplitudes (psi's block, then lambda's), so the rows of a tile of
// both states lie 512 KiB apart instead of a whole state array apart.  Measured at n = 28, p = 8,
// 64 states: step 2262 ms with separate arrays, 2224 / 2214 / 2227 / 2253 ms with blocks of 2^12,
// 2^16, 2^20, 2^24 amplitudes (the adjoint turn on the set {12..15, 24..27}: 105 ms apart, 96 ms
// interleaved by 2^16); n = 32 with four QPUs, partitioned: 592 -> 565 ms.
constexpr int kIlvBit = 16;

struct Layout {
    size_t psi = 0, lam = 0, partial = 0, params = 0, out = 0, total = 0;
    size_t stride = 0;  // amplitudes from one state's region to the next
    int ilv = 0;        // 0, or kIlvBit: psi and lambda interleaved in blocks of 2^kIlvBit amplitudes
    int G = 1;
    int blocked = 0;  // tile order of the specialised kernels
    int nslots = 0;
};

Layout make_layout(const qq_problem *pb, int p, int B, int flags, const Plan &plan, int G = 0)
{
    Layout L;
    const size_t es = (flags & QQ_C128) ? 16 : 8;
    const bool grad = flags & QQ_GRAD;
    const bool multi = plan.sets.size() > 1;
    // interleave where every pass is a complex64 per-pass kernel, the state has more than one block,
    // and no run of four qubits of a high set straddles bit kIlvBit (the low set's runs lie below it)
    if (grad && multi && !(flags & QQ_C128) && pb->n <= kFastMaxN && pb->n > kIlvBit) {
        bool ok = true;
        for (const PassPlan &pp : plan.passes) ok = ok && pp.fkind >= 0;
        auto one_side = [](int q) { return q >= kIlvBit || q + 4 <= kIlvBit; };
        for (const SetDesc &sd : plan.sets) ok = ok && (!sd.high || (one_side(sd.pos4) && one_side(sd.pos8)));
        if (ok) L.ilv = kIlvBit;
    }
    L.stride = L.ilv ? 2 * (size_t)pb->dim : (size_t)pb->dim;
    const size_t state = L.stride * es * (size_t)B;
    L.G = G > 0 ? G : choose_G(pb->n, B);
    L.nslots = plan.nslots;
    size_t off = 0;
    L.psi = off;
    off += align_up(state);  // also used by qq_state for a single-pass plan
    L.lam = L.ilv ? L.psi + ((size_t)1 << L.ilv) * es : off;
    if (grad && multi && !L.ilv) off += align_up(state);
    L.partial = off;
    off += align_up((size_t)std::max(1, plan.nslots) * B * L.G * sizeof(double));
    L.params = off;
    off += align_up((size_t)B * 2 * p * sizeof(double));
    L.out = off;
    off += align_up((size_t)B * (1 + 2 * p) * sizeof(double));
    L.total = off;
    return L;
}

int plan_mode(int flags, bool store)
{
    int m = 0;
    if (flags & QQ_ENERGY) m |= PM_ENERGY;
    if (flags & QQ_GRAD) m |= PM_GRAD | PM_ENERGY;
    if (flags & QQ_PARTITIONED) m |= PM_PART;
    if (store) m |= PM_STORE;
    return m;
}

// Flags that change the plan or the layout (the energy is always computed).
int sched_flags(int flags) { return flags & (QQ_GRAD | QQ_PARTITIONED | QQ_C128); }

const qq_problem::Sched *find_sched(const qq_problem *pb, int p, int batch, int flags)
{
    for (const auto &e : pb->sched)
        if (e.p == p && e.batch == batch && e.flags == sched_flags(flags)) return &e;
    return nullptr;
}

// Plan and layout of an evaluation, under the problem's pinned schedule if any.
Plan plan_for(const qq_problem *pb, int p, int batch, int flags, bool store)
{
    const auto *e = find_sched(pb, p, batch, flags);
    return make_plan(pb->n, p, plan_mode(flags | QQ_ENERGY, store), e ? e->pairing : 0,
                     e ? e->set_order : default_set_order(pb->n));
}

Layout layout_for(const qq_problem *pb, int p, int batch, int flags, const Plan &plan)
{
    const auto *e = find_sched(pb, p, batch, flags);
    Layout L = make_layout(pb, p, batch, flags, plan, e ? e->G : 0);
    L.blocked = e ? e->blocked : 0;
    return L;
}

qq_status check_params_host(const double *params, size_t count)
{
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return fail(QQ_E_INVALID, "params[%zu] is not finite", i);
    return QQ_OK;
}

qq_status check_device_fits(int device, size_t bytes, const char *what)
{
    size_t freeb = 0, totalb = 0;
    QQ_HIP(hipSetDevice(device));
    QQ_HIP(hipMemGetInfo(&freeb, &totalb));
    if (bytes > totalb)
        return fail(QQ_E_TOO_LARGE, "%s needs %zu bytes; the device has %zu in total", what, bytes, totalb);
    return QQ_OK;
}

// Algorithmic HBM bytes of one pass: every state load and store (per state),
// plus one cost-diagonal read per operation that needs C(z) -- counted once per
// launch, since every state of the batch reads the same diagonal entries (the
// partitioned phase also reads the cross-QPU diagonal).
double pass_bytes(const qq_problem *pb, const PassPlan &pp, int B, bool c128, bool fast)
{
    const double es = c128 ? 16.0 : 8.0, d = diag_bytes_of(pb->diag_type);
    int moves = 0;
    if (pp.flags & PF_LOAD_PSI) ++moves;
    if (pp.flags & PF_LOAD_LAM) ++moves;
    if (pp.flags & PF_STORE_PSI) ++moves;
    if (pp.flags & PF_STORE_LAM) ++moves;
    // reads of the cost diagonal and of the cross-QPU diagonal (a partitioned phase reads the
    // cross diagonal and the small local tables instead of the cost diagonal)
    double diag_reads = 0, cross_reads = 0;
    for (const Op &o : pp.ops) {
        const bool part = (o.flags & OPF_PARTITIONED) != 0;
        if ((o.kind == OP_PHASE && !part) || o.kind == OP_ENERGY || o.kind == OP_ENERGY_LAMBDA || o.kind == OP_GGAMMA)
            diag_reads += 1;
        if ((o.kind == OP_PHASE || (o.kind == OP_GGAMMA && (o.flags & OPF_UNPHASE))) && part) cross_reads += 1;
    }
    // the specialised kernels read one table row per tile of 4096 entries in place of the cost (and
    // cross-QPU) diagonal, forming the 4096 values from it
    if (fast) {
        diag_reads *= kCostRow * sizeof(double) / (4096.0 * d);
        cross_reads *= kCostRow * sizeof(double) / (4096.0 * d);
    }
    return (double)pb->dim * (B * moves * es + (diag_reads + cross_reads) * d);
}

// The tables a problem of n variables needs: one per set geometry of every pairing and per layout.
std::vector<qq_problem::CostTab> cost_table_list(int n)
{
    std::vector<qq_problem::CostTab> tabs;
    if (n <= kTileBits || n > kFastMaxN) return tabs;
    auto add = [&](const SetDesc &sd, int lane_q) {
        for (const auto &t : tabs)
            if (t.high == sd.high && t.pos4 == sd.pos4 && t.pos8 == sd.pos8 && t.lane_q == lane_q) return;
        tabs.push_back({sd.high, sd.pos4, sd.pos8, lane_q, 0});
    };
    for (int pr = 0; pr < (pairing_applies(n) ? kPairings : 1); ++pr)
        for (const SetDesc &sd : make_sets(n, pr)) {
            add(sd, sd.pos4);
            add(sd, sd.pos8);
        }
    return tabs;
}

size_t cost_table_bytes(int n)
{
    if (n <= kTileBits || n > kFastMaxN) return 0;
    return cost_table_list(n).size() * ((size_t)tiles_per_state(n) * kCostRow + 256 * 8) * sizeof(double);
}

// Per-tile tables of one quadratic cost c0 + sum l_i z_i + sum_{i<j} b_ij z_i z_j (see
// qq_problem::CostTab): the rows on the device from the device coefficient lists, the per-thread
// constants (P(E) and l_Rj + sum_{q in E} b_q,Rj, with E the thread's lane and wave bits) on the host.
// `ell` / `B` give the host coefficients; `*d_out` receives the one allocation.
template <typename BF>
qq_status build_tables(int n, const std::vector<double> &ell, BF B, const double *d_ell, int np,
                       const int32_t *d_pij, const double *d_pb, double c0, std::vector<qq_problem::CostTab> &tabs,
                       double **d_out, hipStream_t stream)
{
    tabs = cost_table_list(n);
    if (tabs.empty()) return QQ_OK;
    const uint64_t T = tiles_per_state(n);
    const size_t per = (size_t)T * kCostRow + 256 * 8;
    if (hipMalloc((void **)d_out, per * tabs.size() * sizeof(double)) != hipSuccess)
        return fail(QQ_E_NOMEM, "hipMalloc(%zu) for the cost tables failed", per * tabs.size() * sizeof(double));
    std::vector<double> thr(256 * 8 * tabs.size(), 0.0);
    for (size_t k = 0; k < tabs.size(); ++k) {
        qq_problem::CostTab &tb = tabs[k];
        tb.off = k * per;
        const int lq = tb.lane_q, rq = lq == tb.pos4 ? tb.pos8 : tb.pos4;
        QQ_HIP(launch_cost_table(n, tb.high, tb.pos4, tb.pos8, lq, rq, T, d_ell, np, d_pij, d_pb, c0, *d_out + tb.off,
                                 stream));
        const int eq[8] = {0, 1, 2, 3, lq, lq + 1, lq + 2, lq + 3};
        for (int t = 0; t < 256; ++t) {
            double P = 0.0;
            for (int a = 0; a < 8; ++a) {
                if (!((t >> a) & 1)) continue;
                P += ell[eq[a]];
                for (int c = a + 1; c < 8; ++c)
                    if ((t >> c) & 1) P += B(eq[a], eq[c]);
            }
            double *row = &thr[(k * 256 + t) * 8];
            row[0] = P;
            for (int j = 0; j < 4; ++j) {
                double q = ell[rq + j];
                for (int a = 0; a < 8; ++a)
                    if ((t >> a) & 1) q += B(eq[a], rq + j);
                row[1 + j] = q;
            }
        }
    }
    for (size_t k = 0; k < tabs.size(); ++k)
        QQ_HIP(hipMemcpyAsync(*d_out + tabs[k].off + (size_t)T * kCostRow, &thr[k * 256 * 8], 256 * 8 * sizeof(double),
                              hipMemcpyHostToDevice, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

// The cost tables of the whole cost (at problem creation).
qq_status build_cost_tables(qq_problem *pb, hipStream_t stream)
{
    const int n = pb->n;
    auto B = [&](int i, int j) { return i < j ? pb->b[(size_t)i * n + j] : pb->b[(size_t)j * n + i]; };
    return build_tables(n, pb->ell, B, pb->d_ell, (int)pb->pair_b.size(), pb->d_pair_ij, pb->d_pair_b, pb->c0,
                        pb->ctabs, &pb->d_ctab, stream);
}

const double *find_table(const std::vector<qq_problem::CostTab> &tabs, const double *base, const SetDesc &sd,
                         int lane_q)
{
    for (const auto &t : tabs)
        if (t.high == sd.high && t.pos4 == sd.pos4 && t.pos8 == sd.pos8 && t.lane_q == lane_q) return base + t.off;
    return nullptr;
}

const double *find_cost_table(const qq_problem *pb, const SetDesc &sd, int lane_q)
{
    return find_table(pb->ctabs, pb->d_ctab, sd, lane_q);
}

// Run every pass of a plan and the final reduction.  `ws` is device memory laid out by `L`.
qq_status run_plan(qq_problem *pb, const Plan &plan, const Layout &L, int p, int B, int flags, char *ws,
                   const double *d_params, hipStream_t stream, bool capturing = false)
{
    const bool prof = g_prof && !capturing;  // no event records inside a captured graph
    const bool c128 = flags & QQ_C128;
    const uint64_t T = tiles_per_state(pb->n);
    const size_t es = c128 ? 16 : 8;
    (void)es;
    if (plan.nslots > kMaxSlots) return fail(QQ_E_UNSUPPORTED, "plan needs %d accumulator slots (max %d)", plan.nslots, kMaxSlots);
    // Specialised complex64 kernels serve multi-pass, non-partitioned plans.
    const bool use_fast = !c128 && plan.sets.size() > 1 && pb->n <= kFastMaxN;
    int slot_base = 0;
    for (const auto &pp : plan.passes) {
        if ((int)pp.ops.size() > kMaxOps) return fail(QQ_E_UNSUPPORTED, "pass has %zu ops (max %d)", pp.ops.size(), kMaxOps);
        const SetDesc &sd = plan.sets[pp.set];
        PassArgs a;
        std::memset(&a, 0, sizeof a);
        a.n = pb->n;
        a.p = p;
        a.B = B;
        a.G = L.G;
        a.tiles = T;
        a.dim_mask = pb->dim - 1;
        a.pos4 = sd.pos4;
        a.pos8 = sd.pos8;
        a.high = sd.high;
        a.w1 = sd.pos4 - 4;
        a.w2 = sd.pos8 - sd.pos4 - 4;
        a.flags = pp.flags;
        a.nops = (int)pp.ops.size();
        a.nslots = (int)pp.slot_out.size();
        a.slot_base = slot_base;
        a.slot_stride = B * L.G;
        a.amp0 = 1.0 / std::sqrt((double)pb->dim);
        a.params = d_params;
        a.diag = pb->d_diag;
        a.psi = ws + L.psi;
        a.lam = ws + L.lam;
        a.state_stride = L.stride;
        a.partial = reinterpret_cast<double *>(ws + L.partial);
        a.part_tables = pb->d_tables;
        a.cross_diag = pb->d_cross;
        a.part = pb->d_part;
        for (size_t i = 0; i < pp.ops.size(); ++i) a.ops[i] = pp.ops[i];
        ProfRec rec{};
        if (prof) {
            QQ_HIP(hipEventCreate(&rec.start));
            QQ_HIP(hipEventCreate(&rec.stop));
            QQ_HIP(hipEventRecord(rec.start, stream));
        }
        if (use_fast && pp.fkind >= 0) {
            FastPassParams fp;
            fp.blocked = L.blocked;
            fp.part = (flags & QQ_PARTITIONED) ? 1 : 0;
            fp.part_desc = pb->d_part;
            fp.part_tables = pb->d_tables;
            fp.B = B;
            fp.G = L.G;
            fp.p = p;
            fp.k = pp.fk;
            fp.tiles = T;
            fp.dim_mask = pb->dim - 1;
            fp.pos4 = sd.pos4;
            fp.pos8 = sd.pos8;
            fp.w1 = sd.pos4 - 4;
            fp.w2 = sd.pos8 - sd.pos4 - 4;
            fp.active = sd.active;
            fp.store_psi = (pp.flags & PF_STORE_PSI) ? 1 : 0;
            fp.slot_base = slot_base;
            fp.slot_stride = B * L.G;
            fp.amp0 = a.amp0;
            fp.params = d_params;
            fp.diag = pb->d_diag;
            fp.psi = a.psi;
            fp.lam = a.lam;
            fp.state_stride = L.stride;
            fp.ilv = L.ilv;
            fp.partial = a.partial;
            fp.cq = pb->d_regq + 16 * (pp.fkind == FK_FIRST ? sd.pos8 : sd.pos4);
            fp.part_cq = pb->d_part_cq;
            fp.part_cq_runs = std::max(1, pb->n - 3);
            fp.shift = pb->alpha;
            // the table of the layout the pass reads the cost in: lanes at pos4 for the first pass, at pos8 else
            fp.ctab = find_cost_table(pb, sd, pp.fkind == FK_FIRST ? sd.pos4 : sd.pos8);
            if (!fp.ctab) return fail(QQ_E_DEVICE, "no cost table for the set at qubits %d / %d", sd.pos4, sd.pos8);
            fp.cthr = fp.ctab + (size_t)T * kCostRow;
            fp.xtab = fp.xthr = nullptr;
            if (fp.part) {
                fp.xtab = find_table(pb->xtabs, pb->d_xtab, sd, pp.fkind == FK_FIRST ? sd.pos4 : sd.pos8);
                if (!fp.xtab) return fail(QQ_E_DEVICE, "no cross table for the set at qubits %d / %d", sd.pos4, sd.pos8);
                fp.xthr = fp.xtab + (size_t)T * kCostRow;
            }
            QQ_HIP(launch_fast_pass(pp.fkind, sd.high != 0, pb->diag_type, fp, stream));
        } else {
            QQ_HIP(launch_pass(a, c128, pp.nstates, pb->diag_type, stream));
        }
        if (prof) {
            QQ_HIP(hipEventRecord(rec.stop, stream));
            rec.meta.kind = pp.nstates > 1 ? 2 : 1;
            rec.meta.pass_kind = (use_fast && pp.fkind >= 0) ? pp.fkind : -1;
            rec.meta.part = (flags & QQ_PARTITIONED) && (pp.fkind == FK_FIRST || pp.fkind == FK_TURN ||
                                                          pp.fkind == FK_BTURN || !use_fast) ? 1 : 0;
            rec.meta.high = sd.high;
            rec.meta.full = !sd.high || sd.active == 0x0ff0;
            rec.meta.diag_bytes = diag_bytes_of(pb->diag_type);
            rec.meta.c128 = c128;
            rec.meta.n = pb->n;
            rec.meta.batch = B;
            rec.meta.bytes = pass_bytes(pb, pp, B, c128, use_fast && pp.fkind >= 0);
            g_prof_log.push_back(rec);
        }
        slot_base += a.nslots;
    }
    FinalizeArgs fa;
    std::memset(&fa, 0, sizeof fa);
    fa.B = B;
    fa.G = L.G;
    fa.p = p;
    fa.nslots = plan.nslots;
    fa.escale = pb->n < kTileBits ? std::ldexp(1.0, pb->n - kTileBits) : 1.0;
    // the specialised kernels accumulate with C - alpha (every pass of a multi-pass complex64 plan)
    fa.shift = (use_fast && !plan.passes.empty() && plan.passes[0].fkind >= 0) ? pb->alpha : 0.0;
    fa.partial = reinterpret_cast<const double *>(ws + L.partial);
    fa.out = reinterpret_cast<double *>(ws + L.out);
    int s = 0;
    for (const auto &pp : plan.passes)
        for (int o : pp.slot_out) fa.slot_out[s++] = (uint16_t)o;
    ProfRec rec{};
    if (prof) {
        QQ_HIP(hipEventCreate(&rec.start));
        QQ_HIP(hipEventCreate(&rec.stop));
        QQ_HIP(hipEventRecord(rec.start, stream));
    }
    QQ_HIP(launch_finalize(fa, stream));
    if (prof) {
        QQ_HIP(hipEventRecord(rec.stop, stream));
        rec.meta.kind = 3;
        rec.meta.pass_kind = -1;
        rec.meta.c128 = c128;
        rec.meta.n = pb->n;
        rec.meta.batch = B;
        rec.meta.bytes = (double)plan.nslots * B * L.G * sizeof(double);
        g_prof_log.push_back(rec);
    }
    return QQ_OK;
}

qq_status validate_eval(const qq_problem *pb, int p, int batch, int flags)
{
    if (!pb) return fail(QQ_E_INVALID, "problem is NULL");
    if (p < 1 || p > QQ_MAX_P) return fail(QQ_E_INVALID, "p = %d outside [1, %d]", p, QQ_MAX_P);
    if (batch < 1) return fail(QQ_E_INVALID, "batch = %d must be >= 1", batch);
    const int known = QQ_ENERGY | QQ_GRAD | QQ_PARTITIONED | QQ_C128 | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE;
    if (flags & ~known) return fail(QQ_E_INVALID, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & QQ_PARTITIONED) && pb->num_qpus == 0)
        return fail(QQ_E_ALLOCATION, "QQ_PARTITIONED requested but no allocation is set (qq_set_allocation)");
    return QQ_OK;
}

// Evaluate a plan for `batch` parameter sets into ws; leaves results at ws + L.out on the device.
qq_status eval_core(qq_problem *pb, int p, int batch, const double *params, int flags, const Plan &plan,
                    const Layout &L, char *ws, hipStream_t stream)
{
    const double *d_params = params;
    if (!(flags & QQ_PARAMS_ON_DEVICE)) {
        d_params = reinterpret_cast<const double *>(ws + L.params);
        QQ_HIP(hipMemcpyAsync(ws + L.params, params, (size_t)batch * 2 * p * sizeof(double), hipMemcpyHostToDevice,
                              stream));
    }
    return run_plan(pb, plan, L, p, batch, flags, ws, d_params, stream);
}

// ---- many problems in one persistent launch -----------------------------------------------
// One launch per cost-diagonal element type present (the kernel is specialised on it).
struct ManyGroup {
    int diag_type = DIAG_F64;
    std::vector<int> members;  // problem indices, in queue priority order
    std::vector<ManyInst> inst;
    std::vector<ManyPass> pass;
    std::vector<PassArgs> gpass;  // complex128: the general pass of each entry of `pass`
    std::vector<ManySeg> seg;
    std::vector<uint16_t> slot_out;
    uint32_t total = 0;
    int nstates = 0;
    size_t partial_doubles = 0;
    size_t state_bytes = 0;
    double bytes = 0;  // algorithmic HBM bytes of the launch
    // workspace offsets
    size_t ctl = 0, desc = 0, partial = 0, states = 0;
    size_t inst_off = 0, pass_off = 0, gpass_off = 0, seg_off = 0, slot_off = 0, desc_bytes = 0;
};

struct ManyLayout {
    std::vector<ManyGroup> groups;
    std::vector<size_t> param_off, out_off;  // doubles, per problem
    size_t params = 0, out = 0, total = 0;
};

// ---- graph-captured optimisation steps ------------------------------------------------------
}  // namespace

struct qq_graph {
    qq_problem *pb = nullptr;
    int p = 0, B = 0, flags = 0, device = 0;
    Plan plan;
    Layout L;
    double lr = 0.01, beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
    double *x = nullptr;  // caller's device parameters [B][2p]
    void *mem = nullptr;  // workspace, moments, outputs, counter (one allocation)
    char *ws = nullptr;
    double *m = nullptr, *v = nullptr, *energy = nullptr, *grad = nullptr, *hist = nullptr;
    int *step = nullptr;
    int hist_len = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~qq_graph()
    {
        (void)hipSetDevice(device);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (mem) (void)hipFree(mem);
    }
};

namespace {

// One optimisation step on `stream`: the evaluation's pass and finalize kernels, then Adam.
qq_status enqueue_step(qq_graph *g, hipStream_t stream, bool capturing)
{
    if (qq_status st = run_plan(g->pb, g->plan, g->L, g->p, g->B, g->flags, g->ws, g->x, stream, capturing);
        st != QQ_OK)
        return st;
    AdamArgs a;
    a.B = g->B;
    a.p = g->p;
    a.lr = g->lr;
    a.beta1 = g->beta1;
    a.beta2 = g->beta2;
    a.eps = g->eps;
    a.result = reinterpret_cast<const double *>(g->ws + g->L.out);
    a.x = g->x;
    a.m = g->m;
    a.v = g->v;
    a.step = g->step;
    a.energy_out = g->energy;
    a.grad_out = g->grad;
    a.history = g->hist;
    a.history_len = g->hist_len;
    QQ_HIP(launch_adam(a, stream));
    return QQ_OK;
}

qq_status zero_state(qq_graph *g, hipStream_t stream)
{
    const size_t np = (size_t)g->B * 2 * g->p;
    QQ_HIP(launch_fill_f64(g->m, 0.0, np, stream));
    QQ_HIP(launch_fill_f64(g->v, 0.0, np, stream));
    QQ_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(g->step), 0u, 1, stream));
    return QQ_OK;
}

constexpr double kDefaultWaitMs = 2000.0;

// ---- autotuning -----------------------------------------------------------------------------
// Candidates are timed with HIP events (one warm-up, then the median of three
// runs) on seeded parameter sets; the best is pinned in the problem handle and,
// given a cache path, appended to a JSON-lines file that later calls read
// before timing anything.
std::string device_tag(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string t = std::string(prop.name) + "|" + prop.gcnArchName;
    for (char &c : t)
        if (c == '"' || c == '\\' || c == '\n') c = '_';
    return t;
}

// Seeded parameters in [0, pi) (a 64-bit LCG; the values only need to be typical).
std::vector<double> tune_params(size_t count, uint64_t seed)
{
    std::vector<double> x(count);
    uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
    for (double &v : x) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        v = (double)(st >> 11) * (3.141592653589793 / 9007199254740992.0);
    }
    return x;
}

// The value of "key": in a cache line (numbers only), or false.
bool json_num(const std::string &line, const char *key, double &out)
{
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    return std::sscanf(line.c_str() + at + k.size(), "%lf", &out) == 1;
}

bool cache_lookup(const char *path, const std::string &key, std::string &line_out)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char buf[1024];
    bool found = false;
    while (std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        if (line.compare(0, key.size(), key) == 0) {
            line_out = line;  // the last matching entry wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

qq_status cache_append(const char *path, const std::string &line)
{
    if (!path) return QQ_OK;
    FILE *f = std::fopen(path, "a");
    if (!f) return fail(QQ_E_INVALID, "cannot open the tuning cache %s for appending", path);
    std::fputs(line.c_str(), f);
    std::fputc('\n', f);
    std::fclose(f);
    return QQ_OK;
}

// Median of three timed runs of `run` after a timed warm-up, in ms; a single run when the
// warm-up took over 200 ms (timing noise is then small against the run, and the tuning
// of a large evaluation stays within a minute or two).
template <typename F>
qq_status time_median(hipStream_t stream, F run, double &ms)
{
    hipEvent_t a, b;
    QQ_HIP(hipEventCreate(&a));
    QQ_HIP(hipEventCreate(&b));
    float warm = 0.0f;
    qq_status st = QQ_OK;
    if (hipEventRecord(a, stream) != hipSuccess) st = fail(QQ_E_DEVICE, "hipEventRecord failed");
    if (st == QQ_OK) st = run();
    if (st == QQ_OK && (hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&warm, a, b) != hipSuccess))
        st = fail(QQ_E_DEVICE, "event timing failed");
    const int reps = warm > 200.0f ? 1 : 3;
    double t[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < reps && st == QQ_OK; ++r) {
        float f = 0.0f;
        if (hipEventRecord(a, stream) != hipSuccess) st = fail(QQ_E_DEVICE, "hipEventRecord failed");
        if (st == QQ_OK) st = run();
        if (st == QQ_OK && (hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                            hipEventElapsedTime(&f, a, b) != hipSuccess))
            st = fail(QQ_E_DEVICE, "event timing failed");
        t[r] = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != QQ_OK) return st;
    std::sort(t, t + reps);
    ms = t[reps / 2];
    return QQ_OK;
}

void pin_sched(qq_problem *pb, int p, int batch, int flags, int G, int pairing, int blocked, int set_order,
               double ms)
{
    const int sf = sched_flags(flags);
    for (auto &e : pb->sched)
        if (e.p == p && e.batch == batch && e.flags == sf) {
            e.G = G;
            e.pairing = pairing;
            e.blocked = blocked;
            e.set_order = set_order;
            e.ms = ms;
            return;
        }
    pb->sched.push_back({p, batch, sf, G, pairing, blocked, set_order, ms});
}

uint64_t fnv1a(uint64_t h, int64_t v)
{
    for (int i = 0; i < 8; ++i) {
        h ^= (uint64_t)((v >> (8 * i)) & 0xff);
        h *= 1099511628211ull;
    }
    return h;
}

int many_tiles_per_chunk(uint64_t tiles, const qq_many_options *opt, bool c128)
{
    // 24 tiles (768 KiB of one complex64 state) per item: each item ends with an XCD-wide
    // cache write-back and two device-scope atomics, which such an item amortises, while a
    // 2^22-amplitude pass still splits into 43 items (measured on MI355X with the 512-problem
    // uneven batch: 1 tile 107 ms, 8 tiles 30 ms in an earlier version; now 16 tiles 22.0 ms,
    // 24 20.9, 32 21.1, 48 22.0, 64 23.6).
    // Complex128 (one resident workgroup per compute unit): 8 tiles, so that the longest pass
    // chains split finely (the batch's 88 flagged sets: 2 tiles 13.5 ms, 4 11.4, 8 10.6, 16 11.8,
    // 64 25.5)
    const uint64_t want = (opt && opt->tiles_per_chunk > 0) ? (uint64_t)opt->tiles_per_chunk : (c128 ? 8 : 24);
    return (int)std::min<uint64_t>(want, tiles);
}

qq_status plan_many(int count, qq_problem *const *pbs, const int *p, const int *batch, int flags,
                    const qq_many_options *opt, ManyLayout &M)
{
    const bool grad = flags & QQ_GRAD;
    const bool c128 = flags & QQ_C128;
    const int mode = plan_mode(flags | QQ_ENERGY, false);
    // problem order (the tie-break of the ticket order below): longest pass chain first, then most tiles
    std::vector<int> order(count);
    std::vector<Plan> plans(count);
    for (int i = 0; i < count; ++i) {
        order[i] = i;
        plans[i] = make_plan(pbs[i]->n, p[i], mode);
        if (plans[i].nslots > kMaxSlots)
            return fail(QQ_E_UNSUPPORTED, "problem %d: plan needs %d accumulator slots (max %d)", i, plans[i].nslots,
                        kMaxSlots);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const size_t pa = plans[a].passes.size(), pb = plans[b].passes.size();
        if (pa != pb) return pa > pb;
        return pbs[a]->n > pbs[b]->n;
    });
    const int types[3] = {DIAG_F64, DIAG_I32, DIAG_I16};
    M.param_off.assign(count, 0);
    M.out_off.assign(count, 0);
    size_t poff = 0, ooff = 0;
    for (int i = 0; i < count; ++i) {
        M.param_off[i] = poff;
        poff += (size_t)batch[i] * 2 * p[i];
        M.out_off[i] = ooff;
        ooff += (size_t)batch[i] * (1 + 2 * p[i]);
    }
    size_t off = 0;
    M.params = off;
    off += align_up(poff * sizeof(double));
    M.out = off;
    off += align_up(ooff * sizeof(double));
    for (int dt : types) {
        ManyGroup G;
        G.diag_type = dt;
        for (int i : order)
            if (pbs[i]->diag_type == dt) G.members.push_back(i);
        if (G.members.empty()) continue;
        size_t state_off = 0;
        for (int i : G.members) {
            const qq_problem *pb = pbs[i];
            const Plan &plan = plans[i];
            ManyInst I;
            std::memset(&I, 0, sizeof I);
            I.n = pb->n;
            I.p = p[i];
            I.B = batch[i];
            I.tiles = tiles_per_state(pb->n);
            I.dim_mask = pb->dim - 1;
            I.amp0 = 1.0 / std::sqrt((double)pb->dim);
            I.escale = pb->n < kTileBits ? std::ldexp(1.0, pb->n - kTileBits) : 1.0;
            I.state0 = G.nstates;
            G.nstates += I.B;
            I.pass_off = (int)G.pass.size();
            I.slot_off = (int)G.slot_out.size();
            I.partial_off = G.partial_doubles;
            if (c128) {
                // complex128: the general pass bodies, chunks of tiles for every problem (one pass of
                // one tile for n <= 12); the passes accumulate with C itself (shift 0)
                I.tpc = many_tiles_per_chunk(I.tiles, opt, c128);
                I.nchunks = (int)((I.tiles + (uint64_t)I.tpc - 1) / (uint64_t)I.tpc);
                I.npasses = (int)plan.passes.size();
                int slot_base = 0;
                for (const PassPlan &pp : plan.passes) {
                    const SetDesc &sd = plan.sets[pp.set];
                    if ((int)pp.ops.size() > kMaxOps)
                        return fail(QQ_E_UNSUPPORTED, "pass has %zu ops (max %d)", pp.ops.size(), kMaxOps);
                    ManyPass P;
                    std::memset(&P, 0, sizeof P);
                    P.kind = -1;
                    P.geom = pp.nstates;
                    P.slot_base = slot_base;
                    P.nslots = (int)pp.slot_out.size();
                    PassArgs a;
                    std::memset(&a, 0, sizeof a);
                    a.n = pb->n;
                    a.p = I.p;
                    a.B = I.B;
                    a.G = 1;
                    a.tiles = I.tiles;
                    a.dim_mask = I.dim_mask;
                    a.pos4 = sd.pos4;
                    a.pos8 = sd.pos8;
                    a.high = sd.high;
                    a.w1 = sd.pos4 - 4;
                    a.w2 = sd.pos8 - sd.pos4 - 4;
                    a.flags = pp.flags;
                    a.nops = (int)pp.ops.size();
                    a.nslots = P.nslots;
                    a.amp0 = I.amp0;
                    a.state_stride = pb->dim;  // params, diag, psi, lam: device addresses, set at launch
                    for (size_t o = 0; o < pp.ops.size(); ++o) a.ops[o] = pp.ops[o];
                    slot_base += P.nslots;
                    for (int o : pp.slot_out) G.slot_out.push_back((uint16_t)o);
                    G.pass.push_back(P);
                    G.gpass.push_back(a);
                    G.bytes += pass_bytes(pb, pp, I.B, true, false);
                }
                I.nslots = slot_base;
                const size_t sb = (size_t)pb->dim * 16 * I.B;
                I.psi = reinterpret_cast<void *>(state_off);  // relative; fixed up at launch
                state_off += align_up(sb);
                if (grad) {
                    I.lam = reinterpret_cast<void *>(state_off);
                    state_off += align_up(sb);
                }
            } else if (plan.sets.size() == 1) {
                // the whole evaluation in one item per parameter set; slot o is output o
                ManyPass P;
                std::memset(&P, 0, sizeof P);
                P.kind = FK_SINGLE;
                P.active = plan.sets[0].active;
                P.nact = __builtin_popcount(P.active);
                P.nslots = grad ? 1 + 2 * I.p : 1;
                G.pass.push_back(P);
                I.npasses = 1;
                I.nchunks = 1;
                I.tpc = 1;
                I.nslots = P.nslots;
                for (int o = 0; o < I.nslots; ++o) G.slot_out.push_back((uint16_t)o);
                G.bytes += (double)pb->dim * diag_bytes_of(pb->diag_type);
            } else {
                I.shift = pb->alpha;  // the pass bodies accumulate with C - alpha
                I.tpc = many_tiles_per_chunk(I.tiles, opt, c128);
                I.nchunks = (int)((I.tiles + (uint64_t)I.tpc - 1) / (uint64_t)I.tpc);
                I.npasses = (int)plan.passes.size();
                int slot_base = 0;
                for (const PassPlan &pp : plan.passes) {
                    const SetDesc &sd = plan.sets[pp.set];
                    ManyPass P;
                    std::memset(&P, 0, sizeof P);
                    P.kind = pp.fkind;
                    P.k = pp.fk;
                    P.geom = !sd.high ? 0 : (sd.active == 0x0ff0 ? 1 : 2);
                    P.pos4 = sd.pos4;
                    P.pos8 = sd.pos8;
                    P.w1 = sd.pos4 - 4;
                    P.w2 = sd.pos8 - sd.pos4 - 4;
                    P.active = sd.active;
                    P.nact = __builtin_popcount(sd.active);
                    P.store_psi = (pp.flags & PF_STORE_PSI) ? 1 : 0;
                    P.slot_base = slot_base;
                    P.nslots = (int)pp.slot_out.size();
                    P.ctab = find_cost_table(pb, sd, pp.fkind == FK_FIRST ? sd.pos4 : sd.pos8);
                    if (!P.ctab) return fail(QQ_E_DEVICE, "no cost table for the set at qubits %d / %d", sd.pos4, sd.pos8);
                    P.cthr = P.ctab + (size_t)I.tiles * kCostRow;
                    slot_base += P.nslots;
                    for (int o : pp.slot_out) G.slot_out.push_back((uint16_t)o);
                    G.pass.push_back(P);
                    G.bytes += pass_bytes(pb, pp, I.B, false, true);
                }
                I.nslots = slot_base;
                const size_t sb = (size_t)pb->dim * sizeof(float2) * I.B;
                I.psi = reinterpret_cast<void *>(state_off);  // relative; fixed up below
                state_off += align_up(sb);
                if (grad) {
                    I.lam = reinterpret_cast<void *>(state_off);
                    state_off += align_up(sb);
                }
            }
            G.partial_doubles += (size_t)I.nslots * I.B * I.nchunks;
            G.inst.push_back(I);
        }
        G.state_bytes = state_off;
        // segments in the order of the fraction (j + 1) / L of its problem's chain of L passes that
        // pass j completes (ties: longer chains, then the problem order above): every chain advances
        // in step with the whole queue, so the long chains do not trail alone at the end, and the
        // single-item problems (L = 1) come last, where they fill the workgroups the chains leave
        // idle.  Measured on the 512-problem uneven batch at 32 tiles per item: 21.0 ms against
        // 22.0 ms level-major (every problem's pass 0, then pass 1, ...).  Pass j of a state always
        // precedes its pass j + 1, which is all the queue needs.
        struct SegKey {
            int num, den, k, b;  // key num / den = (j + 1) / L
        };
        std::vector<SegKey> keys;
        for (size_t k = 0; k < G.inst.size(); ++k)
            for (int j = 0; j < G.inst[k].npasses; ++j)
                for (int b = 0; b < G.inst[k].B; ++b) keys.push_back({j + 1, G.inst[k].npasses, (int)k, b});
        std::sort(keys.begin(), keys.end(), [](const SegKey &x, const SegKey &y) {
            const int64_t lx = (int64_t)x.num * y.den, ly = (int64_t)y.num * x.den;
            if (lx != ly) return lx < ly;
            if (x.den != y.den) return x.den > y.den;
            if (x.k != y.k) return x.k < y.k;
            if (x.num != y.num) return x.num < y.num;
            return x.b < y.b;
        });
        uint64_t ticket = 0;
        for (const SegKey &x : keys) {
            G.seg.push_back({(uint32_t)ticket, (uint32_t)x.k, (uint32_t)x.b, (uint32_t)(x.num - 1)});
            ticket += (uint64_t)G.inst[x.k].nchunks;
        }
        if (ticket >= 0xffffffffull) return fail(QQ_E_TOO_LARGE, "%llu work items exceed 2^32", (unsigned long long)ticket);
        G.total = (uint32_t)ticket;
        // workspace regions of the group
        G.ctl = off;
        off += align_up((size_t)(2 + G.nstates) * sizeof(uint32_t));
        G.inst_off = 0;
        G.pass_off = align_up(G.inst.size() * sizeof(ManyInst), 16);
        G.gpass_off = G.pass_off + align_up(G.pass.size() * sizeof(ManyPass), 16);
        G.seg_off = G.gpass_off + align_up(G.gpass.size() * sizeof(PassArgs), 16);
        G.slot_off = G.seg_off + align_up(G.seg.size() * sizeof(ManySeg), 16);
        G.desc_bytes = G.slot_off + G.slot_out.size() * sizeof(uint16_t);
        G.desc = off;
        off += align_up(G.desc_bytes);
        G.partial = off;
        off += align_up(std::max<size_t>(1, G.partial_doubles) * sizeof(double));
        G.states = off;
        off += align_up(G.state_bytes);
        M.groups.push_back(std::move(G));
    }
    M.total = off;
    return QQ_OK;
}

qq_status validate_many(int count, qq_problem *const *pbs, const int *p, const int *batch, int flags)
{
    if (count < 1) return fail(QQ_E_INVALID, "count = %d must be >= 1", count);
    if (!pbs || !p || !batch) return fail(QQ_E_INVALID, "problems / p / batch is NULL");
    const int known = QQ_ENERGY | QQ_GRAD | QQ_C128 | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE;
    if (flags & QQ_PARTITIONED)
        return fail(QQ_E_UNSUPPORTED, "qq_evaluate_many runs monolithic evaluations only "
                                      "(use qq_evaluate for QQ_PARTITIONED)");
    if (flags & ~known) return fail(QQ_E_INVALID, "unknown flag bits 0x%x", flags & ~known);
    for (int i = 0; i < count; ++i) {
        if (!pbs[i]) return fail(QQ_E_INVALID, "problems[%d] is NULL", i);
        if (pbs[i]->device != pbs[0]->device)
            return fail(QQ_E_INVALID, "problems[%d] is on device %d, problems[0] on %d", i, pbs[i]->device,
                        pbs[0]->device);
        if (pbs[i]->n > kManyMaxN)
            return fail(QQ_E_UNSUPPORTED, "problems[%d]: n = %d above %d (use qq_evaluate)", i, pbs[i]->n, kManyMaxN);
        if (p[i] < 1 || p[i] > QQ_MAX_P) return fail(QQ_E_INVALID, "p[%d] = %d outside [1, %d]", i, p[i], QQ_MAX_P);
        if (batch[i] < 1) return fail(QQ_E_INVALID, "batch[%d] = %d must be >= 1", i, batch[i]);
    }
    return QQ_OK;
}

}  // namespace

namespace qq {
qq_status set_error(qq_status st, const char *msg)
{
    g_err = msg;
    return st;
}
int problem_device(const qq_problem *pb) { return pb->device; }
}  // namespace qq

namespace {

// Bound on ||dg||_inf of a complex64 gradient (see qq_evaluate_guarded in the header): a part relative
// to the gradient, and the random part of the rounding of 2^n stored amplitudes in sums whose terms
// carry (C - alpha)^2, which grows as 2^(-n/2) of sigma_C^2 per unit rounding.
double c64_grad_bound(int n, double sigma_c, double gmax)
{
    return QQ_GUARD_REL * gmax + QQ_GUARD_K * std::ldexp(sigma_c * sigma_c, -24) * std::pow(2.0, -0.5 * n);
}

constexpr double kC128GradRel = 1e-10;

double max_abs(const double *g, int m)
{
    double r = 0.0;
    for (int j = 0; j < m; ++j) r = std::max(r, std::fabs(g[j]));
    return r;
}

// The flagged parameter sets of one problem, to be recomputed with complex128 states.
struct C128Job {
    qq_problem *pb;
    int p;
    const double *params;  // host [batch][2p]
    std::vector<int> sets;
    double *energy, *grad;  // host outputs, indexed by set
};

// Streams owned for the length of one call (default priority), destroyed on every return path.
struct SideStreams {
    std::vector<hipStream_t> s;
    ~SideStreams()
    {
        for (hipStream_t x : s) (void)hipStreamDestroy(x);
    }
};

// Recompute every job's sets with complex128 states (host in, host out; all problems on one device).
// Several problems with monolithic phases: one persistent complex128 launch (qq_evaluate_many) over
// all of them (the uneven batch's 88 flagged sets: 10.6 ms against about 20 ms of per-problem
// launches).  One problem, or partitioned phases: per-problem evaluations with the per-pass kernels,
// which are faster for a single problem (n = 26, p = 4, 8 sets: 175 ms against 200-219 ms through
// the persistent launch; n = 20, one set: 0.3 against 1.1 ms).  Their parameters go to the device in
// one copy; the jobs run round-robin on up to kC128Streams streams of their own, each with its own
// workspace (the largest any job needs), so that the small per-problem launches of different
// problems overlap; one device output buffer is read back after all of them.
constexpr int kC128Streams = 4;

qq_status recompute_c128(std::vector<C128Job> &jobs, int flags, void *stream_)
{
    const int f = (flags & (QQ_ENERGY | QQ_GRAD | QQ_PARTITIONED)) | QQ_C128;
    const bool grad = flags & QQ_GRAD;
    int with_sets = 0;
    for (const C128Job &j : jobs) with_sets += j.sets.empty() ? 0 : 1;
    if (!(f & QQ_PARTITIONED) && with_sets > 1) {
        // every recomputed set in one persistent complex128 launch (per cost-diagonal element type)
        std::vector<qq_problem *> pbs;
        std::vector<int> ps, bs;
        std::vector<std::vector<double>> xs, es, gs;
        std::vector<C128Job *> owner;
        for (C128Job &j : jobs) {
            if (j.sets.empty()) continue;
            const int m = (int)j.sets.size(), w = 2 * j.p;
            pbs.push_back(j.pb);
            ps.push_back(j.p);
            bs.push_back(m);
            std::vector<double> x((size_t)m * w);
            for (int i = 0; i < m; ++i)
                std::memcpy(&x[(size_t)i * w], j.params + (size_t)j.sets[i] * w, w * sizeof(double));
            xs.push_back(std::move(x));
            es.emplace_back(m);
            gs.emplace_back(grad ? (size_t)m * w : 0);
            owner.push_back(&j);
        }
        if (pbs.empty()) return QQ_OK;
        const int count = (int)pbs.size();
        std::vector<const double *> xp(count);
        std::vector<double *> ep(count), gp(count);
        for (int q = 0; q < count; ++q) {
            xp[q] = xs[q].data();
            ep[q] = es[q].data();
            gp[q] = grad ? gs[q].data() : nullptr;
        }
        if (qq_status st = qq_evaluate_many(count, pbs.data(), ps.data(), bs.data(), xp.data(), f, nullptr, nullptr, 0,
                                            stream_, ep.data(), grad ? gp.data() : nullptr);
            st != QQ_OK)
            return st;
        for (int q = 0; q < count; ++q) {
            C128Job &j = *owner[q];
            const int w = 2 * j.p;
            for (size_t i = 0; i < j.sets.size(); ++i) {
                j.energy[j.sets[i]] = es[q][i];
                if (grad) std::memcpy(j.grad + (size_t)j.sets[i] * w, &gs[q][i * w], w * sizeof(double));
            }
        }
        return QQ_OK;
    }
    // one problem, or partitioned phases: per-problem evaluations spread over side streams
    size_t wsmax = 0, nx = 0, nout = 0;
    int nj = 0;
    for (const C128Job &j : jobs) {
        if (j.sets.empty()) continue;
        const int m = (int)j.sets.size();
        size_t w = 0;
        if (qq_status st = qq_workspace_size(j.pb, j.p, m, f, &w); st != QQ_OK) return st;
        wsmax = std::max(wsmax, w);
        nx += (size_t)m * 2 * j.p;
        nout += (size_t)m * (1 + (grad ? 2 * j.p : 0));
        ++nj;
    }
    if (nj == 0) return QQ_OK;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const int device = jobs[0].pb->device;
    QQ_HIP(hipSetDevice(device));
    const int ns = std::min(kC128Streams, nj);
    const size_t wsa = align_up(wsmax);
    const size_t need = (size_t)ns * wsa + (nx + nout) * sizeof(double);
    if (qq_status st = check_device_fits(device, need, "the complex128 recomputation"); st != QQ_OK) return st;
    DevBuf ws, buf;
    if (hipMalloc(&ws.p, (size_t)ns * wsa) != hipSuccess || hipMalloc(&buf.p, (nx + nout) * sizeof(double)) != hipSuccess)
        return fail(QQ_E_NOMEM, "hipMalloc of %zu bytes for the complex128 recomputation failed", need);
    double *d_x = static_cast<double *>(buf.p), *d_out = d_x + nx;
    std::vector<double> x(nx), h(nout);
    size_t xo = 0;
    for (const C128Job &j : jobs) {
        if (j.sets.empty()) continue;
        const int m = (int)j.sets.size(), w = 2 * j.p;
        for (int i = 0; i < m; ++i)
            std::memcpy(&x[xo + (size_t)i * w], j.params + (size_t)j.sets[i] * w, w * sizeof(double));
        xo += (size_t)m * w;
    }
    QQ_HIP(hipMemcpyAsync(d_x, x.data(), nx * sizeof(double), hipMemcpyHostToDevice, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    SideStreams side;
    for (int k = 0; k < ns; ++k) {
        hipStream_t sk = nullptr;
        QQ_HIP(hipStreamCreateWithFlags(&sk, hipStreamNonBlocking));
        side.s.push_back(sk);
    }
    xo = 0;
    size_t oo = 0;
    int q = 0;
    for (const C128Job &j : jobs) {
        if (j.sets.empty()) continue;
        const int m = (int)j.sets.size(), w = 2 * j.p;
        char *wq = static_cast<char *>(ws.p) + (size_t)(q % ns) * wsa;
        if (qq_status st = qq_evaluate(j.pb, j.p, m, d_x + xo, f | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE, wq, wsmax,
                                       side.s[q % ns], d_out + oo, grad ? d_out + oo + m : nullptr);
            st != QQ_OK) {
            for (hipStream_t sk : side.s) (void)hipStreamSynchronize(sk);
            return st;
        }
        xo += (size_t)m * w;
        oo += (size_t)m * (1 + (grad ? w : 0));
        ++q;
    }
    for (hipStream_t sk : side.s) QQ_HIP(hipStreamSynchronize(sk));
    QQ_HIP(hipMemcpyAsync(h.data(), d_out, nout * sizeof(double), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    oo = 0;
    for (C128Job &j : jobs) {
        if (j.sets.empty()) continue;
        const int m = (int)j.sets.size(), w = 2 * j.p;
        for (int i = 0; i < m; ++i) {
            j.energy[j.sets[i]] = h[oo + i];
            if (grad) std::memcpy(j.grad + (size_t)j.sets[i] * w, &h[oo + m + (size_t)i * w], w * sizeof(double));
        }
        oo += (size_t)m * (1 + (grad ? w : 0));
    }
    return QQ_OK;
}

// Decide, for the complex64 results of one problem, which sets to recompute; fill the outputs.
std::vector<int> guard_sets(const qq_problem *pb, int p, int batch, const double *grad, double tol, bool c128_all,
                            int32_t *c128_out, double *err_out)
{
    std::vector<int> sets;
    for (int b = 0; b < batch; ++b) {
        const double gmax = grad ? max_abs(grad + (size_t)b * 2 * p, 2 * p) : 0.0;
        bool up = c128_all;
        double err = 0.0;
        if (grad && !c128_all) {
            err = c64_grad_bound(pb->n, pb->sigma_c, gmax);
            up = err > tol * gmax;
        }
        if (up && grad && !c128_all) sets.push_back(b);
        if (c128_out) c128_out[b] = up ? 1 : 0;
        if (err_out) err_out[b] = grad ? (up ? kC128GradRel * gmax : err) : 0.0;
    }
    return sets;
}

}  // namespace

extern "C" {

const char *qq_last_error(void) { return g_err.c_str(); }

int qq_abi_version(void) { return 1; }

qq_status qq_device_count(int *count)
{
    if (!count) return fail(QQ_E_INVALID, "count is NULL");
    int c = 0;
    hipError_t e = hipGetDeviceCount(&c);
    if (e != hipSuccess) c = 0;
    *count = c;
    return QQ_OK;
}

qq_status qq_problem_create(int n, const double *H, const double *f, double c0, int device, void *stream_,
                            qq_problem **out)
{
    g_err.clear();
    if (!out) return fail(QQ_E_INVALID, "out is NULL");
    if (n < 1 || n > QQ_MAX_N) return fail(QQ_E_INVALID, "n = %d outside [1, %d]", n, QQ_MAX_N);
    if (!H) return fail(QQ_E_INVALID, "H is NULL");
    if (!std::isfinite(c0)) return fail(QQ_E_INVALID, "c0 is not finite");
    for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(H[i])) return fail(QQ_E_INVALID, "H[%d][%d] is not finite", i / n, i % n);
    if (f)
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(f[i])) return fail(QQ_E_INVALID, "f[%d] is not finite", i);
    if (device < 0) return fail(QQ_E_INVALID, "device = %d", device);

    qq_problem *pb = new (std::nothrow) qq_problem();
    if (!pb) return fail(QQ_E_NOMEM, "host allocation failed");
    std::unique_ptr<qq_problem> guard(pb);
    pb->n = n;
    pb->device = device;
    pb->H.assign(H, H + (size_t)n * n);
    pb->f.assign(n, 0.0);
    if (f) pb->f.assign(f, f + n);
    pb->c0 = c0;

    // eq. (4)-(5)
    pb->ell.assign(n, 0.0);
    pb->b.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) pb->ell[i] = pb->f[i] + pb->H[(size_t)i * n + i];
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) pb->b[(size_t)i * n + j] = pb->H[(size_t)i * n + j] + pb->H[(size_t)j * n + i];

    // integer classification: integral inputs whose canonical magnitudes sum below 2^31
    bool integral = std::nearbyint(c0) == c0;
    for (double v : pb->H) integral = integral && std::nearbyint(v) == v;
    for (double v : pb->f) integral = integral && std::nearbyint(v) == v;
    double mag = std::fabs(c0);
    for (double v : pb->ell) mag += std::fabs(v);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) mag += std::fabs(pb->b[(size_t)i * n + j]);
    pb->is_integer = integral && mag < kTwo31;
    pb->diag_type = !pb->is_integer ? DIAG_F64 : (mag < kTwo15 ? DIAG_I16 : DIAG_I32);
    pb->c0_i = pb->is_integer ? (int32_t)c0 : 0;
    pb->ell_i.assign(n, 0);
    if (pb->is_integer)
        for (int i = 0; i < n; ++i) pb->ell_i[i] = (int32_t)pb->ell[i];
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double v = pb->b[(size_t)i * n + j];
            if (v == 0.0) continue;
            pb->pair_ij.push_back(i);
            pb->pair_ij.push_back(j);
            pb->pair_b.push_back(v);
            pb->pair_bi.push_back(pb->is_integer ? (int32_t)v : 0);
        }

    // Pauli coefficients of eq. (9) and the spread of C
    {
        double alpha = c0, s2 = 0.0;
        std::vector<double> h(n, 0.0);
        for (int i = 0; i < n; ++i) {
            alpha += pb->ell[i] / 2.0;
            h[i] -= pb->ell[i] / 2.0;
        }
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                const double v = pb->b[(size_t)i * n + j];
                alpha += v / 4.0;
                h[i] -= v / 4.0;
                h[j] -= v / 4.0;
                s2 += (v / 4.0) * (v / 4.0);
            }
        for (double x : h) s2 += x * x;
        pb->alpha = alpha;
        pb->sigma_c = std::sqrt(s2);
    }

    pb->dim = 1ull << n;
    const size_t dbytes = (size_t)pb->dim * diag_bytes_of(pb->diag_type);
    if (qq_status st = check_device_fits(device, dbytes + cost_table_bytes(n), "the cost diagonal and its tables");
        st != QQ_OK)
        return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(device));
    const int np = (int)pb->pair_b.size();
    if (hipMalloc(&pb->d_diag, dbytes) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for the diagonal failed", dbytes);
    QQ_HIP(hipMalloc((void **)&pb->d_ell, sizeof(double) * n));
    QQ_HIP(hipMalloc((void **)&pb->d_ell_i, sizeof(int32_t) * n));
    QQ_HIP(hipMalloc((void **)&pb->d_pair_ij, sizeof(int32_t) * std::max(2, 2 * np)));
    QQ_HIP(hipMalloc((void **)&pb->d_pair_b, sizeof(double) * std::max(1, np)));
    QQ_HIP(hipMalloc((void **)&pb->d_pair_bi, sizeof(int32_t) * std::max(1, np)));
    {
        std::vector<double> regq(16 * (size_t)std::max(1, n - 3), 0.0);
        for (int q = 0; q + 4 <= n; ++q)
            for (int r = 1; r < 16; ++r) {
                const int j = __builtin_ctz(r);
                double sum = 0.0;
                for (int k = j + 1; k < 4; ++k)
                    if ((r >> k) & 1) sum += pb->b[(size_t)(q + j) * n + (q + k)];
                regq[16 * (size_t)q + r] = sum;
            }
        QQ_HIP(hipMalloc((void **)&pb->d_regq, sizeof(double) * regq.size()));
        QQ_HIP(hipMemcpy(pb->d_regq, regq.data(), sizeof(double) * regq.size(), hipMemcpyHostToDevice));
    }
    QQ_HIP(hipMemcpyAsync(pb->d_ell, pb->ell.data(), sizeof(double) * n, hipMemcpyHostToDevice, stream));
    QQ_HIP(hipMemcpyAsync(pb->d_ell_i, pb->ell_i.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    if (np) {
        QQ_HIP(hipMemcpyAsync(pb->d_pair_ij, pb->pair_ij.data(), sizeof(int32_t) * 2 * np, hipMemcpyHostToDevice, stream));
        QQ_HIP(hipMemcpyAsync(pb->d_pair_b, pb->pair_b.data(), sizeof(double) * np, hipMemcpyHostToDevice, stream));
        QQ_HIP(hipMemcpyAsync(pb->d_pair_bi, pb->pair_bi.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, stream));
    }
    QQ_HIP(prof_aux(5, n, diag_bytes_of(pb->diag_type), (double)dbytes, stream, [&]() {
        return launch_cost_diag(n, pb->diag_type, pb->d_ell, pb->d_ell_i, np, pb->d_pair_ij, pb->d_pair_b,
                                pb->d_pair_bi, c0, pb->c0_i, pb->d_diag, pb->dim, stream);
    }));
    if (qq_status st = build_cost_tables(pb, stream); st != QQ_OK) return st;

    // min / argmin / max of C
    const int nblk = (int)std::min<uint64_t>(1024, (pb->dim + 255) / 256);
    DevBuf part;
    QQ_HIP(hipMalloc(&part.p, (size_t)nblk * (2 * sizeof(double) + sizeof(uint64_t))));
    double *d_part = static_cast<double *>(part.p);
    uint64_t *d_idx = reinterpret_cast<uint64_t *>(d_part + 2 * nblk);
    QQ_HIP(prof_aux(6, n, diag_bytes_of(pb->diag_type), (double)dbytes, stream, [&]() {
        return launch_minmax(pb->d_diag, pb->diag_type, pb->dim, d_part, d_idx, nblk, stream);
    }));
    std::vector<double> hp(2 * nblk);
    std::vector<uint64_t> hi(nblk);
    QQ_HIP(hipMemcpyAsync(hp.data(), d_part, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipMemcpyAsync(hi.data(), d_idx, sizeof(uint64_t) * nblk, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    double mn = INFINITY, mx = -INFINITY;
    uint64_t mi = ~0ull;
    for (int k = 0; k < nblk; ++k) {
        if (hp[2 * k] < mn || (hp[2 * k] == mn && hi[k] < mi)) {
            mn = hp[2 * k];
            mi = hi[k];
        }
        mx = std::max(mx, hp[2 * k + 1]);
    }
    pb->cmin = mn;
    pb->cmax = mx;
    pb->argmin = mi;
    *out = guard.release();
    return QQ_OK;
}

qq_status qq_problem_destroy(qq_problem *prob)
{
    g_err.clear();
    if (prob && prob->graphs > 0)
        return fail(QQ_E_INVALID, "%d captured graph(s) still use this problem; destroy them first", prob->graphs);
    delete prob;
    return QQ_OK;
}

qq_status qq_problem_info(const qq_problem *pb, qq_info *out)
{
    if (!pb || !out) return fail(QQ_E_INVALID, "NULL argument");
    qq_info in;
    std::memset(&in, 0, sizeof in);
    in.n = pb->n;
    in.is_integer = pb->is_integer;
    in.diag_bytes = diag_bytes_of(pb->diag_type);
    in.num_qpus = pb->num_qpus;
    in.c0 = pb->c0;
    in.alpha = pb->alpha;
    in.sigma_c = pb->sigma_c;
    in.cmin = pb->cmin;
    in.cmax = pb->cmax;
    in.argmin_index = pb->argmin;
    in.nonzero_couplings = (int64_t)pb->pair_b.size();
    in.cross_terms = pb->cross_terms;
    *out = in;
    return QQ_OK;
}

qq_status qq_coefficients(const qq_problem *pb, double *ell, double *b, double *alpha, double *h, double *J)
{
    if (!pb) return fail(QQ_E_INVALID, "problem is NULL");
    const int n = pb->n;
    if (ell) std::copy(pb->ell.begin(), pb->ell.end(), ell);
    if (b) std::copy(pb->b.begin(), pb->b.end(), b);
    if (alpha) *alpha = pb->alpha;
    if (h || J) {
        std::vector<double> hh(n, 0.0), JJ((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) hh[i] = -pb->ell[i] / 2.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                const double v = pb->b[(size_t)i * n + j];
                hh[i] -= v / 4.0;
                hh[j] -= v / 4.0;
                JJ[(size_t)i * n + j] = v / 4.0;
            }
        if (h) std::copy(hh.begin(), hh.end(), h);
        if (J) std::copy(JJ.begin(), JJ.end(), J);
    }
    return QQ_OK;
}

qq_status qq_cost_diagonal(const qq_problem *pb, void *out, int flags, void *stream_)
{
    if (!pb || !out) return fail(QQ_E_INVALID, "NULL argument");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    const size_t ob = (size_t)pb->dim * (pb->is_integer ? 4 : 8);
    if (flags & QQ_OUT_ON_DEVICE) {
        QQ_HIP(launch_widen_diag(pb->d_diag, pb->diag_type, pb->dim, out, stream));
        return QQ_OK;
    }
    DevBuf tmp;
    if (hipMalloc(&tmp.p, ob) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) failed", ob);
    QQ_HIP(launch_widen_diag(pb->d_diag, pb->diag_type, pb->dim, tmp.p, stream));
    QQ_HIP(hipMemcpyAsync(out, tmp.p, ob, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

qq_status qq_set_allocation(qq_problem *pb, int M, const int32_t *qpu_of_var, const int32_t *capacities,
                            int64_t *cross_out, int64_t *remote_out)
{
    if (!pb || !qpu_of_var) return fail(QQ_E_INVALID, "NULL argument");
    if (pb->graphs > 0)
        return fail(QQ_E_INVALID, "%d captured graph(s) use this problem's current allocation; destroy them first",
                    pb->graphs);
    const int n = pb->n;
    if (M < 1 || M > QQ_MAX_QPUS) return fail(QQ_E_INVALID, "num_qpus = %d outside [1, %d]", M, QQ_MAX_QPUS);
    std::vector<int> count(M, 0);
    for (int i = 0; i < n; ++i) {
        if (qpu_of_var[i] < 0 || qpu_of_var[i] >= M)
            return fail(QQ_E_ALLOCATION, "variable %d assigned to QPU %d outside [0, %d)", i + 1, qpu_of_var[i], M);
        ++count[qpu_of_var[i]];
    }
    for (int m = 0; m < M; ++m) {
        if (count[m] == 0) return fail(QQ_E_ALLOCATION, "QPU %d has no variable (every QPU must be used)", m);
        if (capacities && capacities[m] < 0) return fail(QQ_E_INVALID, "capacity of QPU %d is negative", m);
        if (capacities && count[m] > capacities[m])
            return fail(QQ_E_ALLOCATION, "QPU %d holds %d variables, capacity %d", m, count[m], capacities[m]);
    }
    int64_t cross = 0;
    std::vector<int32_t> xij;
    std::vector<double> xb;
    std::vector<int32_t> xbi;
    for (size_t k = 0; k < pb->pair_b.size(); ++k) {
        const int i = pb->pair_ij[2 * k], j = pb->pair_ij[2 * k + 1];
        if (qpu_of_var[i] != qpu_of_var[j]) {
            ++cross;
            xij.push_back(i);
            xij.push_back(j);
            xb.push_back(pb->pair_b[k]);
            xbi.push_back(pb->pair_bi[k]);
        }
    }
    PartDesc pd;
    std::memset(&pd, 0, sizeof pd);
    pd.nparts = M;
    uint64_t total = 0;
    for (int m = 0; m < M; ++m) {
        pd.table_off[m] = total;
        for (int i = 0; i < n; ++i)
            if (qpu_of_var[i] == m) {
                pd.vars[m][pd.nvars[m]++] = (uint8_t)i;
                pd.vmask[m] |= 1ull << i;
            }
        total += 1ull << pd.nvars[m];
    }
    const int es = diag_bytes_of(pb->diag_type);
    if (qq_status st = check_device_fits(pb->device, (size_t)pb->dim * es * 2 + 2 * cost_table_bytes(n),
                                         "the cross-QPU diagonal and its tables");
        st != QQ_OK)
        return st;
    QQ_HIP(hipSetDevice(pb->device));
    // release a previous allocation
    void *olds[] = {pb->d_qpu, pb->d_tables, pb->d_cross, pb->d_part, pb->d_part_cq, pb->d_xtab};
    for (void *q : olds)
        if (q) QQ_HIP(hipFree(q));
    pb->d_xtab = nullptr;
    pb->xtabs.clear();
    pb->d_part_cq = nullptr;
    pb->d_qpu = nullptr;
    pb->d_tables = pb->d_cross = nullptr;
    pb->d_part = nullptr;
    pb->num_qpus = 0;
    hipStream_t stream = nullptr;
    QQ_HIP(hipMalloc((void **)&pb->d_qpu, sizeof(int32_t) * n));
    QQ_HIP(hipMalloc(&pb->d_tables, total * es));
    if (hipMalloc(&pb->d_cross, (size_t)pb->dim * es) != hipSuccess)
        return fail(QQ_E_NOMEM, "hipMalloc for the cross diagonal failed");
    QQ_HIP(hipMalloc((void **)&pb->d_part, sizeof(PartDesc)));
    {
        // pair sums of every factor among each run of four consecutive qubits (see d_part_cq)
        const int runs = std::max(1, n - 3);
        std::vector<double> pcq((size_t)(M + 1) * runs * 16, 0.0);
        for (int f = 0; f <= M; ++f)
            for (int q = 0; q + 4 <= n; ++q)
                for (int r = 1; r < 16; ++r) {
                    const int j = __builtin_ctz(r), a = q + j;
                    double sum = 0.0;
                    for (int k = j + 1; k < 4; ++k) {
                        if (!((r >> k) & 1)) continue;
                        const int c = q + k;
                        const bool local = qpu_of_var[a] == qpu_of_var[c];
                        if ((f == M && !local) || (f < M && local && qpu_of_var[a] == f)) sum += pb->b[(size_t)a * n + c];
                    }
                    pcq[((size_t)f * runs + q) * 16 + r] = sum;
                }
        QQ_HIP(hipMalloc((void **)&pb->d_part_cq, sizeof(double) * pcq.size()));
        QQ_HIP(hipMemcpy(pb->d_part_cq, pcq.data(), sizeof(double) * pcq.size(), hipMemcpyHostToDevice));
    }
    QQ_HIP(hipMemcpy(pb->d_qpu, qpu_of_var, sizeof(int32_t) * n, hipMemcpyHostToDevice));
    QQ_HIP(hipMemcpy(pb->d_part, &pd, sizeof(PartDesc), hipMemcpyHostToDevice));
    QQ_HIP(launch_local_tables(n, pb->diag_type, pb->d_part, pb->d_ell, pb->d_ell_i, (int)pb->pair_b.size(),
                               pb->d_pair_ij, pb->d_pair_b, pb->d_pair_bi, pb->d_qpu, pb->c0, pb->c0_i, pb->d_tables,
                               total, stream));
    // cross diagonal: the cost diagonal of the cross couplings alone (no linear terms, no constant)
    {
        const int nx = (int)xb.size();
        DevBuf zero_ell, zero_elli, dij, db, dbi;
        QQ_HIP(hipMalloc(&zero_ell.p, sizeof(double) * n));
        QQ_HIP(hipMalloc(&zero_elli.p, sizeof(int32_t) * n));
        QQ_HIP(hipMemset(zero_ell.p, 0, sizeof(double) * n));
        QQ_HIP(hipMemset(zero_elli.p, 0, sizeof(int32_t) * n));
        QQ_HIP(hipMalloc(&dij.p, sizeof(int32_t) * std::max(2, 2 * nx)));
        QQ_HIP(hipMalloc(&db.p, sizeof(double) * std::max(1, nx)));
        QQ_HIP(hipMalloc(&dbi.p, sizeof(int32_t) * std::max(1, nx)));
        if (nx) {
            QQ_HIP(hipMemcpy(dij.p, xij.data(), sizeof(int32_t) * 2 * nx, hipMemcpyHostToDevice));
            QQ_HIP(hipMemcpy(db.p, xb.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
            QQ_HIP(hipMemcpy(dbi.p, xbi.data(), sizeof(int32_t) * nx, hipMemcpyHostToDevice));
        }
        QQ_HIP(launch_cost_diag(n, pb->diag_type, static_cast<double *>(zero_ell.p), static_cast<int32_t *>(zero_elli.p),
                                nx, static_cast<int32_t *>(dij.p), static_cast<double *>(db.p),
                                static_cast<int32_t *>(dbi.p), 0.0, 0, pb->d_cross, pb->dim, stream));
        // and its per-tile tables (the partitioned phases of the complex64 kernels read these)
        const std::vector<double> zeros(n, 0.0);
        auto BX = [&](int i, int j) {
            if (qpu_of_var[i] == qpu_of_var[j]) return 0.0;
            return i < j ? pb->b[(size_t)i * n + j] : pb->b[(size_t)j * n + i];
        };
        if (qq_status st = build_tables(n, zeros, BX, static_cast<double *>(zero_ell.p), nx,
                                        static_cast<int32_t *>(dij.p), static_cast<double *>(db.p), 0.0, pb->xtabs,
                                        &pb->d_xtab, stream);
            st != QQ_OK)
            return st;
        QQ_HIP(hipDeviceSynchronize());
    }
    pb->num_qpus = M;
    pb->qpu.assign(qpu_of_var, qpu_of_var + n);
    pb->cross_terms = cross;
    if (cross_out) *cross_out = cross;
    if (remote_out) *remote_out = 2 * cross;
    return QQ_OK;
}

qq_status qq_workspace_size(const qq_problem *pb, int p, int batch, int flags, size_t *bytes)
{
    if (!bytes) return fail(QQ_E_INVALID, "bytes is NULL");
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    const Plan plan = plan_for(pb, p, batch, flags, false);
    *bytes = layout_for(pb, p, batch, flags, plan).total;
    return QQ_OK;
}

static qq_status evaluate_impl(qq_problem *pb, int p, int batch, const double *params, int flags, void *workspace,
                      size_t ws_bytes, void *stream_, double *energy_out, double *grad_out)
{
    g_err.clear();
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    if (!params) return fail(QQ_E_INVALID, "params is NULL");
    if (!energy_out) return fail(QQ_E_INVALID, "energy_out is NULL");
    if ((flags & QQ_GRAD) && !grad_out) return fail(QQ_E_INVALID, "QQ_GRAD requires grad_out");
    if (!(flags & QQ_PARAMS_ON_DEVICE))
        if (qq_status st = check_params_host(params, (size_t)batch * 2 * p); st != QQ_OK) return st;
    const Plan plan = plan_for(pb, p, batch, flags, false);
    const Layout L = layout_for(pb, p, batch, flags, plan);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    DevBuf own;
    char *ws = static_cast<char *>(workspace);
    if (!ws) {
        if (qq_status st = check_device_fits(pb->device, L.total, "the workspace"); st != QQ_OK) return st;
        if (hipMalloc(&own.p, L.total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for the workspace failed", L.total);
        ws = static_cast<char *>(own.p);
    } else if (ws_bytes < L.total) {
        return fail(QQ_E_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
    }
    QQ_HIP(poison(ws, L.total, stream));
    if (qq_status st = eval_core(pb, p, batch, params, flags, plan, L, ws, stream); st != QQ_OK) return st;
    const double *d_out = reinterpret_cast<const double *>(ws + L.out);
    const size_t nout = 1 + 2 * (size_t)p;
    const bool grad = flags & QQ_GRAD;
    if (flags & QQ_OUT_ON_DEVICE) {
        QQ_HIP(hipMemcpy2DAsync(energy_out, sizeof(double), d_out, nout * sizeof(double), sizeof(double), batch,
                                hipMemcpyDeviceToDevice, stream));
        if (grad)
            QQ_HIP(hipMemcpy2DAsync(grad_out, 2 * p * sizeof(double), d_out + 1, nout * sizeof(double),
                                    2 * p * sizeof(double), batch, hipMemcpyDeviceToDevice, stream));
        if (own.p) QQ_HIP(hipStreamSynchronize(stream));
        return QQ_OK;
    }
    std::vector<double> h((size_t)batch * nout);
    QQ_HIP(hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    for (int b = 0; b < batch; ++b) {
        energy_out[b] = h[(size_t)b * nout];
        if (grad)
            for (int j = 0; j < 2 * p; ++j) grad_out[(size_t)b * 2 * p + j] = h[(size_t)b * nout + 1 + j];
    }
    return QQ_OK;
}

static qq_status evaluate_static_impl(qq_problem *pb, int p, int batch, const double *params, int flags, void *stream_,
                             double *energy_out, double *grad_out)
{
    g_err.clear();
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    if (!params) return fail(QQ_E_INVALID, "params is NULL");
    if (!energy_out) return fail(QQ_E_INVALID, "energy_out is NULL");
    if ((flags & QQ_GRAD) && !grad_out) return fail(QQ_E_INVALID, "QQ_GRAD requires grad_out");
    if (!(flags & QQ_PARAMS_ON_DEVICE))
        if (qq_status st = check_params_host(params, (size_t)batch * 2 * p); st != QQ_OK) return st;
    const Plan plan = plan_for(pb, p, batch, flags, false);
    const Layout L = layout_for(pb, p, batch, flags, plan);
    if (L.total > (size_t)QQ_STATIC_SCRATCH_BYTES)
        return fail(QQ_E_WORKSPACE, "this evaluation needs %zu bytes of workspace; the fixed scratch array holds %zu",
                    L.total, (size_t)QQ_STATIC_SCRATCH_BYTES);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    void *sp = nullptr;
    QQ_HIP(static_scratch(pb->device, &sp));
    char *ws = static_cast<char *>(sp);
    QQ_HIP(poison(ws, L.total, stream));
    const double *d_params = params;
    if (!(flags & QQ_PARAMS_ON_DEVICE)) {
        d_params = reinterpret_cast<const double *>(ws + L.params);
        QQ_HIP(hipMemcpyAsync(ws + L.params, params, (size_t)batch * 2 * p * sizeof(double), hipMemcpyHostToDevice,
                              stream));
    }
    // no profiling events here (capturing = true): they are not part of the computation
    if (qq_status st = run_plan(pb, plan, L, p, batch, flags, ws, d_params, stream, true); st != QQ_OK) return st;
    const double *d_out = reinterpret_cast<const double *>(ws + L.out);
    const size_t nout = 1 + 2 * (size_t)p;
    const bool grad = flags & QQ_GRAD;
    const hipMemcpyKind kind = (flags & QQ_OUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    QQ_HIP(hipMemcpy2DAsync(energy_out, sizeof(double), d_out, nout * sizeof(double), sizeof(double), batch, kind,
                            stream));
    if (grad)
        QQ_HIP(hipMemcpy2DAsync(grad_out, 2 * p * sizeof(double), d_out + 1, nout * sizeof(double),
                                2 * p * sizeof(double), batch, kind, stream));
    if (!(flags & QQ_OUT_ON_DEVICE)) QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

// Forward evaluation of one parameter set with the final state kept in `own`.
static qq_status state_into(qq_problem *pb, int p, const double *params, int flags, hipStream_t stream, DevBuf &own,
                            Layout &L)
{
    if (qq_status st = validate_eval(pb, p, 1, flags); st != QQ_OK) return st;
    if (!params) return fail(QQ_E_INVALID, "params is NULL");
    if (!(flags & QQ_PARAMS_ON_DEVICE))
        if (qq_status st = check_params_host(params, 2 * (size_t)p); st != QQ_OK) return st;
    const int f = (flags & ~QQ_GRAD) | QQ_ENERGY;
    const Plan plan = plan_for(pb, p, 1, f, true);
    L = layout_for(pb, p, 1, f, plan);
    QQ_HIP(hipSetDevice(pb->device));
    if (qq_status st = check_device_fits(pb->device, L.total, "the state"); st != QQ_OK) return st;
    if (hipMalloc(&own.p, L.total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) failed", L.total);
    QQ_HIP(poison(own.p, L.total, stream));
    return eval_core(pb, p, 1, params, f, plan, L, static_cast<char *>(own.p), stream);
}

qq_status qq_state(qq_problem *pb, int p, const double *params, int flags, void *psi_out, void *stream_)
{
    g_err.clear();
    if (!psi_out) return fail(QQ_E_INVALID, "psi_out is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevBuf own;
    Layout L;
    if (qq_status st = state_into(pb, p, params, flags, stream, own, L); st != QQ_OK) return st;
    const size_t bytes = (size_t)pb->dim * ((flags & QQ_C128) ? 16 : 8);
    QQ_HIP(hipMemcpyAsync(psi_out, static_cast<char *>(own.p) + L.psi, bytes,
                          (flags & QQ_OUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

qq_status qq_telegate_state(qq_problem *pb, int p, const double *params, const double *uniforms, int flags,
                            void *psi_out, int32_t *outcomes_out, int64_t *remote_out, void *stream_)
{
    g_err.clear();
    if (!pb || !params || !psi_out) return fail(QQ_E_INVALID, "problem / params / psi_out is NULL");
    if (p < 1 || p > QQ_MAX_P) return fail(QQ_E_INVALID, "p = %d outside [1, %d]", p, QQ_MAX_P);
    if (flags & ~QQ_OUT_ON_DEVICE) return fail(QQ_E_INVALID, "flags 0x%x: only QQ_OUT_ON_DEVICE applies", flags);
    if (pb->num_qpus < 1 || !pb->d_cross) return fail(QQ_E_ALLOCATION, "no allocation set (qq_set_allocation)");
    if (pb->n > kTelegateMaxN) return fail(QQ_E_TOO_LARGE, "n = %d: the trajectory holds n + 2 qubits, n <= %d", pb->n, kTelegateMaxN);
    if (qq_status st = check_params_host(params, 2 * (size_t)p); st != QQ_OK) return st;
    // cross-QPU couplings, row-major (pairs are stored in that order)
    std::vector<int> ci, cj;
    std::vector<double> cb;
    for (size_t k = 0; k < pb->pair_b.size(); ++k) {
        const int i = pb->pair_ij[2 * k], j = pb->pair_ij[2 * k + 1];
        if (pb->qpu[i] != pb->qpu[j]) {
            ci.push_back(i);
            cj.push_back(j);
            cb.push_back(pb->pair_b[k]);
        }
    }
    const int64_t nremote = 2 * (int64_t)ci.size() * p, nmeas = 2 * nremote;
    if (nmeas > 0 && !uniforms) return fail(QQ_E_INVALID, "uniforms is NULL (%lld needed)", (long long)nmeas);
    for (int64_t i = 0; i < nmeas; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0))
            return fail(QQ_E_INVALID, "uniforms[%lld] = %g is not in [0, 1)", (long long)i, uniforms[i]);
    const int n = pb->n, nq = n + 2, ca = n, cbq = n + 1;
    const uint64_t dim = 1ull << nq;
    const int nblocks = 256;
    const size_t o_part = align_up(dim * 16), o_out = o_part + align_up(nblocks * 8),
                 o_scale = o_out + align_up(std::max<int64_t>(1, nmeas) * 4), total = o_scale + align_up(std::max<int64_t>(1, nmeas) * 8);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    if (qq_status st = check_device_fits(pb->device, total, "the trajectory state"); st != QQ_OK) return st;
    DevBuf buf;
    if (hipMalloc(&buf.p, total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) failed", total);
    char *b = static_cast<char *>(buf.p);
    double2 *psi = reinterpret_cast<double2 *>(b);
    double *partial = reinterpret_cast<double *>(b + o_part);
    int *outcome = reinterpret_cast<int *>(b + o_out);
    double *scale = reinterpret_cast<double *>(b + o_scale);
    int slot = 0;
    // remote CNOT(c -> t): entangle the communication pair, couple and measure each side, correct the
    // data qubits (X^m1 on t, Z^m2 on c), reset the pair and remove the global phase (-1)^(m1 m2)
    auto remote_cnot = [&](int c, int t) -> qq_status {
        QQ_HIP(tg_launch_pair(psi, nq, ca, 1, 0, 0, 0, outcome, 0, stream));
        QQ_HIP(tg_launch_pair(psi, nq, cbq, 0, ca, 0, 0, outcome, 0, stream));
        QQ_HIP(tg_launch_pair(psi, nq, ca, 0, c, 0, 0, outcome, 0, stream));
        QQ_HIP(tg_launch_measure(psi, nq, ca, uniforms[slot], partial, nblocks, outcome, scale, slot, stream));
        QQ_HIP(tg_launch_pair(psi, nq, t, 0, cbq, 0, 0, outcome, 0, stream));
        QQ_HIP(tg_launch_pair(psi, nq, cbq, 1, 0, 0, 0, outcome, 0, stream));
        QQ_HIP(tg_launch_measure(psi, nq, cbq, uniforms[slot + 1], partial, nblocks, outcome, scale, slot + 1, stream));
        QQ_HIP(tg_launch_pair(psi, nq, t, 3, 0, 0, 0, outcome, slot, stream));
        QQ_HIP(tg_launch_pair(psi, nq, c, 4, 0, 0, 0, outcome, slot + 1, stream));
        QQ_HIP(tg_launch_pair(psi, nq, ca, 3, 0, 0, 0, outcome, slot, stream));
        QQ_HIP(tg_launch_pair(psi, nq, cbq, 3, 0, 0, 0, outcome, slot + 1, stream));
        QQ_HIP(tg_launch_sign(psi, nq, outcome, slot, stream));
        slot += 2;
        return QQ_OK;
    };
    QQ_HIP(tg_launch_init(psi, n, stream));
    for (int k = 0; k < p; ++k) {
        const double g = params[2 * k], be = params[2 * k + 1];
        QQ_HIP(tg_launch_local_phase(psi, n, pb->d_diag, pb->d_cross, pb->diag_type, g, stream));
        for (size_t x = 0; x < ci.size(); ++x) {
            // exp(-i g b z_i z_j) = phases exp(-i g b / 2) on z_i = 1 and on z_j = 1, and the parity phase
            // exp(+i g b (z_i xor z_j) / 2) = CNOT(i -> j) diag_j(1, e^{+i g b / 2}) CNOT(i -> j)
            QQ_HIP(tg_launch_phase1(psi, nq, ci[x], -g * cb[x] / 2.0, stream));
            QQ_HIP(tg_launch_phase1(psi, nq, cj[x], -g * cb[x] / 2.0, stream));
            if (qq_status st = remote_cnot(ci[x], cj[x]); st != QQ_OK) return st;
            QQ_HIP(tg_launch_phase1(psi, nq, cj[x], g * cb[x] / 2.0, stream));
            if (qq_status st = remote_cnot(ci[x], cj[x]); st != QQ_OK) return st;
        }
        for (int q = 0; q < n; ++q) QQ_HIP(tg_launch_pair(psi, nq, q, 2, 0, std::cos(be), std::sin(be), outcome, 0, stream));
    }
    // the data register with the communication pair in |00>
    QQ_HIP(hipMemcpyAsync(psi_out, psi, ((size_t)1 << n) * 16,
                          (flags & QQ_OUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
    if (outcomes_out && nmeas > 0)
        QQ_HIP(hipMemcpyAsync(outcomes_out, outcome, (size_t)nmeas * 4, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    if (remote_out) *remote_out = nremote;
    return QQ_OK;
}

qq_status qq_sample(qq_problem *pb, int p, const double *params, int flags, int64_t shots, const double *uniforms,
                    void *stream_, uint64_t *indices_out)
{
    g_err.clear();
    if (!uniforms || !indices_out) return fail(QQ_E_INVALID, "uniforms / indices_out is NULL");
    if (shots < 1) return fail(QQ_E_INVALID, "shots = %lld must be >= 1", (long long)shots);
    if (flags & ~(QQ_C128 | QQ_PARTITIONED | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE))
        return fail(QQ_E_INVALID, "flags 0x%x: only QQ_C128, QQ_PARTITIONED and the *_ON_DEVICE flags apply", flags);
    const bool dev_in = flags & QQ_PARAMS_ON_DEVICE, dev_out = flags & QQ_OUT_ON_DEVICE;
    if (!dev_in)
        for (int64_t i = 0; i < shots; ++i)
            if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0))
                return fail(QQ_E_INVALID, "uniforms[%lld] = %g is not in [0, 1)", (long long)i, uniforms[i]);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevBuf own;
    Layout L;
    if (qq_status st = state_into(pb, p, params, flags, stream, own, L); st != QQ_OK) return st;
    const void *psi = static_cast<char *>(own.p) + L.psi;
    const bool c128 = flags & QQ_C128;
    const uint64_t nblk = std::max<uint64_t>(1, pb->dim >> kTileBits);
    const size_t o_start = align_up(nblk * sizeof(double)), o_u = o_start + align_up((nblk + 1) * sizeof(double)),
                 o_out = o_u + (dev_in ? 0 : align_up((size_t)shots * sizeof(double))),
                 total = o_out + (dev_out ? 0 : align_up((size_t)shots * sizeof(uint64_t)));
    DevBuf buf;
    if (hipMalloc(&buf.p, total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for the shots failed", total);
    char *b = static_cast<char *>(buf.p);
    double *d_mass = reinterpret_cast<double *>(b), *d_start = reinterpret_cast<double *>(b + o_start);
    const double *d_u = dev_in ? uniforms : reinterpret_cast<const double *>(b + o_u);
    uint64_t *d_out = dev_out ? indices_out : reinterpret_cast<uint64_t *>(b + o_out);
    if (!dev_in)
        QQ_HIP(hipMemcpyAsync(b + o_u, uniforms, (size_t)shots * sizeof(double), hipMemcpyHostToDevice, stream));
    QQ_HIP(launch_block_mass(psi, c128, pb->dim, nblk, d_mass, stream));
    // prefix over the block masses in index order (host, sequential FP64)
    std::vector<double> h(nblk), start(nblk + 1);
    QQ_HIP(hipMemcpyAsync(h.data(), d_mass, nblk * sizeof(double), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    start[0] = 0.0;
    uint64_t last_blk = nblk - 1;  // the last block of nonzero mass (the last block if none has any)
    for (uint64_t i = 0; i < nblk; ++i) {
        start[i + 1] = start[i] + h[i];
        if (h[i] > 0.0) last_blk = i;
    }
    QQ_HIP(hipMemcpyAsync(d_start, start.data(), (nblk + 1) * sizeof(double), hipMemcpyHostToDevice, stream));
    QQ_HIP(launch_shots(psi, c128, pb->dim, nblk, d_start, last_blk, d_u, shots, d_out, stream));
    if (!dev_out)
        QQ_HIP(hipMemcpyAsync(indices_out, d_out, (size_t)shots * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

qq_status qq_sample_stats(qq_problem *pb, int64_t shots, const uint64_t *indices, double margin, int k, void *stream_,
                          qq_sample_stats_t *out, uint64_t *elite_index, int64_t *elite_count, double *elite_cost)
{
    g_err.clear();
    if (!pb || !indices || !out) return fail(QQ_E_INVALID, "problem / indices / out is NULL");
    if (shots < 1) return fail(QQ_E_INVALID, "shots = %lld must be >= 1", (long long)shots);
    if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(QQ_E_INVALID, "margin must be finite and >= 0");
    if (k < 0) return fail(QQ_E_INVALID, "k = %d must be >= 0", k);
    if (k > 0 && (!elite_index || !elite_count)) return fail(QQ_E_INVALID, "elite_index / elite_count is NULL");
    for (int64_t i = 0; i < shots; ++i)
        if (indices[i] >= pb->dim) return fail(QQ_E_INVALID, "indices[%lld] is not below 2^n", (long long)i);
    // distinct sampled bitstrings and their counts, in index order
    std::vector<uint64_t> sorted(indices, indices + shots);
    std::sort(sorted.begin(), sorted.end());
    std::vector<uint64_t> uniq;
    std::vector<int64_t> cnt;
    for (int64_t i = 0; i < shots; ++i) {
        if (i == 0 || sorted[i] != sorted[i - 1]) {
            uniq.push_back(sorted[i]);
            cnt.push_back(0);
        }
        ++cnt.back();
    }
    const int64_t m = (int64_t)uniq.size();
    // their costs from the stored diagonal
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    DevBuf buf;
    if (hipMalloc(&buf.p, (size_t)m * 16) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc failed");
    uint64_t *d_idx = static_cast<uint64_t *>(buf.p);
    double *d_cost = reinterpret_cast<double *>(d_idx + m);
    std::vector<double> cost(m);
    QQ_HIP(hipMemcpyAsync(d_idx, uniq.data(), (size_t)m * 8, hipMemcpyHostToDevice, stream));
    QQ_HIP(launch_gather_cost(pb->d_diag, pb->diag_type, d_idx, m, d_cost, stream));
    QQ_HIP(hipMemcpyAsync(cost.data(), d_cost, (size_t)m * 8, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));

    std::memset(out, 0, sizeof *out);
    const double S = (double)shots;
    double best = INFINITY, mean = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        best = std::min(best, cost[i]);
        mean += (double)cnt[i] * cost[i];
    }
    int64_t bi = -1, at_best = 0, low = 0, at_exact = 0, exact_idx = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (cost[i] == best) {
            at_best += cnt[i];
            if (bi < 0 || cnt[i] > cnt[bi]) bi = i;  // most frequent, then lowest index
        }
        if (cost[i] <= best + margin) low += cnt[i];
        if (cost[i] == pb->cmin) at_exact += cnt[i];
        if (uniq[i] == pb->argmin) exact_idx = cnt[i];
    }
    out->shots = shots;
    out->distinct = m;
    out->best_index = uniq[bi];
    out->best_cost = best;
    out->best_frequency = (double)cnt[bi] / S;
    out->best_cost_mass = (double)at_best / S;
    out->mean_cost = mean / S;
    out->low_cost_mass = (double)low / S;
    out->exact_cost = pb->cmin;
    out->exact_index = pb->argmin;
    out->matches_exact_cost = best == pb->cmin ? 1 : 0;
    out->matches_exact_index = uniq[bi] == pb->argmin ? 1 : 0;
    out->exact_cost_mass = (double)at_exact / S;
    out->exact_index_frequency = (double)exact_idx / S;
    // elite: the k most frequent, ties to the lower index
    std::vector<int64_t> order(m);
    for (int64_t i = 0; i < m; ++i) order[i] = i;
    const int64_t kk = std::min<int64_t>(k, m);
    std::partial_sort(order.begin(), order.begin() + kk, order.end(),
                      [&](int64_t a, int64_t b) { return cnt[a] > cnt[b] || (cnt[a] == cnt[b] && uniq[a] < uniq[b]); });
    for (int j = 0; j < k; ++j) {
        const bool have = j < kk;
        elite_index[j] = have ? uniq[order[j]] : 0;
        elite_count[j] = have ? cnt[order[j]] : 0;
        if (elite_cost) elite_cost[j] = have ? cost[order[j]] : 0.0;
    }
    out->elite = (int)kk;
    return QQ_OK;
}

qq_status qq_probabilities(qq_problem *pb, int p, const double *params, int flags, double *prob_out, void *stream_)
{
    g_err.clear();
    if (!prob_out) return fail(QQ_E_INVALID, "prob_out is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevBuf own;
    Layout L;
    if (qq_status st = state_into(pb, p, params, flags, stream, own, L); st != QQ_OK) return st;
    const void *psi = static_cast<char *>(own.p) + L.psi;
    if (flags & QQ_OUT_ON_DEVICE) {
        QQ_HIP(prof_aux(7, pb->n, 0, (double)pb->dim * (((flags & QQ_C128) ? 16 : 8) + 8), stream, [&]() {
            return launch_probabilities(psi, flags & QQ_C128, pb->dim, prob_out, stream);
        }));
        QQ_HIP(hipStreamSynchronize(stream));
        return QQ_OK;
    }
    DevBuf tmp;
    if (hipMalloc(&tmp.p, (size_t)pb->dim * sizeof(double)) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc failed");
    QQ_HIP(prof_aux(7, pb->n, 0, (double)pb->dim * (((flags & QQ_C128) ? 16 : 8) + 8), stream, [&]() {
        return launch_probabilities(psi, flags & QQ_C128, pb->dim, static_cast<double *>(tmp.p), stream);
    }));
    QQ_HIP(hipMemcpyAsync(prob_out, tmp.p, (size_t)pb->dim * sizeof(double), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    return QQ_OK;
}

qq_status qq_topk(qq_problem *pb, int p, const double *params, int flags, int k, uint64_t *idx_out, double *prob_out,
                  double *cost_out, void *stream_)
{
    g_err.clear();
    if (k < 1 || k > QQ_MAX_TOPK) return fail(QQ_E_INVALID, "k = %d outside [1, %d]", k, QQ_MAX_TOPK);
    if (pb && (uint64_t)k > pb->dim) return fail(QQ_E_INVALID, "k = %d exceeds 2^n", k);
    if (!idx_out || !prob_out) return fail(QQ_E_INVALID, "idx_out / prob_out is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    DevBuf own;
    Layout L;
    if (qq_status st = state_into(pb, p, params, flags, stream, own, L); st != QQ_OK) return st;
    const void *psi = static_cast<char *>(own.p) + L.psi;
    const int nblocks = (int)std::min<uint64_t>(1024, (pb->dim + 255) / 256);
    DevBuf scratch;
    const size_t sb = (size_t)nblocks * k * 16 + (size_t)k * 24 + 256;
    if (hipMalloc(&scratch.p, sb) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc failed");
    char *sc = static_cast<char *>(scratch.p);
    uint64_t *d_idx = reinterpret_cast<uint64_t *>(sc + (size_t)nblocks * k * 16);
    double *d_prob = reinterpret_cast<double *>(d_idx + k);
    double *d_cost = d_prob + k;
    QQ_HIP(prof_aux(8, pb->n, 0, (double)pb->dim * ((flags & QQ_C128) ? 16 : 8), stream, [&]() {
        return launch_topk(psi, flags & QQ_C128, pb->dim, k, pb->d_diag, pb->diag_type, d_idx, d_prob, d_cost, sc,
                           nblocks, stream);
    }));
    std::vector<uint64_t> hi(k);
    std::vector<double> hp(k), hc(k);
    QQ_HIP(hipMemcpyAsync(hi.data(), d_idx, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipMemcpyAsync(hp.data(), d_prob, sizeof(double) * k, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipMemcpyAsync(hc.data(), d_cost, sizeof(double) * k, hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    std::copy(hi.begin(), hi.end(), idx_out);
    std::copy(hp.begin(), hp.end(), prob_out);
    if (cost_out) std::copy(hc.begin(), hc.end(), cost_out);
    return QQ_OK;
}

qq_status qq_workspace_size_many(int count, qq_problem *const *problems, const int *p, const int *batch, int flags,
                                 const qq_many_options *opt, size_t *bytes)
{
    g_err.clear();
    if (!bytes) return fail(QQ_E_INVALID, "bytes is NULL");
    if (qq_status st = validate_many(count, problems, p, batch, flags); st != QQ_OK) return st;
    ManyLayout M;
    if (qq_status st = plan_many(count, problems, p, batch, flags, opt, M); st != QQ_OK) return st;
    *bytes = M.total;
    return QQ_OK;
}

static qq_status evaluate_many_impl(int count, qq_problem *const *problems, const int *p, const int *batch,
                           const double *const *params, int flags, const qq_many_options *opt, void *workspace,
                           size_t ws_bytes, void *stream_, double *const *energy_out, double *const *grad_out)
{
    g_err.clear();
    if (qq_status st = validate_many(count, problems, p, batch, flags); st != QQ_OK) return st;
    const bool grad = flags & QQ_GRAD;
    const bool c128 = flags & QQ_C128;
    if (!params || !energy_out || (grad && !grad_out)) return fail(QQ_E_INVALID, "params / energy_out / grad_out is NULL");
    for (int i = 0; i < count; ++i) {
        if (!params[i]) return fail(QQ_E_INVALID, "params[%d] is NULL", i);
        if (!energy_out[i]) return fail(QQ_E_INVALID, "energy_out[%d] is NULL", i);
        if (grad && !grad_out[i]) return fail(QQ_E_INVALID, "grad_out[%d] is NULL", i);
        if (!(flags & QQ_PARAMS_ON_DEVICE))
            if (qq_status st = check_params_host(params[i], (size_t)batch[i] * 2 * p[i]); st != QQ_OK) return st;
    }
    if (opt && (opt->tiles_per_chunk < 0 || opt->max_workgroups < 0 || !(opt->wait_limit_ms >= 0.0)))
        return fail(QQ_E_INVALID, "negative or non-finite option");
    ManyLayout M;
    if (qq_status st = plan_many(count, problems, p, batch, flags, opt, M); st != QQ_OK) return st;
    const int device = problems[0]->device;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(device));
    DevBuf own;
    char *ws = static_cast<char *>(workspace);
    if (!ws) {
        if (qq_status st = check_device_fits(device, M.total, "the workspace"); st != QQ_OK) return st;
        if (hipMalloc(&own.p, M.total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for the workspace failed", M.total);
        ws = static_cast<char *>(own.p);
    } else if (ws_bytes < M.total) {
        return fail(QQ_E_WORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, M.total);
    }
    QQ_HIP(poison(ws, M.total, stream));
    int rate_khz = 0;
    QQ_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device));
    const double wait_ms = (opt && opt->wait_limit_ms > 0.0) ? opt->wait_limit_ms : kDefaultWaitMs;
    const uint64_t spin_ticks = (uint64_t)(wait_ms * std::max(1, rate_khz));

    // host staging: packed parameters, then each group's descriptors (device addresses fixed up)
    std::vector<char> stage;
    const size_t nparam = M.out - M.params;
    if (!(flags & QQ_PARAMS_ON_DEVICE)) {
        stage.resize(nparam);
        for (int i = 0; i < count; ++i)
            std::memcpy(stage.data() + M.param_off[i] * sizeof(double), params[i],
                        (size_t)batch[i] * 2 * p[i] * sizeof(double));
        QQ_HIP(hipMemcpyAsync(ws + M.params, stage.data(), nparam, hipMemcpyHostToDevice, stream));
    }
    std::vector<std::vector<char>> blobs(M.groups.size());
    for (size_t gi = 0; gi < M.groups.size(); ++gi) {
        ManyGroup &G = M.groups[gi];
        for (size_t k = 0; k < G.inst.size(); ++k) {
            ManyInst &I = G.inst[k];
            const int i = G.members[k];
            I.params = (flags & QQ_PARAMS_ON_DEVICE) ? params[i]
                                                     : reinterpret_cast<const double *>(ws + M.params) + M.param_off[i];
            I.diag = problems[i]->d_diag;
            I.regq = problems[i]->d_regq;
            if (I.npasses > 1 || G.pass[I.pass_off].kind != FK_SINGLE) {
                I.psi = ws + G.states + reinterpret_cast<size_t>(I.psi);
                I.lam = grad ? ws + G.states + reinterpret_cast<size_t>(I.lam) : nullptr;
            }
            if (!G.gpass.empty()) {
                for (int j = I.pass_off; j < I.pass_off + I.npasses; ++j) {
                    PassArgs &a = G.gpass[j];
                    a.params = I.params;
                    a.diag = I.diag;
                    a.psi = I.psi;
                    a.lam = I.lam;
                }
            }
            if (flags & QQ_OUT_ON_DEVICE) {
                I.energy_out = energy_out[i];
                I.grad_out = grad ? grad_out[i] : nullptr;
                I.out_ws = nullptr;
            } else {
                I.energy_out = nullptr;
                I.grad_out = nullptr;
                I.out_ws = reinterpret_cast<double *>(ws + M.out) + M.out_off[i];
            }
        }
        std::vector<char> &blob = blobs[gi];
        blob.assign(G.desc_bytes, 0);
        std::memcpy(blob.data() + G.inst_off, G.inst.data(), G.inst.size() * sizeof(ManyInst));
        std::memcpy(blob.data() + G.pass_off, G.pass.data(), G.pass.size() * sizeof(ManyPass));
        if (!G.gpass.empty())
            std::memcpy(blob.data() + G.gpass_off, G.gpass.data(), G.gpass.size() * sizeof(PassArgs));
        std::memcpy(blob.data() + G.seg_off, G.seg.data(), G.seg.size() * sizeof(ManySeg));
        std::memcpy(blob.data() + G.slot_off, G.slot_out.data(), G.slot_out.size() * sizeof(uint16_t));
        QQ_HIP(hipMemcpyAsync(ws + G.desc, blob.data(), G.desc_bytes, hipMemcpyHostToDevice, stream));
    }
    for (ManyGroup &G : M.groups) {
        QQ_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(ws + G.ctl), 0u, (size_t)(2 + G.nstates), stream));
        ManyArgs a;
        a.inst = reinterpret_cast<const ManyInst *>(ws + G.desc + G.inst_off);
        a.pass = reinterpret_cast<const ManyPass *>(ws + G.desc + G.pass_off);
        a.gpass = G.gpass.empty() ? nullptr : reinterpret_cast<const PassArgs *>(ws + G.desc + G.gpass_off);
        a.seg = reinterpret_cast<const ManySeg *>(ws + G.desc + G.seg_off);
        a.slot_out = reinterpret_cast<const uint16_t *>(ws + G.desc + G.slot_off);
        a.nseg = (int)G.seg.size();
        a.grad = grad ? 1 : 0;
        a.total = G.total;
        a.ctl = reinterpret_cast<uint32_t *>(ws + G.ctl);
        a.partial = reinterpret_cast<double *>(ws + G.partial);
        a.spin_ticks = spin_ticks;
        ProfRec rec{};
        if (g_prof) {
            QQ_HIP(hipEventCreate(&rec.start));
            QQ_HIP(hipEventCreate(&rec.stop));
            QQ_HIP(hipEventRecord(rec.start, stream));
        }
        int grid = 0;
        QQ_HIP(launch_many(a, c128, G.diag_type, opt ? opt->max_workgroups : 0, stream, &grid));
        if (g_prof) {
            QQ_HIP(hipEventRecord(rec.stop, stream));
            rec.meta.kind = 4;
            rec.meta.pass_kind = -1;
            rec.meta.c128 = c128;
            rec.meta.diag_bytes = diag_bytes_of(G.diag_type);
            rec.meta.n = 0;
            rec.meta.batch = G.nstates;
            rec.meta.bytes = G.bytes;
            g_prof_log.push_back(rec);
        }
    }
    // error flags (and host outputs)
    std::vector<uint32_t> flags_h(M.groups.size(), 0);
    for (size_t gi = 0; gi < M.groups.size(); ++gi)
        QQ_HIP(hipMemcpyAsync(&flags_h[gi], ws + M.groups[gi].ctl + sizeof(uint32_t), sizeof(uint32_t),
                              hipMemcpyDeviceToHost, stream));
    std::vector<double> h;
    if (!(flags & QQ_OUT_ON_DEVICE)) {
        size_t nout = 0;
        for (int i = 0; i < count; ++i) nout += (size_t)batch[i] * (1 + 2 * p[i]);
        h.resize(nout);
        QQ_HIP(hipMemcpyAsync(h.data(), ws + M.out, nout * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    QQ_HIP(hipStreamSynchronize(stream));
    for (uint32_t f : flags_h)
        if (f) return fail(QQ_E_DEVICE, "persistent launch: a dependency wait exceeded %.0f ms; results are invalid", wait_ms);
    if (!(flags & QQ_OUT_ON_DEVICE)) {
        for (int i = 0; i < count; ++i) {
            const size_t nout = 1 + 2 * (size_t)p[i];
            const double *src = h.data() + M.out_off[i];
            for (int b = 0; b < batch[i]; ++b) {
                energy_out[i][b] = src[(size_t)b * nout];
                if (grad)
                    for (int j = 0; j < 2 * p[i]; ++j) grad_out[i][(size_t)b * 2 * p[i] + j] = src[(size_t)b * nout + 1 + j];
            }
        }
    }
    return QQ_OK;
}

static qq_status evaluate_guarded_impl(qq_problem *pb, int p, int batch, const double *params, int flags, double tol,
                              void *stream, double *energy_out, double *grad_out, int32_t *c128_out,
                              double *grad_err_out)
{
    g_err.clear();
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    if (flags & (QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE))
        return fail(QQ_E_UNSUPPORTED, "qq_evaluate_guarded takes host parameters and outputs");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(QQ_E_INVALID, "tol must be finite and >= 0");
    if (tol == 0.0) tol = 1e-5;
    if (!params || !energy_out) return fail(QQ_E_INVALID, "params / energy_out is NULL");
    const bool grad = flags & QQ_GRAD;
    if (grad && !grad_out) return fail(QQ_E_INVALID, "QQ_GRAD requires grad_out");
    // first pass in the requested precision (complex64 unless QQ_C128), into local buffers so that
    // nothing is written to the caller's outputs on error
    std::vector<double> e(batch), g(grad ? (size_t)batch * 2 * p : 0);
    if (qq_status st = qq_evaluate(pb, p, batch, params, flags, nullptr, 0, stream, e.data(), grad ? g.data() : nullptr);
        st != QQ_OK)
        return st;
    std::vector<int32_t> up(batch);
    std::vector<double> err(batch);
    const std::vector<int> sets =
        guard_sets(pb, p, batch, grad ? g.data() : nullptr, tol, (flags & QQ_C128) != 0, up.data(), err.data());
    std::vector<C128Job> jobs{{pb, p, params, sets, e.data(), g.data()}};
    if (qq_status st = recompute_c128(jobs, flags, stream); st != QQ_OK) return st;
    if (grad)
        for (int b : sets) err[b] = kC128GradRel * max_abs(&g[(size_t)b * 2 * p], 2 * p);
    std::memcpy(energy_out, e.data(), batch * sizeof(double));
    if (grad) std::memcpy(grad_out, g.data(), g.size() * sizeof(double));
    if (c128_out) std::memcpy(c128_out, up.data(), batch * sizeof(int32_t));
    if (grad_err_out) std::memcpy(grad_err_out, err.data(), batch * sizeof(double));
    return QQ_OK;
}

static qq_status evaluate_many_guarded_impl(int count, qq_problem *const *problems, const int *p, const int *batch,
                                   const double *const *params, int flags, const qq_many_options *opt, double tol,
                                   void *stream, double *const *energy_out, double *const *grad_out,
                                   int32_t *const *c128_out, double *const *grad_err_out)
{
    g_err.clear();
    if (qq_status st = validate_many(count, problems, p, batch, flags); st != QQ_OK) return st;
    if (flags & (QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE))
        return fail(QQ_E_UNSUPPORTED, "qq_evaluate_many_guarded takes host parameters and outputs");
    if (flags & QQ_C128) return fail(QQ_E_UNSUPPORTED, "qq_evaluate_many_guarded evaluates in complex64 first");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(QQ_E_INVALID, "tol must be finite and >= 0");
    if (tol == 0.0) tol = 1e-5;
    const bool grad = flags & QQ_GRAD;
    if (!params || !energy_out || (grad && !grad_out)) return fail(QQ_E_INVALID, "params / energy_out / grad_out is NULL");
    for (int i = 0; i < count; ++i)
        if (!energy_out[i] || (grad && !grad_out[i])) return fail(QQ_E_INVALID, "output %d is NULL", i);
    std::vector<std::vector<double>> e(count), g(count);
    std::vector<double *> ep(count), gp(count);
    for (int i = 0; i < count; ++i) {
        e[i].resize(batch[i]);
        g[i].resize(grad ? (size_t)batch[i] * 2 * p[i] : 1);
        ep[i] = e[i].data();
        gp[i] = g[i].data();
    }
    if (qq_status st = qq_evaluate_many(count, problems, p, batch, params, flags, opt, nullptr, 0, stream, ep.data(),
                                        grad ? gp.data() : nullptr);
        st != QQ_OK)
        return st;
    std::vector<std::vector<int32_t>> up(count);
    std::vector<std::vector<double>> err(count);
    std::vector<C128Job> jobs;
    for (int i = 0; i < count; ++i) {
        up[i].resize(batch[i]);
        err[i].resize(batch[i]);
        std::vector<int> sets =
            guard_sets(problems[i], p[i], batch[i], grad ? g[i].data() : nullptr, tol, false, up[i].data(), err[i].data());
        if (!sets.empty()) jobs.push_back({problems[i], p[i], params[i], std::move(sets), e[i].data(), g[i].data()});
    }
    if (qq_status st = recompute_c128(jobs, flags, stream); st != QQ_OK) return st;
    for (int i = 0; i < count; ++i)
        if (grad)
            for (int b = 0; b < batch[i]; ++b)
                if (up[i][b]) err[i][b] = kC128GradRel * max_abs(&g[i][(size_t)b * 2 * p[i]], 2 * p[i]);
    for (int i = 0; i < count; ++i) {
        std::memcpy(energy_out[i], e[i].data(), batch[i] * sizeof(double));
        if (grad) std::memcpy(grad_out[i], g[i].data(), (size_t)batch[i] * 2 * p[i] * sizeof(double));
        if (c128_out && c128_out[i]) std::memcpy(c128_out[i], up[i].data(), batch[i] * sizeof(int32_t));
        if (grad_err_out && grad_err_out[i]) std::memcpy(grad_err_out[i], err[i].data(), batch[i] * sizeof(double));
    }
    return QQ_OK;
}

qq_status qq_graph_create(qq_problem *pb, int p, int batch, int flags, const double *adam, double *params,
                          int history, void *stream_, qq_graph **out)
{
    g_err.clear();
    if (!out) return fail(QQ_E_INVALID, "out is NULL");
    if (!params) return fail(QQ_E_INVALID, "params is NULL (device [batch][2p] parameters)");
    if (flags & (QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE))
        return fail(QQ_E_INVALID, "qq_graph_create takes device parameters implicitly; pass no *_ON_DEVICE flag");
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    if (history < 0) return fail(QQ_E_INVALID, "history = %d must be >= 0", history);
    double hp[4] = {0.01, 0.9, 0.999, 1e-8};
    if (adam) {
        for (int i = 0; i < 4; ++i) hp[i] = adam[i];
        if (!(hp[0] > 0.0 && std::isfinite(hp[0])) || !(hp[1] >= 0.0 && hp[1] < 1.0) || !(hp[2] >= 0.0 && hp[2] < 1.0) ||
            !(hp[3] > 0.0 && std::isfinite(hp[3])))
            return fail(QQ_E_INVALID, "Adam hyperparameters need lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
    }
    std::unique_ptr<qq_graph> g(new (std::nothrow) qq_graph());
    if (!g) return fail(QQ_E_NOMEM, "host allocation failed");
    g->pb = pb;
    g->p = p;
    g->B = batch;
    g->flags = (flags | QQ_ENERGY | QQ_GRAD | QQ_PARAMS_ON_DEVICE) & ~QQ_OUT_ON_DEVICE;
    g->device = pb->device;
    g->lr = hp[0];
    g->beta1 = hp[1];
    g->beta2 = hp[2];
    g->eps = hp[3];
    g->x = params;
    g->hist_len = history;
    g->plan = plan_for(pb, p, batch, g->flags, false);
    g->L = layout_for(pb, p, batch, g->flags, g->plan);
    if (g->plan.nslots > kMaxSlots) return fail(QQ_E_UNSUPPORTED, "plan needs %d accumulator slots", g->plan.nslots);
    const size_t np = (size_t)batch * 2 * p;
    const size_t o_m = align_up(g->L.total), o_v = o_m + align_up(np * 8), o_e = o_v + align_up(np * 8),
                 o_g = o_e + align_up((size_t)batch * 8), o_h = o_g + align_up(np * 8),
                 o_s = o_h + align_up((size_t)std::max(1, history) * batch * 8), total = o_s + 256;
    QQ_HIP(hipSetDevice(g->device));
    if (qq_status st = check_device_fits(g->device, total, "the optimiser workspace"); st != QQ_OK) return st;
    if (hipMalloc(&g->mem, total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) failed", total);
    char *base = static_cast<char *>(g->mem);
    g->ws = base;
    g->m = reinterpret_cast<double *>(base + o_m);
    g->v = reinterpret_cast<double *>(base + o_v);
    g->energy = reinterpret_cast<double *>(base + o_e);
    g->grad = reinterpret_cast<double *>(base + o_g);
    g->hist = history > 0 ? reinterpret_cast<double *>(base + o_h) : nullptr;
    g->step = reinterpret_cast<int *>(base + o_s);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (qq_status st = zero_state(g.get(), stream); st != QQ_OK) return st;
    if (history > 0) QQ_HIP(launch_fill_f64(g->hist, 0.0, (size_t)history * batch, stream));
    QQ_HIP(launch_fill_f64(g->energy, 0.0, (size_t)batch, stream));
    QQ_HIP(launch_fill_f64(g->grad, 0.0, np, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    // capture one step on a private stream (default priority)
    QQ_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    QQ_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    const qq_status st = enqueue_step(g.get(), g->cap, true);
    const std::string err = g_err;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
    g->graph = graph;
    if (st != QQ_OK) return fail(st, "capturing the step failed: %s", err.c_str());
    if (ec != hipSuccess) return fail(QQ_E_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    QQ_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    ++pb->graphs;
    *out = g.release();
    return QQ_OK;
}

qq_status qq_graph_run(qq_graph *g, int steps, void *stream_)
{
    g_err.clear();
    if (!g) return fail(QQ_E_INVALID, "graph is NULL");
    if (steps < 0) return fail(QQ_E_INVALID, "steps = %d must be >= 0", steps);
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(g->device));
    for (int i = 0; i < steps; ++i) QQ_HIP(hipGraphLaunch(g->exec, stream));
    return QQ_OK;
}

qq_status qq_graph_step_eager(qq_graph *g, void *stream_)
{
    g_err.clear();
    if (!g) return fail(QQ_E_INVALID, "graph is NULL");
    QQ_HIP(hipSetDevice(g->device));
    return enqueue_step(g, static_cast<hipStream_t>(stream_), false);
}

qq_status qq_graph_reset(qq_graph *g, void *stream_)
{
    g_err.clear();
    if (!g) return fail(QQ_E_INVALID, "graph is NULL");
    QQ_HIP(hipSetDevice(g->device));
    return zero_state(g, static_cast<hipStream_t>(stream_));
}

qq_status qq_graph_read(qq_graph *g, double *energy, double *grad, double *history, int *steps, int flags,
                        void *stream_)
{
    g_err.clear();
    if (!g) return fail(QQ_E_INVALID, "graph is NULL");
    if (flags & ~QQ_OUT_ON_DEVICE) return fail(QQ_E_INVALID, "only QQ_OUT_ON_DEVICE is accepted");
    if (history && g->hist_len == 0) return fail(QQ_E_INVALID, "the graph keeps no history (created with history = 0)");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(g->device));
    const hipMemcpyKind kind = (flags & QQ_OUT_ON_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t np = (size_t)g->B * 2 * g->p;
    if (energy) QQ_HIP(hipMemcpyAsync(energy, g->energy, (size_t)g->B * 8, kind, stream));
    if (grad) QQ_HIP(hipMemcpyAsync(grad, g->grad, np * 8, kind, stream));
    if (history) QQ_HIP(hipMemcpyAsync(history, g->hist, (size_t)g->hist_len * g->B * 8, kind, stream));
    int hs = 0;
    if (steps) QQ_HIP(hipMemcpyAsync(&hs, g->step, sizeof(int), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    if (steps) *steps = hs;
    return QQ_OK;
}

qq_status qq_graph_destroy(qq_graph *g)
{
    if (g && g->exec) --g->pb->graphs;  // counted once instantiated
    delete g;
    return QQ_OK;
}

qq_status qq_set_schedule(qq_problem *pb, int p, int batch, int flags, const qq_schedule *sch)
{
    g_err.clear();
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    if (!sch) {  // back to the built-in heuristic
        const int sf = sched_flags(flags);
        pb->sched.erase(std::remove_if(pb->sched.begin(), pb->sched.end(),
                                       [&](const qq_problem::Sched &e) {
                                           return e.p == p && e.batch == batch && e.flags == sf;
                                       }),
                        pb->sched.end());
        return QQ_OK;
    }
    const uint64_t T = tiles_per_state(pb->n);
    const int G = sch->workgroups_per_state;
    if (G < 1 || (G & (G - 1)) || (uint64_t)G > T)
        return fail(QQ_E_INVALID, "workgroups_per_state = %d must be a power of two in [1, %llu]", G,
                    (unsigned long long)T);
    if (sch->set_pairing < 0 || sch->set_pairing >= kPairings || (sch->set_pairing != 0 && !pairing_applies(pb->n)))
        return fail(QQ_E_INVALID, "set_pairing = %d is not available at n = %d", sch->set_pairing, pb->n);
    if ((size_t)batch * (size_t)G > 0x7fffffffull) return fail(QQ_E_INVALID, "batch * workgroups_per_state too large");
    if (sch->tile_order != 0 && sch->tile_order != 1)
        return fail(QQ_E_INVALID, "tile_order = %d must be 0 (strided) or 1 (blocked)", sch->tile_order);
    if (sch->set_order < 0 || sch->set_order > 1 || (sch->set_order == 1 && !set_order_applies(pb->n)))
        return fail(QQ_E_INVALID, "set_order = %d is not available at n = %d", sch->set_order, pb->n);
    pin_sched(pb, p, batch, flags, G, sch->set_pairing, sch->tile_order, sch->set_order, sch->ms);
    return QQ_OK;
}

qq_status qq_get_schedule(const qq_problem *pb, int p, int batch, int flags, qq_schedule *out)
{
    g_err.clear();
    if (!out) return fail(QQ_E_INVALID, "out is NULL");
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    std::memset(out, 0, sizeof *out);
    if (const auto *e = find_sched(pb, p, batch, flags)) {
        out->workgroups_per_state = e->G;
        out->set_pairing = e->pairing;
        out->tile_order = e->blocked;
        out->set_order = e->set_order;
        out->ms = e->ms;
        out->pinned = 1;
    } else {
        out->workgroups_per_state = choose_G(pb->n, batch);
        out->set_pairing = 0;
        out->set_order = default_set_order(pb->n);
    }
    return QQ_OK;
}

qq_status qq_autotune(qq_problem *pb, int p, int batch, int flags, const char *cache_path, void *stream_,
                      qq_schedule *out)
{
    g_err.clear();
    if (!out) return fail(QQ_E_INVALID, "out is NULL");
    flags &= ~(QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE);
    if (qq_status st = validate_eval(pb, p, batch, flags); st != QQ_OK) return st;
    std::memset(out, 0, sizeof *out);
    char keybuf[512];
    std::snprintf(keybuf, sizeof keybuf,
                  "{\"kind\":\"evaluate\",\"device\":\"%s\",\"n\":%d,\"p\":%d,\"batch\":%d,\"flags\":%d,"
                  "\"diag_bytes\":%d,",
                  device_tag(pb->device).c_str(), pb->n, p, batch, sched_flags(flags), diag_bytes_of(pb->diag_type));
    const std::string key(keybuf);
    std::string line;
    if (cache_lookup(cache_path, key, line)) {
        double G = 0, pr = 0, ms = 0, order = 0, so = 0;
        if (json_num(line, "G", G) && json_num(line, "pairing", pr) && json_num(line, "ms", ms) &&
            json_num(line, "tile_order", order) && json_num(line, "set_order", so)) {
            qq_schedule s{(int)G, (int)pr, ms, 1, 1, 0, (int)order, (int)so};
            if (qq_status st = qq_set_schedule(pb, p, batch, flags, &s); st == QQ_OK) {
                *out = s;
                return QQ_OK;
            }
            g_err.clear();  // a stale entry: tune again
        }
    }
    // stage 1: the heuristic G, half and double it, times every pairing where it applies (strided
    // tile order, default set order); stage 2: the blocked tile order at the best pairing, for the
    // best G, half and double; stage 3: the other set order at the best of those
    const uint64_t T = tiles_per_state(pb->n);
    const int G0 = choose_G(pb->n, batch);
    auto g_candidates = [&](int Gc) {
        std::vector<int> v;
        for (int G : {Gc / 2, Gc, Gc * 2})
            if (G >= 1 && (uint64_t)G <= T && (size_t)batch * G <= 0x7fffffffull) v.push_back(G);
        return v;
    };
    const std::vector<int> Gs = g_candidates(G0);
    const int npair = pairing_applies(pb->n) ? kPairings : 1;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(pb->device));
    size_t need = 0;
    const Plan plan0 = make_plan(pb->n, p, plan_mode(flags | QQ_ENERGY, false), 0);
    for (int G : g_candidates(G0 * 2)) need = std::max(need, make_layout(pb, p, batch, flags, plan0, G).total);
    if (qq_status st = check_device_fits(pb->device, need, "the tuning workspace"); st != QQ_OK) return st;
    DevBuf ws, dx;
    if (hipMalloc(&ws.p, need) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for tuning failed", need);
    const std::vector<double> x = tune_params((size_t)batch * 2 * p, 0x5eed + (uint64_t)pb->n * 131 + p);
    QQ_HIP(hipMalloc(&dx.p, x.size() * sizeof(double)));
    QQ_HIP(hipMemcpy(dx.p, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice));
    const int eflags = flags | QQ_PARAMS_ON_DEVICE;
    double best = INFINITY;
    const int so0 = default_set_order(pb->n);
    int bestG = G0, bestP = 0, bestO = 0, bestS = so0, tried = 0;
    auto time_one = [&](int pr, int G, int order, int so) -> qq_status {
        const Plan plan = make_plan(pb->n, p, plan_mode(flags | QQ_ENERGY, false), pr, so);
        Layout L = make_layout(pb, p, batch, flags, plan, G);
        L.blocked = order;
        double ms = 0;
        auto run = [&]() {
            return run_plan(pb, plan, L, p, batch, eflags, static_cast<char *>(ws.p), static_cast<const double *>(dx.p),
                            stream, true);
        };
        if (qq_status st = time_median(stream, run, ms); st != QQ_OK) return st;
        ++tried;
        if (ms < best) {
            best = ms;
            bestG = G;
            bestP = pr;
            bestO = order;
            bestS = so;
        }
        return QQ_OK;
    };
    for (int pr = 0; pr < npair; ++pr)
        for (int G : Gs)
            if (qq_status st = time_one(pr, G, 0, so0); st != QQ_OK) return st;
    const bool multi_pass = make_sets(pb->n, 0).size() > 1 && !(flags & QQ_C128) && pb->n <= kFastMaxN;
    if (multi_pass) {  // the tile order only applies to the specialised multi-pass kernels
        const int pr = bestP;
        for (int G : g_candidates(bestG))
            if (qq_status st = time_one(pr, G, 1, so0); st != QQ_OK) return st;
    }
    if (set_order_applies(pb->n))
        if (qq_status st = time_one(bestP, bestG, bestO, 1 - so0); st != QQ_OK) return st;
    pin_sched(pb, p, batch, flags, bestG, bestP, bestO, bestS, best);
    char tail[200];
    std::snprintf(tail, sizeof tail, "\"G\":%d,\"pairing\":%d,\"tile_order\":%d,\"set_order\":%d,\"ms\":%.4f}",
                  bestG, bestP, bestO, bestS, best);
    if (qq_status st = cache_append(cache_path, key + tail); st != QQ_OK) return st;
    *out = qq_schedule{bestG, bestP, best, 1, 0, tried, bestO, bestS};
    return QQ_OK;
}

qq_status qq_autotune_many(int count, qq_problem *const *problems, const int *p, const int *batch, int flags,
                           const char *cache_path, void *stream_, qq_many_options *out, double *ms_out)
{
    g_err.clear();
    if (!out) return fail(QQ_E_INVALID, "out is NULL");
    flags &= ~(QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE);
    if (qq_status st = validate_many(count, problems, p, batch, flags); st != QQ_OK) return st;
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < count; ++i) {
        h = fnv1a(h, problems[i]->n);
        h = fnv1a(h, p[i]);
        h = fnv1a(h, batch[i]);
        h = fnv1a(h, diag_bytes_of(problems[i]->diag_type));
    }
    const int device = problems[0]->device;
    char keybuf[512];
    std::snprintf(keybuf, sizeof keybuf, "{\"kind\":\"many\",\"device\":\"%s\",\"count\":%d,\"flags\":%d,\"shape\":\"%016llx\",",
                  device_tag(device).c_str(), count, sched_flags(flags), (unsigned long long)h);
    const std::string key(keybuf);
    std::string line;
    if (cache_lookup(cache_path, key, line)) {
        double tpc = 0, mw = 0, ms = 0;
        if (json_num(line, "tiles_per_chunk", tpc) && json_num(line, "max_workgroups", mw) && json_num(line, "ms", ms) &&
            tpc >= 1 && mw >= 0) {
            out->tiles_per_chunk = (int)tpc;
            out->max_workgroups = (int)mw;
            out->wait_limit_ms = 0.0;
            if (ms_out) *ms_out = ms;
            return QQ_OK;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    QQ_HIP(hipSetDevice(device));
    int cus = 0;
    QQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    // parameters on the device, outputs on the device
    std::vector<std::vector<double>> xs(count);
    size_t np = 0, ne = 0;
    for (int i = 0; i < count; ++i) {
        xs[i] = tune_params((size_t)batch[i] * 2 * p[i], 0x5eed + (uint64_t)i);
        np += xs[i].size();
        ne += (size_t)batch[i];
    }
    DevBuf dparams, dout;
    QQ_HIP(hipMalloc(&dparams.p, np * sizeof(double)));
    QQ_HIP(hipMalloc(&dout.p, (ne + np) * sizeof(double)));
    std::vector<const double *> pp(count);
    std::vector<double *> ep(count), gp(count);
    {
        double *dp = static_cast<double *>(dparams.p), *de = static_cast<double *>(dout.p), *dg = de + ne;
        for (int i = 0; i < count; ++i) {
            QQ_HIP(hipMemcpy(dp, xs[i].data(), xs[i].size() * sizeof(double), hipMemcpyHostToDevice));
            pp[i] = dp;
            ep[i] = de;
            gp[i] = dg;
            dp += xs[i].size();
            de += batch[i];
            dg += xs[i].size();
        }
    }
    const int eflags = flags | QQ_ENERGY | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE;
    std::vector<qq_many_options> cands;
    for (int tpc : {4, 8, 16, 24, 32, 48, 64})
        for (int mw : {0, 2 * cus}) cands.push_back({tpc, mw, 0.0});
    size_t need = 0;
    for (const auto &c : cands) {
        ManyLayout M;
        if (qq_status st = plan_many(count, problems, p, batch, eflags, &c, M); st != QQ_OK) return st;
        need = std::max(need, M.total);
    }
    if (qq_status st = check_device_fits(device, need, "the tuning workspace"); st != QQ_OK) return st;
    DevBuf ws;
    if (hipMalloc(&ws.p, need) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) for tuning failed", need);
    double best = INFINITY;
    qq_many_options bopt{16, 0, 0.0};
    for (const auto &c : cands) {
        double ms = 0;
        auto run = [&]() {
            return qq_evaluate_many(count, problems, p, batch, pp.data(), eflags, &c, ws.p, need, stream, ep.data(),
                                    (flags & QQ_GRAD) ? gp.data() : nullptr);
        };
        if (qq_status st = time_median(stream, run, ms); st != QQ_OK) return st;
        if (ms < best) {
            best = ms;
            bopt = c;
        }
    }
    char tail[160];
    std::snprintf(tail, sizeof tail, "\"tiles_per_chunk\":%d,\"max_workgroups\":%d,\"ms\":%.4f}", bopt.tiles_per_chunk,
                  bopt.max_workgroups, best);
    if (qq_status st = cache_append(cache_path, key + tail); st != QQ_OK) return st;
    *out = bopt;
    if (ms_out) *ms_out = best;
    return QQ_OK;
}

qq_status qq_profile_enable(int enable)
{
    g_prof = enable != 0;
    return QQ_OK;
}

qq_status qq_profile_read(qq_launch_record *out, int max, int *count)
{
    if (!count || (max > 0 && !out)) return fail(QQ_E_INVALID, "NULL argument");
    int k = 0;
    qq_status st = QQ_OK;
    for (auto &r : g_prof_log) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            st = fail(QQ_E_DEVICE, "event timing failed");
        r.meta.ms = ms;
        if (k < max) out[k] = r.meta;
        ++k;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_log.clear();
    *count = std::min(k, std::max(max, 0));
    return st;
}

qq_status qq_evaluate_plain(qq_problem *pb, int p, const double *params, int flags, void *stream_, double *energy_out,
                            double *grad_out)
{
    g_err.clear();
    if (qq_status st = validate_eval(pb, p, 1, flags); st != QQ_OK) return st;
    if (flags & (QQ_PARTITIONED | QQ_PARAMS_ON_DEVICE | QQ_OUT_ON_DEVICE))
        return fail(QQ_E_UNSUPPORTED, "the plain per-gate path takes host params/outputs and no partitioning");
    if (!params || !energy_out) return fail(QQ_E_INVALID, "NULL argument");
    if ((flags & QQ_GRAD) && !grad_out) return fail(QQ_E_INVALID, "QQ_GRAD requires grad_out");
    if (qq_status st = check_params_host(params, 2 * (size_t)p); st != QQ_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const bool grad = flags & QQ_GRAD;
    const size_t state = (size_t)pb->dim * 16;
    const int nblocks = (int)std::min<uint64_t>(2048, std::max<uint64_t>(1, pb->dim / 512));
    const size_t total = align_up(state) * (grad ? 2 : 1) + align_up(sizeof(double) * nblocks) +
                         align_up(sizeof(double) * (1 + 2 * p));
    QQ_HIP(hipSetDevice(pb->device));
    if (qq_status st = check_device_fits(pb->device, total, "the plain-path states"); st != QQ_OK) return st;
    DevBuf own;
    if (hipMalloc(&own.p, total) != hipSuccess) return fail(QQ_E_NOMEM, "hipMalloc(%zu) failed", total);
    char *ws = static_cast<char *>(own.p);
    PlainArgs a;
    a.n = pb->n;
    a.p = p;
    a.grad = grad;
    a.dim = pb->dim;
    a.params = params;
    a.diag = pb->d_diag;
    a.diag_type = pb->diag_type;
    a.psi = ws;
    a.lam = grad ? ws + align_up(state) : nullptr;
    a.partial = reinterpret_cast<double *>(ws + align_up(state) * (grad ? 2 : 1));
    a.result = reinterpret_cast<double *>(ws + align_up(state) * (grad ? 2 : 1) + align_up(sizeof(double) * nblocks));
    a.nblocks = nblocks;
    // profiled as one record: the whole per-gate launch sequence, without the allocation and the copy-out
    QQ_HIP(prof_aux(9, pb->n, diag_bytes_of(pb->diag_type), 0.0, stream, [&]() { return run_plain(a, stream); }));
    std::vector<double> h(1 + 2 * p);
    QQ_HIP(hipMemcpyAsync(h.data(), a.result, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream));
    QQ_HIP(hipStreamSynchronize(stream));
    energy_out[0] = h[0];
    if (grad)
        for (int j = 0; j < 2 * p; ++j) grad_out[j] = h[1 + j];
    return QQ_OK;
}

// ---- public evaluation entry points (QQ_LOG: one line per call) ------------------------------

qq_status qq_evaluate(qq_problem *pb, int p, int batch, const double *params, int flags, void *workspace,
                      size_t ws_bytes, void *stream, double *energy_out, double *grad_out)
{
    CallLog log("qq_evaluate", pb ? pb->n : -1, p, batch, flags);
    return log(evaluate_impl(pb, p, batch, params, flags, workspace, ws_bytes, stream, energy_out, grad_out));
}

qq_status qq_evaluate_static(qq_problem *pb, int p, int batch, const double *params, int flags, void *stream,
                             double *energy_out, double *grad_out)
{
    CallLog log("qq_evaluate_static", pb ? pb->n : -1, p, batch, flags);
    return log(evaluate_static_impl(pb, p, batch, params, flags, stream, energy_out, grad_out));
}

qq_status qq_evaluate_many(int count, qq_problem *const *problems, const int *p, const int *batch,
                           const double *const *params, int flags, const qq_many_options *opt, void *workspace,
                           size_t ws_bytes, void *stream, double *const *energy_out, double *const *grad_out)
{
    CallLog log("qq_evaluate_many", count, -1, -1, flags);
    return log(evaluate_many_impl(count, problems, p, batch, params, flags, opt, workspace, ws_bytes, stream,
                                  energy_out, grad_out));
}

qq_status qq_evaluate_guarded(qq_problem *pb, int p, int batch, const double *params, int flags, double tol,
                              void *stream, double *energy_out, double *grad_out, int32_t *c128_out,
                              double *grad_err_out)
{
    CallLog log("qq_evaluate_guarded", pb ? pb->n : -1, p, batch, flags);
    return log(evaluate_guarded_impl(pb, p, batch, params, flags, tol, stream, energy_out, grad_out, c128_out,
                                     grad_err_out));
}

qq_status qq_evaluate_many_guarded(int count, qq_problem *const *problems, const int *p, const int *batch,
                                   const double *const *params, int flags, const qq_many_options *opt, double tol,
                                   void *stream, double *const *energy_out, double *const *grad_out,
                                   int32_t *const *c128_out, double *const *grad_err_out)
{
    CallLog log("qq_evaluate_many_guarded", count, -1, -1, flags);
    return log(evaluate_many_guarded_impl(count, problems, p, batch, params, flags, opt, tol, stream, energy_out,
                                          grad_out, c128_out, grad_err_out));
}

}  // extern "C"
