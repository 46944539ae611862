// qq_internal.h -- internal types shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qaoa_qubo.h"

namespace qq {

// ---- tile geometry of the fused pass kernel ------------------------------------------------
// A tile is 2^12 amplitudes of one state held in registers by 256 threads
// (4 waves), 16 amplitudes per thread and state.  Tile-local bit j maps to a
// global qubit: bits 0..3 always map to qubits 0..3 (a 16-amplitude, 128-byte
// contiguous run for complex64); bits 4..11 map either to qubits 4..11 (the
// "low" tile, fully contiguous) or to two runs of four qubits, pos4..pos4+3 and
// pos8..pos8+3 (a "high" tile).
// The 12 tile bits form three 4-bit register groups; a group is mixed in
// registers after an LDS transpose brings it into the per-thread register index.
constexpr int kTileBits = 12;
constexpr int kTile = 1 << kTileBits;
constexpr int kThreads = 256;
constexpr int kRegs = 16;
constexpr int kMaxOps = 4 * QQ_MAX_P + 4;
constexpr int kMaxLocalSlots = 4;
constexpr int kMaxSlots = 512;
constexpr int kMaxImmSlots = 1 + 2 * QQ_MAX_P;  // slots of a single-pass plan
constexpr uint8_t kNoSlot = 0xff;

enum OpKind : uint8_t {
    OP_MIX = 1,            // RX(+-2 beta_k) on the active tile bits of the selected states
    OP_PHASE = 2,          // states *= exp(-+ i gamma_k C)
    OP_ENERGY = 3,         // acc += |psi|^2 C
    OP_ENERGY_LAMBDA = 4,  // acc += |psi|^2 C ; lambda = C psi (lambda becomes live)
    OP_GGAMMA = 5          // acc += C Im(conj(lambda) psi) ; optionally un-phase both states
};

enum OpFlag : uint8_t {
    OPF_INVERSE = 1,      // MIX/PHASE: apply the inverse rotation
    OPF_UNPHASE = 2,      // GGAMMA: afterwards multiply both states by exp(+i gamma_k C)
    OPF_PARTITIONED = 4   // PHASE / GGAMMA un-phase: per-QPU local factors then the cross factor
};

struct Op {
    uint8_t kind;
    uint8_t layer;   // 0-based layer k
    uint8_t states;  // bit 0: psi, bit 1: lambda
    uint8_t flags;   // OpFlag
    uint16_t active; // MIX: tile-bit mask
    uint8_t slot;    // local accumulator slot, kNoSlot = none
    uint8_t pad;
};

enum PassFlag : uint32_t {
    PF_INIT = 1,       // psi = 2^(-n/2) everywhere (no load)
    PF_LOAD_PSI = 2,
    PF_LOAD_LAM = 4,
    PF_STORE_PSI = 8,
    PF_STORE_LAM = 16
};

enum DiagType : int { DIAG_F64 = 0, DIAG_I32 = 1, DIAG_I16 = 2 };

// Variables of each QPU for the partitioned phase: local table m is indexed by
// the bits of its variables, in ascending variable order.
struct PartDesc {
    int nparts;
    int nvars[QQ_MAX_QPUS];
    uint64_t table_off[QQ_MAX_QPUS];  // element offset of table m inside the packed tables buffer
    uint8_t vars[QQ_MAX_QPUS][QQ_MAX_N];
    uint64_t vmask[QQ_MAX_QPUS];      // bit i set when variable i + 1 sits on QPU m
};

struct PassArgs {
    int n;
    int p;
    int B;            // states in this launch
    int G;            // workgroups per state
    uint64_t tiles;   // tiles per state
    uint64_t dim_mask;
    int pos4, pos8;   // qubits of tile bits 4..7 (pos4..pos4+3) and 8..11 (pos8..pos8+3), pos4 + 4 <= pos8
    int high;         // 0: tile bits are qubits 0..11 (pos4 = 4, pos8 = 8)
    int w1, w2;       // tile-index bits below pos4 (above qubit 3) and between the runs
    uint32_t flags;
    int nops;
    int nslots;
    int slot_base;
    int slot_stride;  // B * G
    double amp0;
    const double *params;  // device [B][2p]
    const void *diag;
    void *psi;
    void *lam;
    uint64_t state_stride;
    double *partial;
    const void *part_tables;  // packed local tables (diag element type)
    const void *cross_diag;   // 2^n cross diagonal (diag element type)
    const PartDesc *part;     // device
    Op ops[kMaxOps];
};

struct FinalizeArgs {
    int B;
    int G;
    int p;
    int nslots;
    double escale;        // 2^(n-12) for replicated small states, else 1
    double shift;         // added to the energy: the passes accumulated sum |psi|^2 (C - shift)
    const double *partial;
    double *out;          // [B][1 + 2p] : energy, then interleaved gradient
    uint16_t slot_out[kMaxSlots];  // output index of each global slot
};

// Kernel launchers (qq_kernels.hip).
hipError_t launch_pass(const PassArgs &a, bool c128, int nstates, int diag_type, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t s);
hipError_t launch_cost_diag(int n, int diag_type, const double *d_ell, const int32_t *d_ell_i, int npairs,
                            const int32_t *d_pair_ij, const double *d_pair_b, const int32_t *d_pair_bi, double c0,
                            int32_t c0_i, void *d_out, uint64_t dim, hipStream_t s);
hipError_t launch_minmax(const void *d_diag, int diag_type, uint64_t dim, double *d_part, uint64_t *d_idx,
                         int nblocks, hipStream_t s);
hipError_t launch_widen_diag(const void *d_diag, int diag_type, uint64_t dim, void *d_out, hipStream_t s);
hipError_t launch_probabilities(const void *psi, bool c128, uint64_t dim, double *out, hipStream_t s);
hipError_t launch_topk(const void *psi, bool c128, uint64_t dim, int k, const void *diag, int diag_type,
                       uint64_t *d_idx, double *d_prob, double *d_cost, void *scratch, int nblocks,
                       hipStream_t s);
hipError_t launch_local_tables(int n, int diag_type, const PartDesc *d_pd, const double *d_ell,
                               const int32_t *d_ell_i, int npairs, const int32_t *d_pair_ij, const double *d_pair_b,
                               const int32_t *d_pair_bi, const int32_t *d_qpu, double c0, int32_t c0_i, void *d_tables,
                               uint64_t total, hipStream_t s);

// Specialised complex64 pass kernels (qq_fast.hip): one kernel per pass kind.
enum FastPassKind : int { FK_FIRST = 0, FK_MID, FK_TURN, FK_LAST, FK_LASTG, FK_BMID, FK_BTURN, FK_BLAST, FK_SINGLE };
struct FastPassParams {
    int blocked;  // tile order: 0 strided (tiles g, g + G, ...), 1 blocked (contiguous range per workgroup)
    int part;  // 1: the phase is the product of the per-QPU local factors and the cross factor
    const PartDesc *part_desc;  // device
    const void *part_tables;
    int B, G, p, k;
    uint64_t tiles, dim_mask;
    int pos4, pos8, w1, w2, active, store_psi;
    int slot_base, slot_stride;
    double amp0;
    const double *params;
    const void *diag;
    void *psi;
    void *lam;
    uint64_t state_stride;
    double *partial;
    // device [16]: sums of the couplings among the register qubits of the layout in which the pass
    // reads the diagonal (regq of the problem at that layout's register run)
    const double *cq;
    // partitioned phases: the same sums per factor, [factor (local QPUs, then cross)][run start][16]
    const double *part_cq;
    int part_cq_runs;
    double shift;  // centre of the cost for the accumulations (the mean of C)
    // per-tile cost table of the layout in which the pass reads the cost ([tiles][kCostRow]) and the
    // per-thread constants ([256][8]) that follow it; required by every non-partitioned pass kind that
    // reads the cost
    const double *ctab;
    const double *cthr;
    // the same for the cross-QPU couplings alone; required by the partitioned phases
    const double *xtab;
    const double *xthr;
    int ilv;  // 0, or K: psi and lambda in alternating blocks of 2^K amplitudes (see Layout::ilv)
};
hipError_t launch_fast_pass(int kind, bool high, int diag_type, const FastPassParams &pp, hipStream_t s);

// Per-tile cost table of one tile geometry and layout (qq_kernels.hip).  A tile's 4096 states are
// z = T + E + R: T its base bits, E the thread's bits (qubits 0..3 and the two lane qubits at lane_q:
// the lane l = t & 63; the two wave qubits at lane_q + 2: the wave w = t >> 6), R the register bits
// (the four qubits at reg_q).  Row r of tile r (kCostRow doubles):
//   [l]      C(T) + sum over the lane bits q of l of G_q(T)     (l = 0..63)
//   [64 + w] sum over the wave bits q of w of G_q(T)            (w = 0..3)
//   [68 + j] G_{reg_q + j}(T)                                    (j = 0..3)
// with G_q(T) = sum_{i in T} b_iq and C(T) the cost of the base bits alone (c0 included).
// high: tile bases as in the strided high tiles (tile_base with pos4, pos8), else tile << 12.
constexpr int kCostRow = 72;
hipError_t launch_cost_table(int n, int high, int pos4, int pos8, int lane_q, int reg_q, uint64_t tiles,
                             const double *d_ell, int npairs, const int32_t *d_pair_ij, const double *d_pair_b,
                             double c0, double *out, hipStream_t s);

// Device address of the fixed scratch array (QQ_STATIC_SCRATCH_BYTES) on `device`, taken once per
// device with hipGetSymbolAddress (qq_static.hip).
hipError_t static_scratch(int device, void **ptr);

// Persistent launch over many problems (qq_many.hip).
// Work item = (problem, state b, pass j, chunk c): tiles [c * tpc, min((c + 1) * tpc, tiles))
// of pass j.  Items are numbered so that a state's pass j precedes its pass j + 1 (by
// the fraction of the problem's pass chain done, see plan_many) and taken in that order
// from one atomic ticket counter, so an item only ever waits for items with smaller tickets.
struct ManyInst {
    int n, p, B;
    int npasses, pass_off;  // passes in ManyPass[pass_off ..]
    int nchunks, tpc;
    int nslots, slot_off;   // accumulator slots; their output indices in slot_out[slot_off ..]
    int state0;             // counter index of state 0
    uint64_t tiles, dim_mask;
    uint64_t partial_off;   // doubles, laid out [slot][b][chunk]
    double amp0, escale;
    double shift;           // centre of the cost for the accumulations of the pass bodies (multi-pass)
    const double *params;   // device [B][2p]
    const void *diag;
    const double *regq;     // device [n - 3][16]: register-run coupling sums (see qq_problem::regq)
    void *psi, *lam;        // device [B][2^n] complex64 (multi-pass problems), complex128 (every problem)
    double *energy_out;     // device [B], or NULL: results go to out_ws
    double *grad_out;       // device [B][2p] (with energy_out)
    double *out_ws;         // device [B][1 + 2p]
};
struct ManyPass {
    int kind, k, geom;      // geom 0: qubits 0..11; 1: high set, all 8 bits active; 2: high set, partial
                            // (complex128 launch: kind -1, geom = states the general pass keeps, 1 or 2)
    int pos4, pos8, w1, w2, active, nact, store_psi;
    int slot_base, nslots;  // first accumulator slot of the pass inside its problem
    const double *ctab;     // the cost table of the pass's layout and its per-thread constants
    const double *cthr;
};
struct ManySeg {
    uint32_t first;  // ticket of chunk 0
    uint32_t inst, b, pass;
};
struct ManyArgs {
    const ManyInst *inst;
    const ManyPass *pass;
    const PassArgs *gpass;  // complex128 launch: the general pass of each ManyPass (same index), else NULL
    const ManySeg *seg;
    const uint16_t *slot_out;
    int nseg;
    int grad;
    uint32_t total;       // tickets
    uint32_t *ctl;        // [0] ticket head, [1] error flag, [2 + s] items completed for state s
    double *partial;
    uint64_t spin_ticks;  // bound on one dependency wait, in wall-clock ticks
};
hipError_t launch_many(const ManyArgs &a, bool c128, int diag_type, int max_grid, hipStream_t s, int *grid_out);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);

// Device Adam step (qq_optim.hip).
struct AdamArgs {
    int B, p;
    double lr, beta1, beta2, eps;
    const double *result;  // [B][1 + 2p]: energy, then the interleaved gradient
    double *x;             // [B][2p] parameters, updated in place
    double *m, *v;         // [B][2p] moments
    int *step;             // completed steps (device)
    double *energy_out;    // [B] energy of the step (at the parameters before the update)
    double *grad_out;      // [B][2p] gradient of the step, or NULL
    double *history;       // [history_len][B] energies by step (ring), or NULL
    int history_len;
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);

// Shots from the exact distribution (qq_sample.hip).
hipError_t launch_block_mass(const void *psi, bool c128, uint64_t dim, uint64_t nblk, double *mass, hipStream_t s);
hipError_t launch_shots(const void *psi, bool c128, uint64_t dim, uint64_t nblk, const double *start,
                        uint64_t last_blk, const double *u, int64_t shots, uint64_t *out, hipStream_t s);
hipError_t launch_gather_cost(const void *diag, int diag_type, const uint64_t *idx, int64_t count, double *out,
                              hipStream_t s);

// Gate-level TeleGate trajectory (qq_telegate.hip), complex128 over n + 2 qubits.  tg_launch_pair
// kinds: 0 CNOT(c -> t), 1 H(t), 2 RX(2 beta)(t) with (cos, sin), 3 X(t) if outcome[slot],
// 4 Z(t) if outcome[slot].
hipError_t tg_launch_init(double2 *psi, int n, hipStream_t s);
hipError_t tg_launch_local_phase(double2 *psi, int n, const void *diag, const void *cross, int diag_type, double gamma,
                                 hipStream_t s);
hipError_t tg_launch_phase1(double2 *psi, int nq, int q, double phi, hipStream_t s);
hipError_t tg_launch_pair(double2 *psi, int nq, int t, int kind, int c, double cb, double sb, const int *outcome,
                          int slot, hipStream_t s);
hipError_t tg_launch_measure(double2 *psi, int nq, int q, double u, double *partial, int nblocks, int *outcome,
                             double *scale, int slot, hipStream_t s);
hipError_t tg_launch_sign(double2 *psi, int nq, const int *outcome, int slot, hipStream_t s);

// Host helpers shared with the driver (qq_api.cpp): record the thread's error message; the
// device a problem lives on.
qq_status set_error(qq_status st, const char *msg);
int problem_device(const qq_problem *pb);

// Plain complex128 per-gate path (qq_plain.hip).
struct PlainArgs {
    int n;
    int p;
    int grad;
    uint64_t dim;
    const double *params;  // host [2p]
    const void *diag;
    int diag_type;
    void *psi;   // device complex128 [dim]
    void *lam;   // device complex128 [dim] (grad only)
    double *partial;  // device scratch [nblocks]
    double *result;   // device scratch [1 + 2p]
    int nblocks;
};
hipError_t run_plain(const PlainArgs &a, hipStream_t s);

}  // namespace qq
