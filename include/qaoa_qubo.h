/*
 * qaoa_qubo.h -- C ABI of the MI355X (gfx950) exact QAOA-for-QUBO statevector engine.
 *
 * The engine evaluates, exactly and without shot sampling, the p-layer QAOA
 * training objective of the paper "A Distributed Quantum Approximate
 * Optimization Algorithm Simulator for Engineering Design Optimization":
 *
 *   input form        F(z) = c0 + f^T z + z^T H z                       eq. (2)
 *   canonical form    l_i = f_i + H_ii,  b_ij = H_ij + H_ji (i < j)      eq. (4)-(6)
 *   cost unitary      U_C(gamma) = exp(-i gamma H_C), H_C|z> = F(z)|z>   eq. (8), (10)
 *   mixer             U_M(beta) = exp(-i beta sum_q X_q) = prod_q RX_q(2 beta)   eq. (12)-(13)
 *   state             U_M(b_p)U_C(g_p)...U_M(b_1)U_C(g_1)|+>^n           eq. (11)
 *   objective         J(x) = sum_z P_x(z) F(z)                           eq. (15), (17)
 *   parameters        x = [gamma_1, beta_1, ..., gamma_p, beta_p]        (training-objective section)
 *   local/cross rule  coupling b_ij is local iff q(i) = q(j)             eq. (16)
 *
 * Conventions: variable z_i (i = 1..n) is qubit i-1 = bit (i-1) of a basis
 * index; a printed logical bitstring is z_1 ... z_n (the decoding section's
 * reversal of the little-endian display).  Gradients are returned in the
 * same interleaved layout as x.
 *
 * General rules for every call:
 *  - Every call returns a qq_status and never throws.  On error nothing is
 *    written to the outputs and qq_last_error() describes the cause.
 *  - The caller owns every array it passes.  qq_problem_create copies H and f.
 *  - Host arrays are plain C arrays.  Device arrays (selected by the
 *    QQ_PARAMS_ON_DEVICE / QQ_OUT_ON_DEVICE flags, or documented as device
 *    pointers) must live on the problem's device.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls that write
 *    host outputs synchronise that stream before returning; calls whose
 *    outputs are on the device are asynchronous on it.
 *  - Input validation (sizes, finiteness, allocation rules) runs on the host
 *    before any device work.
 */
#ifndef QAOA_QUBO_H
#define QAOA_QUBO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QQ_OK = 0,
    QQ_E_INVALID = -1,      /* bad argument: size, pointer, non-finite value, unknown flag */
    QQ_E_ALLOCATION = -2,   /* variable-to-QPU allocation violates the validation rules */
    QQ_E_TOO_LARGE = -3,    /* the request cannot fit in device memory (decided before allocating) */
    QQ_E_WORKSPACE = -4,    /* caller workspace smaller than qq_workspace_size() */
    QQ_E_DEVICE = -5,       /* a HIP runtime call failed (message carries the HIP error string) */
    QQ_E_NOMEM = -6,        /* a device or host allocation failed */
    QQ_E_UNSUPPORTED = -7   /* valid request the library does not support (message says which) */
} qq_status;

/* Flags for the evaluation calls (bitwise OR). */
enum {
    QQ_ENERGY = 1,            /* compute J(x) */
    QQ_GRAD = 2,              /* also compute dJ/dx by the adjoint sweep (implies QQ_ENERGY) */
    QQ_PARTITIONED = 4,       /* apply the cost layer as per-QPU local phases then the cross phase */
    QQ_C128 = 8,              /* complex128 state (default complex64) */
    QQ_PARAMS_ON_DEVICE = 16, /* params pointer is device memory */
    QQ_OUT_ON_DEVICE = 32     /* output pointers are device memory (no synchronisation) */
};

#define QQ_MAX_N 34
#define QQ_MAX_P 64
#define QQ_MAX_QPUS 16
#define QQ_MAX_TOPK 16

typedef struct qq_problem qq_problem; /* opaque handle */

typedef struct {
    int n;                    /* number of binary variables = qubits */
    int is_integer;           /* 1: C(z) is exact integer arithmetic (H, f, c0 integral, sum of |coefficients| < 2^31) */
    int diag_bytes;           /* bytes per stored diagonal entry: 2 or 4 (integer), 8 (FP64) */
    int num_qpus;             /* 0 when no allocation is set */
    double c0;                /* constant term of eq. (2) */
    double alpha;             /* identity coefficient of eq. (9) = mean of C over all z */
    double sigma_c;           /* sqrt(sum h_i^2 + sum J_ij^2) = standard deviation of C over all z */
    double cmin, cmax;        /* min / max of C(z) over all z */
    uint64_t argmin_index;    /* lowest basis index attaining cmin (the brute-force optimum) */
    int64_t nonzero_couplings;/* number of b_ij != 0, i < j */
    int64_t cross_terms;      /* number of cross-QPU couplings (eq. (16)), -1 without an allocation */
} qq_info;

/* Thread-local description of the last error on this thread; valid until the next qq_* call. */
const char *qq_last_error(void);

/* ABI version of this header (increments on incompatible changes). */
int qq_abi_version(void);

/* Number of visible HIP devices (0 without a GPU). */
qq_status qq_device_count(int *count);

/*
 * Create a problem from the dense input form of eq. (2).
 *   n       number of variables, 1 <= n <= QQ_MAX_N
 *   H       n*n row-major host array (any, not necessarily symmetric); copied
 *   f       n host array or NULL (= 0); copied
 *   c0      constant term
 *   device  HIP device ordinal
 * The handle canonicalises (eq. (4)-(5)), classifies the problem as integer
 * or real, and builds the cost diagonal C(z) of eq. (6) on the device once
 * (the "build once, bind many" reuse of the circuit-reuse section).  For
 * n > 12 it also builds the per-tile cost tables that the complex64
 * evaluation kernels read instead of the diagonal (C is quadratic, so a
 * tile's 4096 values follow from its base bits): 576 bytes per 4096 states
 * for each set layout, about 0.53 GB in all at n = 28 (2^28 states).
 * Errors: QQ_E_INVALID (n out of range, NULL H/out, non-finite entry),
 * QQ_E_TOO_LARGE (the diagonal and its tables do not fit the device),
 * QQ_E_DEVICE, QQ_E_NOMEM.
 */
qq_status qq_problem_create(int n, const double *H, const double *f, double c0, int device, void *stream,
                            qq_problem **out);

qq_status qq_problem_destroy(qq_problem *prob);

/* Summary of the problem (see qq_info).  Host call; no device work. */
qq_status qq_problem_info(const qq_problem *prob, qq_info *out);

/*
 * Canonical coefficients (eq. (4)-(5)) and the Pauli coefficients of eq. (9):
 *   ell[n], b[n*n] (row-major, strict upper triangle set, rest 0),
 *   alpha, h[n], J[n*n] (strict upper triangle), each may be NULL.
 * alpha = c0 + sum l/2 + sum b/4;  h_i = -l_i/2 - sum_{j != i} b_ij/4;  J_ij = b_ij/4.
 */
qq_status qq_coefficients(const qq_problem *prob, double *ell, double *b, double *alpha, double *h, double *J);

/*
 * Copy the cost diagonal C(z), z = 0..2^n-1 (eq. (6)), to `out`:
 * int32 entries for integer problems (info.is_integer), double otherwise.
 * For real problems every entry is c0 + l_i (ascending i) + b_ij (row-major)
 * summed in FP64 in exactly that order over the set bits of z.
 * flags: QQ_OUT_ON_DEVICE selects a device `out`.
 */
qq_status qq_cost_diagonal(const qq_problem *prob, void *out, int flags, void *stream);

/*
 * Attach a variable-to-QPU allocation (allocation section; eq. (16)).
 *   num_qpus      M, 1 <= M <= QQ_MAX_QPUS
 *   qpu_of_var    n host ints in [0, M): variable i+1 sits on QPU qpu_of_var[i]
 *   capacities    M host ints or NULL (no capacity limit)
 * Validation: every entry in range, no QPU over capacity, every QPU used.
 * Builds, on the device, the per-QPU local cost tables (each indexed by the
 * QPU's own variables; c0 goes to QPU 0) and the cross-QPU diagonal used by
 * QQ_PARTITIONED evaluations.  Outputs (each may be NULL): the number of
 * cross-QPU couplings (nonzero b_ij with q(i) != q(j)) and the per-layer
 * remote-CNOT estimate 2 * cross (multiply by p for a whole circuit).
 * Errors: QQ_E_INVALID, QQ_E_ALLOCATION, QQ_E_DEVICE, QQ_E_NOMEM.
 */
qq_status qq_set_allocation(qq_problem *prob, int num_qpus, const int32_t *qpu_of_var, const int32_t *capacities,
                            int64_t *cross_terms_out, int64_t *remote_cx_per_layer_out);

/* Device bytes qq_evaluate needs for (p, batch, flags). */
qq_status qq_workspace_size(const qq_problem *prob, int p, int batch, int flags, size_t *bytes);

/*
 * Exact J(x) (eq. (17)) and, with QQ_GRAD, dJ/dx for `batch` parameter sets.
 *   params      batch x 2p doubles, interleaved [g1, b1, ..., gp, bp] per set
 *   workspace   device buffer of ws_bytes >= qq_workspace_size(), or NULL to
 *               let the library allocate (and free) one for this call
 *   energy_out  batch doubles
 *   grad_out    batch x 2p doubles (required with QQ_GRAD, else ignored; may be NULL)
 * The state is complex64 unless QQ_C128; the cost diagonal, the phase
 * argument reduction and every energy/gradient accumulator are FP64.
 * Deterministic: identical inputs give bit-identical outputs.
 * Errors: QQ_E_INVALID (p, batch, non-finite params, missing outputs),
 * QQ_E_ALLOCATION (QQ_PARTITIONED without an allocation), QQ_E_WORKSPACE,
 * QQ_E_TOO_LARGE, QQ_E_DEVICE.
 */
qq_status qq_evaluate(qq_problem *prob, int p, int batch, const double *params, int flags, void *workspace,
                      size_t ws_bytes, void *stream, double *energy_out, double *grad_out);

/*
 * The final state |gamma, beta> of eq. (11) for one parameter set (2p doubles).
 * psi_out: 2^n complex64 (interleaved float re, im) or, with QQ_C128,
 * complex128; host memory unless QQ_OUT_ON_DEVICE.
 */
qq_status qq_state(qq_problem *prob, int p, const double *params, int flags, void *psi_out, void *stream);

/* Measurement distribution P_x(z) = |<z|gamma,beta>|^2 (eq. (15)) as 2^n doubles. */
qq_status qq_probabilities(qq_problem *prob, int p, const double *params, int flags, double *prob_out,
                           void *stream);

/*
 * The k most probable bitstrings (the elite top-k of the metrics section),
 * ordered by decreasing probability, ties to the lower basis index.
 *   k <= QQ_MAX_TOPK; idx_out/prob_out/cost_out: k entries each (cost_out may be NULL).
 */
qq_status qq_topk(qq_problem *prob, int p, const double *params, int flags, int k, uint64_t *idx_out,
                  double *prob_out, double *cost_out, void *stream);

/*
 * Many problems of uneven n and p in one persistent launch (runtime
 * optimisation section, throughput subsection: independent evaluations run
 * together instead of one request each).
 *
 * Problem i evaluates batch[i] parameter sets of depth p[i] (params[i]:
 * batch[i] x 2p[i] interleaved doubles, host memory unless
 * QQ_PARAMS_ON_DEVICE) into energy_out[i] (batch[i] doubles) and, with
 * QQ_GRAD, grad_out[i] (batch[i] x 2p[i]); host memory unless
 * QQ_OUT_ON_DEVICE.  Same results as qq_evaluate on each problem, up to the
 * order of the FP64 partial sums (complex64 state, or complex128 with
 * QQ_C128; FP64 diagonal, phase reduction and accumulators).
 *
 * Execution: one launch per cost-diagonal element type present (at most
 * three) drains a queue of (problem, parameter set, pass, tile chunk) items
 * from an atomic ticket, ordered by the fraction (j + 1) / L of its problem's
 * chain of L passes that pass j completes; a problem with n <= 12 is one item
 * per parameter set.  With QQ_C128 the items run the general complex128 pass
 * bodies of qq_evaluate (every problem by tile chunks; for n <= 12 one item of
 * one tile).  Items of a pass wait, bounded in time, for the previous
 * pass on the same state; a wait longer than opt->wait_limit_ms sets a device
 * flag, the launch drains early and the call returns QQ_E_DEVICE.  The call
 * synchronises the stream before returning (it reads that flag).
 *
 * Limits: every problem on one device, n <= 31, 1 <= p <= QQ_MAX_P,
 * batch >= 1.  QQ_PARTITIONED is not served here (QQ_E_UNSUPPORTED; use
 * qq_evaluate).
 * workspace: device buffer of ws_bytes >= qq_workspace_size_many(), or NULL
 * to let the library allocate one for this call.  opt may be NULL (defaults).
 * Errors: QQ_E_INVALID, QQ_E_UNSUPPORTED, QQ_E_WORKSPACE, QQ_E_TOO_LARGE,
 * QQ_E_NOMEM, QQ_E_DEVICE.
 */
typedef struct {
    int tiles_per_chunk;   /* tiles (4096 amplitudes) per work item of a multi-pass problem; 0: 24 (QQ_C128: 8) */
    int max_workgroups;    /* cap on the persistent grid; 0: every workgroup that fits on the device at once */
    double wait_limit_ms;  /* bound on one dependency wait; 0: 2000 ms */
} qq_many_options;

qq_status qq_workspace_size_many(int count, qq_problem *const *problems, const int *p, const int *batch, int flags,
                                 const qq_many_options *opt, size_t *bytes);

qq_status qq_evaluate_many(int count, qq_problem *const *problems, const int *p, const int *batch,
                           const double *const *params, int flags, const qq_many_options *opt, void *workspace,
                           size_t ws_bytes, void *stream, double *const *energy_out, double *const *grad_out);

/*
 * qq_evaluate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments, flags, outputs and errors as qq_evaluate, with
 * the workspace taken from a fixed device array of QQ_STATIC_SCRATCH_BYTES
 * owned by the library instead of a caller buffer.  The call performs no
 * device allocation or free.  Each GPU the library runs on holds its own copy
 * of the array from the first such call on it until the process ends.
 *   Limit: requests whose workspace (qq_workspace_size) exceeds
 *   QQ_STATIC_SCRATCH_BYTES are rejected with QQ_E_WORKSPACE before any device
 *   work (complex64: n = 20 holds up to 7 parameter sets with gradients,
 *   n = 21 three, n = 22 one).
 *   Every call on a GPU shares that GPU's array, which keeps the last call's
 *   contents: calls that overlap on one GPU (other streams or threads) race
 *   and must be serialised by the caller.  Nothing in the array needs to start
 *   at zero: every byte a call reads there was written earlier in that call.
 *   Per-launch profiling (qq_profile_enable) records nothing for these calls.
 */
#define QQ_STATIC_SCRATCH_BYTES (128u << 20)

qq_status qq_evaluate_static(qq_problem *prob, int p, int batch, const double *params, int flags, void *stream,
                             double *energy_out, double *grad_out);

/*
 * Evaluation with every gradient held to a relative tolerance (the error
 * against exact arithmetic stated per result).  Same objective and gradient
 * as qq_evaluate / qq_evaluate_many (eq. (17), adjoint derivatives in the
 * layout of x).
 *
 * Complex64 states carry rounding errors that do not shrink with the
 * gradient: on a parameter set where dJ/dx is small next to the spread of
 * C (sigma_C, eq. (9)), ||dg||_inf / ||g||_inf can exceed any fixed
 * tolerance.  These calls first evaluate in complex64, then bound each
 * set's gradient error by the complex64 error model
 *     ||dg||_inf <= QQ_GUARD_REL * ||g||_inf
 *                   + QQ_GUARD_K * 2^-24 * sigma_C^2 * 2^(-n/2)
 * (a relative part from coefficient and phase roundings, and the random
 * part of the rounding of 2^n stored amplitudes in the gamma-derivative
 * sums, each term of which carries (C - alpha)^2), and recompute with
 * complex128 states every set whose bound exceeds tol * ||g||_inf.  The
 * constants come from measurements against the FP64 oracle (the uneven
 * batch of 512 problems, n = 10..22, p = 1..6) and the complex128 path
 * (n = 28, p = 8, 64 sets; n = 32), with margin over the largest ratio seen.
 * Energies need no recomputation: their complex64 error stays below about
 * 1e-6 of max(|J|, sigma_C).
 *
 *   tol           relative gradient tolerance; 0 selects 1e-5
 *   flags         QQ_ENERGY / QQ_GRAD / QQ_PARTITIONED / QQ_C128 (host
 *                 params and outputs only; without QQ_GRAD nothing is
 *                 recomputed; with QQ_C128 every set is complex128)
 *   c128_out      batch int32 (may be NULL): 1 where the returned result was
 *                 computed with complex128 states
 *   grad_err_out  batch doubles (may be NULL): the bound on ||dg||_inf of
 *                 the returned gradient (complex64 sets: the model above;
 *                 complex128 sets: 1e-10 * ||g||_inf); 0 without QQ_GRAD
 * The library allocates the workspaces of both passes for the call.
 * Errors: those of qq_evaluate (qq_evaluate_many), and QQ_E_UNSUPPORTED for
 * QQ_PARAMS_ON_DEVICE / QQ_OUT_ON_DEVICE.
 */
#define QQ_GUARD_REL 4e-6
#define QQ_GUARD_K 40.0

qq_status qq_evaluate_guarded(qq_problem *prob, int p, int batch, const double *params, int flags, double tol,
                              void *stream, double *energy_out, double *grad_out, int32_t *c128_out,
                              double *grad_err_out);

/* The same for many problems: complex64 through one persistent launch (qq_evaluate_many), then the
 * sets whose bound exceeds the tolerance through a second one with complex128 states (QQ_C128), or
 * through the per-pass complex128 kernels when they all belong to one problem.
 * c128_out[i] and grad_err_out[i] (each array may be NULL, or hold NULL entries) have batch[i]
 * entries.  QQ_C128 and QQ_PARTITIONED are not accepted (QQ_E_UNSUPPORTED). */
qq_status qq_evaluate_many_guarded(int count, qq_problem *const *problems, const int *p, const int *batch,
                                   const double *const *params, int flags, const qq_many_options *opt, double tol,
                                   void *stream, double *const *energy_out, double *const *grad_out,
                                   int32_t *const *c128_out, double *const *grad_err_out);

/*
 * Schedules and the autotuner (circuit-reuse section: work prepared once per
 * problem and settings and reused; here the launch schedule).
 *
 * A schedule fixes, for one (p, batch, flags) of a problem:
 *   workgroups_per_state  G: workgroups that share one state in every pass
 *                         (power of two, 1 <= G <= 2^(n-12)); default
 *                         min(2^(n-12), 4096 / batch) rounded down to a power of two
 *   set_pairing           which 4-qubit runs above qubit 11 share a high pass when
 *                         n - 12 is a multiple of 8 with at least four runs
 *                         (0: run i with run m-1-i, 1: adjacent runs, 2: run i with
 *                         run i + m/2); otherwise only 0
 *   set_order             where the qubit-0..11 set sits in the order in which a
 *                         layer visits the sets (the zig-zag reverses it every
 *                         layer, so the first and last sets are where a pass
 *                         applies the phase between two mixers): 0 first, 1 second
 *                         (needs three or more sets, i.e. n >= 21); default 1
 *                         where it applies, else 0
 * Results do not depend on workgroups_per_state and tile_order beyond the order of
 * FP64 partial sums; set_pairing and set_order change the order of the complex64
 * operations (differences at the complex64 rounding level).
 * qq_set_schedule pins one (NULL restores the default); qq_get_schedule reports
 * the one in force.  qq_workspace_size, qq_evaluate and qq_graph_create use it.
 *
 * qq_autotune times every candidate with HIP events on seeded parameter sets
 * (one warm-up, then the median of three runs, or one run when the warm-up
 * took over 200 ms): G of the default, half and double it, times
 * every pairing that applies, in the strided tile order and the default set
 * order; then the blocked tile order at the best pairing for the best G, half and
 * double it; then the other set order, where one applies, at the best of those.  It pins the
 * fastest and, if cache_path is not
 * NULL, appends it to that JSON-lines file; an entry already there for the same
 * device, n, p, batch, planning flags and diagonal width is used without timing.
 * qq_autotune_many does the same for qq_evaluate_many over tiles_per_chunk in
 * {4, 8, 16, 24, 32, 48, 64} and max_workgroups in {0, 2 x compute units}, keyed by a
 * hash of every problem's (n, p, batch, diagonal width); it returns the options
 * (to pass to qq_evaluate_many) and the measured time in ms_out (may be NULL).
 * Both allocate their own device memory and synchronise `stream`.
 */
typedef struct {
    int workgroups_per_state;
    int set_pairing;
    double ms;        /* timed duration of one evaluation (autotune), else as pinned */
    int pinned;       /* 1 when a schedule is pinned for the key */
    int from_cache;   /* 1 when qq_autotune read it from the cache file */
    int tried;        /* candidates timed by qq_autotune */
    int tile_order;   /* 0: workgroup g takes tiles g, g + G, ... (neighbouring tiles run together);
                         1: workgroup g takes a contiguous range of tiles (specialised kernels only) */
    int set_order;    /* 0: the qubit-0..11 set first in a layer's visiting order; 1: second */
} qq_schedule;

qq_status qq_set_schedule(qq_problem *prob, int p, int batch, int flags, const qq_schedule *schedule);
qq_status qq_get_schedule(const qq_problem *prob, int p, int batch, int flags, qq_schedule *out);
qq_status qq_autotune(qq_problem *prob, int p, int batch, int flags, const char *cache_path, void *stream,
                      qq_schedule *out);
qq_status qq_autotune_many(int count, qq_problem *const *problems, const int *p, const int *batch, int flags,
                           const char *cache_path, void *stream, qq_many_options *out, double *ms_out);

/*
 * Optimisation steps [energy + gradient -> Adam] captured once in a HIP graph
 * and replayed (optimisation-overhead section: Adam with a cheaper gradient,
 * here the exact adjoint one; throughput subsection: parallel multi-start runs,
 * here `batch` starts stepping together).
 *
 * qq_graph_create captures one step for `batch` starts of depth p:
 *   params   device [batch][2p] doubles, interleaved like qq_evaluate's; the
 *            caller owns them, every step updates them in place
 *   adam     4 host doubles {lr, beta1, beta2, eps}, or NULL for
 *            {0.01, 0.9, 0.999, 1e-8}; per parameter, with t the step number:
 *            m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *            x -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 *   history  number of past steps whose energies are kept (ring buffer), or 0
 *   flags    QQ_C128 / QQ_PARTITIONED as for qq_evaluate (QQ_GRAD is implied;
 *            no *_ON_DEVICE flags)
 * The handle owns the evaluation workspace, the Adam moments, the step counter
 * and the last step's energies and gradients (all device memory, allocated here
 * once).  The step counter and moments start at zero.  The problem handle and
 * params must outlive the graph: qq_problem_destroy and qq_set_allocation on
 * the problem return QQ_E_INVALID while a graph captured on it exists.
 * qq_graph_run       replays the captured step `steps` times on `stream`
 *                    (asynchronous; no allocation, no host work per step).
 * qq_graph_step_eager launches the same kernels directly (one step).
 * qq_graph_reset     zeroes the moments and the step counter (kernels on `stream`).
 * qq_graph_read      copies the last step's energies (batch; taken at the
 *                    parameters before that step's update) and gradients
 *                    (batch x 2p), the energy history (history x batch, entry
 *                    (t-1) mod history holds step t) and the number of steps
 *                    taken; any output may be NULL; host memory unless
 *                    QQ_OUT_ON_DEVICE (steps is always host); synchronises `stream`.
 * Errors: QQ_E_INVALID, QQ_E_ALLOCATION, QQ_E_UNSUPPORTED, QQ_E_TOO_LARGE,
 * QQ_E_NOMEM, QQ_E_DEVICE.
 */
typedef struct qq_graph qq_graph;

qq_status qq_graph_create(qq_problem *prob, int p, int batch, int flags, const double *adam, double *params,
                          int history, void *stream, qq_graph **out);
qq_status qq_graph_run(qq_graph *graph, int steps, void *stream);
qq_status qq_graph_step_eager(qq_graph *graph, void *stream);
qq_status qq_graph_reset(qq_graph *graph, void *stream);
qq_status qq_graph_read(qq_graph *graph, double *energy, double *grad, double *history, int *steps, int flags,
                        void *stream);
qq_status qq_graph_destroy(qq_graph *graph);

/*
 * Gate-level trajectory of the distributed circuit with explicit TeleGate remote
 * CNOTs (distributed circuit construction section): n data qubits plus two
 * communication qubits, complex128, for the allocation set by
 * qq_set_allocation.  Per layer: the phase of every QPU-local term (C minus the
 * cross couplings, eq. (16)); each cross coupling b z_i z_j (i < j, row-major)
 * as phases exp(-i gamma b / 2) on z_i = 1 and on z_j = 1 and the parity phase
 * CNOT(i -> j) diag_j(1, e^{+i gamma b / 2}) CNOT(i -> j) with both CNOTs remote;
 * then RX(2 beta) on every data qubit.  A remote CNOT entangles the
 * communication pair, couples and measures one member on each QPU, corrects the
 * data qubits (X on the target, Z on the control, conditioned on the outcomes)
 * and resets the pair; the remaining global phase (-1)^(m1 m2) is removed, so
 * every trajectory's data state equals the exact state of qq_state (complex128).
 *   params        host [2p]
 *   uniforms      host doubles in [0, 1), two per remote CNOT in circuit order
 *                 (4 x cross x p); a measurement gives 1 when its uniform is
 *                 below the probability of 1
 *   psi_out       2^n complex128, host (device with QQ_OUT_ON_DEVICE)
 *   outcomes_out  host int32 [2 x remote] measurement outcomes, or NULL
 *   remote_out    remote CNOTs of the circuit, 2 x cross x p, or NULL
 * n <= 26.  Errors: QQ_E_INVALID, QQ_E_ALLOCATION (no allocation),
 * QQ_E_TOO_LARGE, QQ_E_NOMEM, QQ_E_DEVICE.
 */
qq_status qq_telegate_state(qq_problem *prob, int p, const double *params, const double *uniforms, int flags,
                            void *psi_out, int32_t *outcomes_out, int64_t *remote_out, void *stream);

/*
 * Variable-to-QPU allocation (multi-QPU variable allocation section, Fig. 1).
 * Host-only functions of the dense input form (H as for qq_problem_create, n x n
 * row-major host array); they need no device and feed qq_set_allocation.
 *   qq_balanced_capacities  c_m = floor(n / M) + [m < n mod M] (the paper's
 *                           "as evenly as possible"; 1 <= M <= n)
 *   qq_allocation           one strategy: QQ_ALLOC_CONTIGUOUS fills QPU 0, 1, ...
 *                           with variables in order up to their capacities;
 *                           QQ_ALLOC_GRAPH is a greedy on the weighted coupling
 *                           graph w_ij = |H_ij + H_ji| (the paper names the step
 *                           but not its rule): QPUs are filled in turn, each
 *                           from the unassigned variable of largest strength
 *                           s(v) = sum_u w_uv, then by largest gain
 *                           2 w(v, QPU) - s(v), ties to the lower index.  Every
 *                           QPU keeps room for one variable per later QPU.
 *                           capacities: M host ints >= 1 summing to >= n, or
 *                           NULL for the balanced ones.  qpu_out: n ints (0-based
 *                           QPU of each variable); cross_out (may be NULL): the
 *                           number of nonzero couplings across QPUs (eq. (16)).
 *   qq_allocation_candidates  the graph-aware, the contiguous and (if manual is
 *                           not NULL) the given allocation, in that order, with
 *                           their cross counts and remote-CNOT estimates
 *                           2 x cross x p (remote_out may be NULL); best = the
 *                           candidate with the fewest cross terms, ties to the
 *                           earlier one in that order (the paper's fixed type
 *                           priority is not given; this order is the reading).
 *                           qpu_out: 3 x n ints, count = 2 or 3.
 * Errors: QQ_E_INVALID.
 */
#define QQ_ALLOC_CONTIGUOUS 0
#define QQ_ALLOC_GRAPH 1

qq_status qq_balanced_capacities(int n, int num_qpus, int *capacities_out);
qq_status qq_allocation(int n, const double *H, int num_qpus, const int *capacities, int strategy, int32_t *qpu_out,
                        int64_t *cross_out);
qq_status qq_allocation_candidates(int n, const double *H, int num_qpus, const int *capacities,
                                   const int32_t *manual, int p, int32_t *qpu_out, int64_t *cross_out,
                                   int64_t *remote_out, int *count, int *best);

/*
 * Shots from the exact output distribution (computational-basis measurement;
 * the final shot-based evaluation and the metrics of the measurement decoding
 * section, drawn from the exact state instead of a circuit simulator).
 *
 * qq_sample prepares the depth-p state of one parameter set (params as for
 * qq_state) and draws `shots` basis indices: shot s takes the first index z
 * whose cumulative probability sum_{y <= z} |psi(y)|^2 exceeds
 * uniforms[s] * sum_y |psi(y)|^2 (inverse transform in basis order; sums in
 * FP64; uniforms in [0, 1), drawn by the caller).  flags: QQ_C128,
 * QQ_PARTITIONED; QQ_PARAMS_ON_DEVICE makes params and uniforms device
 * pointers (device uniforms are not range-checked; values outside [0, 1) give
 * the last index of nonzero probability); QQ_OUT_ON_DEVICE makes indices_out a
 * device pointer.  Bit i-1 of an index is variable z_i.  Synchronises `stream`.
 *
 * qq_sample_stats summarises host indices (< 2^n) with the problem's stored
 * costs: best sampled cost; the best sampled bitstring (among those of best
 * cost the most frequent, ties to the lower index) and its frequency; the
 * fraction of shots at the best cost; the sample mean of C (summed over
 * distinct indices in index order); the low-cost mass (fraction of shots with
 * C <= best + margin, margin >= 0 absolute); against the exact optimum of the
 * problem (cmin, argmin_index): whether the best cost and bitstring match it,
 * the fraction of shots at cost cmin and the frequency of argmin_index; and the
 * k most frequent bitstrings (ties to the lower index) with their counts and
 * costs (elite_cost may be NULL; entries beyond the distinct count are zero).
 * Errors: QQ_E_INVALID, QQ_E_NOMEM, QQ_E_DEVICE and those of qq_state.
 */
typedef struct {
    int64_t shots;
    int64_t distinct;              /* distinct sampled indices */
    uint64_t best_index;
    double best_cost;
    double best_frequency;         /* count of best_index / shots */
    double best_cost_mass;         /* shots at best_cost / shots */
    double mean_cost;
    double low_cost_mass;          /* shots with C <= best_cost + margin / shots */
    double exact_cost;             /* cmin of the problem */
    uint64_t exact_index;          /* argmin_index of the problem */
    int matches_exact_cost;
    int matches_exact_index;
    double exact_cost_mass;        /* shots at cost cmin / shots */
    double exact_index_frequency;  /* count of argmin_index / shots */
    int elite;                     /* entries filled in the elite arrays: min(k, distinct) */
} qq_sample_stats_t;

qq_status qq_sample(qq_problem *prob, int p, const double *params, int flags, int64_t shots, const double *uniforms,
                    void *stream, uint64_t *indices_out);
qq_status qq_sample_stats(qq_problem *prob, int64_t shots, const uint64_t *indices, double margin, int k,
                          void *stream, qq_sample_stats_t *out, uint64_t *elite_index, int64_t *elite_count,
                          double *elite_cost);

/*
 * Depth progression with multi-start search (Alg. 1 and the depth-progression /
 * multi-start subsection), on the exact objective: for p = 1 .. p_max, every
 * start runs `iterations` Adam steps of the exact energy with its adjoint
 * gradient (qq_graph_* with all starts of the depth as one batch), the final
 * parameter vector of every start is evaluated once more, the starts are ranked
 * by that energy (ascending; ties to the lower start index) and the best is the
 * depth's representative; the representatives are ranked the same way (ties to
 * the lower depth) and the best is the result.
 *
 * Starts at depth p, in this order: the lifted representative of depth p - 1
 * (p >= 2, if include_warm), perturbed_starts copies of it plus the given
 * offsets (p >= 2), then random_starts given points.  Lifting (the paper does
 * not fix it): linear interpolation of the gamma and beta sequences onto p + 1
 * points, x'_i = ((i - 1) / p) x_{i-1} + ((p - i + 1) / p) x_i for i = 1 .. p + 1
 * with x_0 = x_{p+1} = 0 (the INTERP rule of Zhou et al., Phys. Rev. X 10,
 * 021067 (2020)), applied to gamma and beta separately.
 *
 * Random numbers are inputs:
 *   random_points   host doubles: for p = 1 .. p_max in turn, random_starts
 *                   interleaved [2p] vectors (random_starts * p_max (p_max + 1)
 *                   doubles in all)
 *   perturbations   host doubles: for p = 2 .. p_max in turn, perturbed_starts
 *                   [2p] offsets (perturbed_starts * (p_max (p_max + 1) - 2)
 *                   doubles); may be NULL when perturbed_starts = 0
 * Outputs (host; each may be NULL except result):
 *   result          best depth, its start index, its energy, counts
 *   depth_params    [p_max][2 p_max] representative of every depth, zero padded
 *   depth_energy    [p_max] their energies
 *   start_energy    every start's final energy, depth-major: p = 1 has
 *                   random_starts entries, every later depth
 *                   include_warm + perturbed_starts + random_starts
 * flags: 0, QQ_C128 and/or QQ_PARTITIONED (as for qq_evaluate).  Allocates its
 * own device memory; synchronises `stream`.
 * Errors: QQ_E_INVALID (options, missing inputs, non-finite points or offsets),
 * and those of qq_graph_create and qq_evaluate.
 */
typedef struct {
    int p_max;            /* depths 1 .. p_max, p_max <= QQ_MAX_P */
    int iterations;       /* Adam steps of every start at every depth (>= 0) */
    int random_starts;    /* random points per depth (>= 1) */
    int perturbed_starts; /* perturbed warm starts per depth from depth 2 (>= 0) */
    int include_warm;     /* 1: the lifted representative itself is a start from depth 2 */
    int flags;            /* 0, QQ_C128, QQ_PARTITIONED */
    double adam[4];       /* lr, beta1, beta2, eps (as qq_graph_create) */
} qq_optimize_options;

typedef struct {
    int best_depth;        /* 1 .. p_max */
    int best_start;        /* index of the chosen start at that depth */
    double best_energy;
    long long steps;       /* Adam steps taken, summed over starts */
    long long evaluations; /* energy (+ gradient) evaluations, summed over starts */
} qq_optimize_result;

qq_status qq_optimize(qq_problem *prob, const qq_optimize_options *options, const double *random_points,
                      const double *perturbations, void *stream, qq_optimize_result *result,
                      double *depth_params, double *depth_energy, double *start_energy);

/*
 * Measurement baseline: the plain complex128 form with one kernel per gate
 * (one phase kernel per layer, one RX kernel per qubit and layer, an energy
 * reduction, and the same adjoint equations unfused), one parameter set per
 * call, no batching.  Same outputs as qq_evaluate with batch = 1.
 */
qq_status qq_evaluate_plain(qq_problem *prob, int p, const double *params, int flags, void *stream,
                            double *energy_out, double *grad_out);

/*
 * Per-launch timing of the pass kernels, for measurement tools.
 * qq_profile_enable(1) makes every later evaluation record a pair of HIP
 * events around each kernel launch (on the stream the kernel runs on) plus
 * the launch's algorithmic HBM bytes (state reads/writes and cost-diagonal
 * reads the method needs, counted per state).  qq_profile_read()
 * synchronises those events, copies up to `max` records (oldest first) to
 * `out`, stores the number of records in `count` and clears the log.
 * Profiling is process-wide and off by default; it is not thread-safe.
 */
typedef struct {
    int kind;       /* 1: forward pass (one state), 2: adjoint pass (psi and lambda), 3: final reduction,
                       4: persistent many-problem launch, 5: cost diagonal, 6: min/max of C,
                       7: probabilities, 8: top-k, 9: the whole launch sequence of one qq_evaluate_plain call
                       (bytes 0) */
    int pass_kind;  /* complex64 specialised kernel: 0 first, 1 mid, 2 turn, 3 last, 4 last+adjoint seed,
                       5 adjoint mid, 6 adjoint turn, 7 adjoint last; -1: generic pass kernel */
    int high;       /* 1 when the pass mixes qubits above 11 (strided tile) */
    int full;       /* 1 when every register-group bit of the tile is mixed (compile-time masks) */
    int diag_bytes; /* bytes per cost-diagonal entry the kernel reads */
    int c128;       /* 1 for complex128 state */
    int n;          /* qubits */
    int batch;      /* states in the launch */
    double bytes;   /* algorithmic bytes moved by the launch */
    double ms;      /* event-timed duration */
    int part;       /* 1 when the launch applies partitioned (per-QPU local and cross) phases */
} qq_launch_record;

qq_status qq_profile_enable(int enable);
qq_status qq_profile_read(qq_launch_record *out, int max, int *count);

#ifdef __cplusplus
}
#endif

#endif /* QAOA_QUBO_H */
