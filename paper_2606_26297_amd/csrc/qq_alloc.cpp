// qq_alloc.cpp -- variable-to-QPU allocation strategies and candidate selection (multi-QPU variable
// allocation section, Fig. 1).  Host code only: these run once per problem and feed the
// partitioned phases (eq. (16)) through qq_set_allocation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "qq_internal.h"

using namespace qq;

namespace {

qq_status bad(const char *fmt, int a = 0, int b = 0, int c = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b, c);
    return set_error(QQ_E_INVALID, buf);
}

// Shared argument checks; the coupling weights w_ij = |H_ij + H_ji| (i != j), the magnitudes of the
// canonical quadratic coefficients of eq. (5).
qq_status prepare(int n, const double *H, int M, const int *caps, std::vector<double> &w)
{
    if (n < 1 || n > QQ_MAX_N) return bad("n = %d outside [1, %d]", n, QQ_MAX_N);
    if (!H) return bad("H is NULL");
    if (M < 1 || M > QQ_MAX_QPUS || M > n) return bad("num_qpus = %d outside [1, min(n, %d)]", M, QQ_MAX_QPUS);
    if (caps) {
        int total = 0;
        for (int m = 0; m < M; ++m) {
            if (caps[m] < 1) return bad("capacity of QPU %d is %d; every QPU needs room for a variable", m, caps[m]);
            total += caps[m];
        }
        if (total < n) return bad("capacities hold %d variables, the problem has %d", total, n);
    }
    w.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            const double v = H[(size_t)i * n + j] + H[(size_t)j * n + i];
            if (!std::isfinite(v)) return bad("H has a non-finite coupling at (%d, %d)", i, j);
            w[(size_t)i * n + j] = std::fabs(v);
        }
    return QQ_OK;
}

std::vector<int> capacities_or_balanced(int n, int M, const int *caps)
{
    std::vector<int> c(M);
    for (int m = 0; m < M; ++m) c[m] = caps ? caps[m] : n / M + (m < n % M ? 1 : 0);
    return c;
}

int64_t cross_count(int n, const std::vector<double> &w, const int32_t *q)
{
    int64_t x = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (w[(size_t)i * n + j] != 0.0 && q[i] != q[j]) ++x;
    return x;
}

// Contiguous: variables in order fill QPU 0 up to its capacity, then QPU 1, ...; with capacities
// summing above n, every QPU first keeps one variable for the QPUs after it.
void contiguous(int n, int M, const std::vector<int> &c, int32_t *q)
{
    int i = 0;
    for (int m = 0; m < M; ++m) {
        const int room = std::min(c[m], n - i - (M - 1 - m));
        for (int k = 0; k < room; ++k) q[i++] = m;
    }
}

// Graph-aware greedy: QPUs are filled one after another.  A QPU starts from the unassigned variable
// of largest coupling strength s(v) = sum_u w_uv, then repeatedly takes the unassigned variable with
// the largest gain 2 w(v, QPU) - s(v) (couplings it brings inside minus those it leaves outside)
// until it is full; ties go to the lower variable index.  Each QPU stops early enough to leave one
// variable for every later QPU, and the last QPU takes the rest.
void graph_aware(int n, int M, const std::vector<int> &c, const std::vector<double> &w, int32_t *q)
{
    std::vector<double> s(n, 0.0);
    for (int v = 0; v < n; ++v)
        for (int u = 0; u < n; ++u) s[v] += w[(size_t)v * n + u];
    std::vector<int> free(n, 1);
    int left = n;
    for (int m = 0; m < M; ++m) {
        const int room = (m == M - 1) ? left : std::min(c[m], left - (M - 1 - m));
        std::vector<double> in(n, 0.0);  // w(v, QPU m)
        for (int k = 0; k < room; ++k) {
            int best = -1;
            double key = 0.0;
            for (int v = 0; v < n; ++v) {
                if (!free[v]) continue;
                const double kv = k == 0 ? s[v] : 2.0 * in[v] - s[v];
                if (best < 0 || kv > key) {
                    best = v;
                    key = kv;
                }
            }
            q[best] = m;
            free[best] = 0;
            --left;
            for (int v = 0; v < n; ++v) in[v] += w[(size_t)v * n + best];
        }
    }
}

}  // namespace

extern "C" {

qq_status qq_balanced_capacities(int n, int M, int *capacities_out)
{
    if (!capacities_out) return bad("capacities_out is NULL");
    if (n < 1 || M < 1 || M > n) return bad("need 1 <= num_qpus = %d <= n = %d", M, n);
    for (int m = 0; m < M; ++m) capacities_out[m] = n / M + (m < n % M ? 1 : 0);
    return QQ_OK;
}

qq_status qq_allocation(int n, const double *H, int M, const int *capacities, int strategy, int32_t *qpu_out,
                        int64_t *cross_out)
{
    if (!qpu_out) return bad("qpu_out is NULL");
    if (strategy != QQ_ALLOC_CONTIGUOUS && strategy != QQ_ALLOC_GRAPH) return bad("strategy = %d is unknown", strategy);
    std::vector<double> w;
    if (qq_status st = prepare(n, H, M, capacities, w); st != QQ_OK) return st;
    const std::vector<int> c = capacities_or_balanced(n, M, capacities);
    if (strategy == QQ_ALLOC_CONTIGUOUS) contiguous(n, M, c, qpu_out);
    else graph_aware(n, M, c, w, qpu_out);
    if (cross_out) *cross_out = cross_count(n, w, qpu_out);
    return QQ_OK;
}

qq_status qq_allocation_candidates(int n, const double *H, int M, const int *capacities, const int32_t *manual, int p,
                                   int32_t *qpu_out, int64_t *cross_out, int64_t *remote_out, int *count, int *best)
{
    if (!qpu_out || !cross_out || !count || !best) return bad("qpu_out / cross_out / count / best is NULL");
    if (p < 1 || p > QQ_MAX_P) return bad("p = %d outside [1, %d]", p, QQ_MAX_P);
    std::vector<double> w;
    if (qq_status st = prepare(n, H, M, capacities, w); st != QQ_OK) return st;
    const std::vector<int> c = capacities_or_balanced(n, M, capacities);
    if (manual) {  // validated like qq_set_allocation: every variable once, capacities, every QPU used
        std::vector<int> cnt(M, 0);
        for (int i = 0; i < n; ++i) {
            if (manual[i] < 0 || manual[i] >= M) return bad("manual: variable %d on QPU %d outside [0, %d)", i + 1, manual[i], M);
            ++cnt[manual[i]];
        }
        for (int m = 0; m < M; ++m)
            if (cnt[m] == 0 || cnt[m] > c[m]) return bad("manual: QPU %d holds %d variables (capacity %d)", m, cnt[m], c[m]);
    }
    // candidates in the fixed priority order used to break ties: graph-aware, contiguous, manual
    int k = 0;
    graph_aware(n, M, c, w, qpu_out);
    ++k;
    contiguous(n, M, c, qpu_out + (size_t)n);
    ++k;
    if (manual) {
        for (int i = 0; i < n; ++i) qpu_out[(size_t)2 * n + i] = manual[i];
        ++k;
    }
    int b = 0;
    for (int j = 0; j < k; ++j) {
        cross_out[j] = cross_count(n, w, qpu_out + (size_t)j * n);
        if (remote_out) remote_out[j] = 2 * cross_out[j] * p;
        if (cross_out[j] < cross_out[b]) b = j;
    }
    *count = k;
    *best = b;
    return QQ_OK;
}

}  // extern "C"
