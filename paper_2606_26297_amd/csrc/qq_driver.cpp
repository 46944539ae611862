// qq_driver.cpp -- depth progression with multi-start search on the exact objective (Alg. 1 and
// the depth-progression / multi-start subsection).  Host orchestration of the library's own entry
// points: every depth runs all of its starts as one batch of graph-captured Adam steps
// (qq_graph_*), then one energy evaluation of the final parameter vectors (qq_evaluate).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "qq_internal.h"

using namespace qq;

namespace {

qq_status fail_msg(qq_status st, const char *fmt, int a = 0, int b = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    return set_error(st, buf);
}

// Lift an interleaved [gamma_1, beta_1, ..., gamma_p, beta_p] to depth p + 1 by linear interpolation
// of each sequence onto p + 1 points: y_i = ((i - 1) / p) x_{i-1} + ((p - i + 1) / p) x_i,
// i = 1 .. p + 1, with x_0 = x_{p+1} = 0 (the paper leaves the rule open; this is the INTERP rule of
// Zhou et al., Phys. Rev. X 10, 021067 (2020)).
std::vector<double> lift(const std::vector<double> &x, int p)
{
    std::vector<double> y(2 * (size_t)(p + 1));
    for (int c = 0; c < 2; ++c)
        for (int i = 1; i <= p + 1; ++i) {
            const double lo = i >= 2 ? x[2 * (size_t)(i - 2) + c] : 0.0;
            const double hi = i <= p ? x[2 * (size_t)(i - 1) + c] : 0.0;
            y[2 * (size_t)(i - 1) + c] = ((double)(i - 1) / p) * lo + ((double)(p - i + 1) / p) * hi;
        }
    return y;
}

// Index of the smallest value; ties (and NaN, ranked last) go to the lower index.
int rank_first(const std::vector<double> &e)
{
    int best = 0;
    for (int i = 1; i < (int)e.size(); ++i) {
        const bool better = std::isnan(e[best]) ? !std::isnan(e[i]) : (!std::isnan(e[i]) && e[i] < e[best]);
        if (better) best = i;
    }
    return best;
}

struct DevMem {
    void *p = nullptr;
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
};

struct Graph {
    qq_graph *g = nullptr;
    ~Graph()
    {
        if (g) (void)qq_graph_destroy(g);
    }
};

}  // namespace

extern "C" qq_status qq_optimize(qq_problem *pb, const qq_optimize_options *o, const double *random_points,
                                 const double *perturbations, void *stream_, qq_optimize_result *res,
                                 double *depth_params, double *depth_energy, double *start_energy)
{
    if (!pb) return fail_msg(QQ_E_INVALID, "problem is NULL");
    if (!o) return fail_msg(QQ_E_INVALID, "options is NULL");
    if (!res) return fail_msg(QQ_E_INVALID, "result is NULL");
    const int pmax = o->p_max, R = o->random_starts, P = o->perturbed_starts, W = o->include_warm;
    if (pmax < 1 || pmax > QQ_MAX_P) return fail_msg(QQ_E_INVALID, "p_max = %d must be in [1, %d]", pmax, QQ_MAX_P);
    if (o->iterations < 0) return fail_msg(QQ_E_INVALID, "iterations = %d must be >= 0", o->iterations);
    if (R < 1) return fail_msg(QQ_E_INVALID, "random_starts = %d must be >= 1 (depth 1 has no other start)", R);
    if (P < 0) return fail_msg(QQ_E_INVALID, "perturbed_starts = %d must be >= 0", P);
    if (W != 0 && W != 1) return fail_msg(QQ_E_INVALID, "include_warm = %d must be 0 or 1", W);
    if (o->flags & ~(QQ_C128 | QQ_PARTITIONED))
        return fail_msg(QQ_E_INVALID, "flags 0x%x: only QQ_C128 and QQ_PARTITIONED are accepted", o->flags);
    if (!random_points) return fail_msg(QQ_E_INVALID, "random_points is NULL");
    if (P > 0 && pmax >= 2 && !perturbations) return fail_msg(QQ_E_INVALID, "perturbations is NULL");
    const int64_t nrand = (int64_t)R * pmax * (pmax + 1);
    const int64_t npert = (P > 0 && pmax >= 2) ? (int64_t)P * (pmax * (pmax + 1) - 2) : 0;
    for (int64_t i = 0; i < nrand; ++i)
        if (!std::isfinite(random_points[i])) return fail_msg(QQ_E_INVALID, "random_points has a non-finite value");
    for (int64_t i = 0; i < npert; ++i)
        if (!std::isfinite(perturbations[i])) return fail_msg(QQ_E_INVALID, "perturbations has a non-finite value");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (hipSetDevice(problem_device(pb)) != hipSuccess) return fail_msg(QQ_E_DEVICE, "hipSetDevice failed");

    std::memset(res, 0, sizeof *res);
    if (depth_params) std::memset(depth_params, 0, sizeof(double) * 2 * (size_t)pmax * pmax);
    const double *rp = random_points, *pp = perturbations;
    std::vector<double> prev, rep_energy(pmax);
    std::vector<int> rep_start(pmax);
    size_t start_off = 0;
    for (int p = 1; p <= pmax; ++p) {
        const int S = R + (p >= 2 ? W + P : 0);
        const size_t np = (size_t)S * 2 * p;
        std::vector<double> x(np);
        int k = 0;
        if (p >= 2) {
            const std::vector<double> warm = lift(prev, p - 1);
            if (W) std::memcpy(&x[(size_t)(k++) * 2 * p], warm.data(), sizeof(double) * 2 * p);
            for (int j = 0; j < P; ++j, ++k, pp += 2 * p)
                for (int i = 0; i < 2 * p; ++i) x[(size_t)k * 2 * p + i] = warm[i] + pp[i];
        }
        for (int j = 0; j < R; ++j, ++k, rp += 2 * p) std::memcpy(&x[(size_t)k * 2 * p], rp, sizeof(double) * 2 * p);

        // all starts of the depth step together: one graph-captured Adam step per iteration
        DevMem dx;
        if (hipMalloc(&dx.p, np * sizeof(double)) != hipSuccess)
            return fail_msg(QQ_E_NOMEM, "hipMalloc of %d x %d parameters failed", S, 2 * p);
        if (hipMemcpyAsync(dx.p, x.data(), np * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail_msg(QQ_E_DEVICE, "copying the starting points failed");
        if (o->iterations > 0) {
            Graph g;
            if (qq_status st = qq_graph_create(pb, p, S, o->flags, o->adam, static_cast<double *>(dx.p), 0, stream,
                                               &g.g);
                st != QQ_OK)
                return st;
            if (qq_status st = qq_graph_run(g.g, o->iterations, stream); st != QQ_OK) return st;
            if (hipStreamSynchronize(stream) != hipSuccess) return fail_msg(QQ_E_DEVICE, "the Adam steps failed");
        }
        if (hipMemcpyAsync(x.data(), dx.p, np * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail_msg(QQ_E_DEVICE, "copying the final parameters failed");

        // the exact energy at every start's final parameter vector ranks the starts
        std::vector<double> e(S);
        if (qq_status st = qq_evaluate(pb, p, S, x.data(), o->flags | QQ_ENERGY, nullptr, 0, stream_, e.data(), nullptr);
            st != QQ_OK)
            return st;
        const int b = rank_first(e);
        rep_start[p - 1] = b;
        rep_energy[p - 1] = e[b];
        prev.assign(x.begin() + (size_t)b * 2 * p, x.begin() + (size_t)(b + 1) * 2 * p);
        if (depth_params) std::memcpy(depth_params + (size_t)(p - 1) * 2 * pmax, prev.data(), sizeof(double) * 2 * p);
        if (start_energy) std::memcpy(start_energy + start_off, e.data(), sizeof(double) * S);
        start_off += S;
        res->steps += (long long)S * o->iterations;
        res->evaluations += (long long)S * (o->iterations + 1);
    }
    if (depth_energy) std::memcpy(depth_energy, rep_energy.data(), sizeof(double) * pmax);
    const int d = rank_first(rep_energy);
    res->best_depth = d + 1;
    res->best_start = rep_start[d];
    res->best_energy = rep_energy[d];
    return QQ_OK;
}
