"""Python convenience layer over the C ABI: a Problem handle and a torch.autograd.Function.

Every computation happens in libqaoa_qubo.so; this module only manages
handles, buffers and streams.  torch provides device memory and streams.
"""
from __future__ import annotations

import numpy as np

from . import native as N


def rank_key(stats, use_reference=False):
    """Sort key (smaller is better) of a sampled candidate, following the ranking of the
    depth-progression / multi-start subsection: with a classical reference, agreement with the exact
    optimum cost, then with its bitstring, then the shot fractions at that cost and at that
    bitstring; then (and alone without a reference) the best sampled cost, the fraction of shots at
    it, the frequency of the best sampled bitstring and the sample mean cost."""
    base = (stats["best_cost"], -stats["best_cost_mass"], -stats["best_frequency"], stats["mean_cost"])
    if not use_reference:
        return base
    return (-stats["matches_exact_cost"], -stats["matches_exact_index"], -stats["exact_cost_mass"],
            -stats["exact_index_frequency"]) + base


class Problem:
    """A QUBO in the dense input form F(z) = c0 + f^T z + z^T H z (eq. (2)), resident on one GPU."""

    def __init__(self, H, f=None, c0=0.0, device=0):
        H = np.asarray(H, dtype=np.float64)
        self.n = int(H.shape[0])
        self.device = device
        self.handle = N.qq_problem_create(self.n, H, f, c0, device)

    def close(self):
        if getattr(self, "handle", None):
            N.qq_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> N.QQInfo:
        return N.qq_problem_info(self.handle)

    def optimize(self, p_max, iterations, random_points, perturbations=None, random_starts=1, perturbed_starts=0,
                 include_warm=1, adam=(0.01, 0.9, 0.999, 1e-8), c128=False, partitioned=False, stream=None):
        """Depth progression with multi-start search (qq_optimize); random inputs as laid out by
        workloads.optimizer_draws."""
        flags = (N.QQ_C128 if c128 else 0) | (N.QQ_PARTITIONED if partitioned else 0)
        return N.qq_optimize(self.handle, {"p_max": p_max, "iterations": iterations, "random_starts": random_starts,
                                           "perturbed_starts": perturbed_starts, "include_warm": include_warm,
                                           "flags": flags, "adam": adam}, random_points, perturbations, stream)

    def sample(self, x, uniforms, c128=False, partitioned=False):
        """Basis indices of shots from the exact distribution of the state at x (one parameter set),
        one per uniform in [0, 1)."""
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        flags = (N.QQ_C128 if c128 else 0) | (N.QQ_PARTITIONED if partitioned else 0)
        return N.qq_sample(self.handle, x.shape[0] // 2, x, uniforms, flags)

    def sample_stats(self, indices, margin=0.0, k=10):
        """Sampled-solution metrics of host indices (qq_sample_stats)."""
        return N.qq_sample_stats(self.handle, indices, margin, k)

    def coefficients(self):
        """(l, b, alpha, h, J) of eq. (4)-(5) and eq. (9)."""
        return N.qq_coefficients(self.handle, self.n)

    def diagonal(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.int32 if self.info.is_integer else np.float64)
        return N.qq_cost_diagonal(self.handle, out)

    def set_allocation(self, qpu_of_var, num_qpus=None, capacities=None):
        q = np.asarray(qpu_of_var, dtype=np.int32)
        M = int(q.max()) + 1 if num_qpus is None else int(num_qpus)
        return N.qq_set_allocation(self.handle, M, q, capacities)

    def workspace_size(self, p, batch, flags) -> int:
        return N.qq_workspace_size(self.handle, p, batch, flags)

    def evaluate(self, params, grad=False, c128=False, partitioned=False, workspace=None):
        """Energies (and gradients) for params[B, 2p] given as numpy (host path) or a CUDA tensor (device path)."""
        import torch

        flags = N.QQ_ENERGY | (N.QQ_GRAD if grad else 0) | (N.QQ_C128 if c128 else 0) | \
            (N.QQ_PARTITIONED if partitioned else 0)
        if isinstance(params, torch.Tensor) and params.is_cuda:
            x = params.detach().to(torch.float64).contiguous()
            B, twop = x.shape
            p = twop // 2
            flags |= N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
            e = torch.empty(B, dtype=torch.float64, device=x.device)
            g = torch.empty(B, twop, dtype=torch.float64, device=x.device) if grad else None
            ws_bytes = self.workspace_size(p, B, flags)
            ws = workspace if workspace is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=x.device)
            N.qq_evaluate(self.handle, p, B, x, flags, ws, ws.numel(), torch.cuda.current_stream(x.device), e, g)
            return (e, g) if grad else e
        x = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
        B, twop = x.shape
        p = twop // 2
        e = np.empty(B)
        g = np.empty((B, twop)) if grad else None
        N.qq_evaluate(self.handle, p, B, x, flags, None, 0, None, e, g)
        return (e, g) if grad else e

    def evaluate_guarded(self, params, tol=1e-5, partitioned=False):
        """Energies and gradients (host numpy) with every gradient held to `tol` relative: complex64 first,
        the sets whose complex64 error bound exceeds the tolerance again with complex128 states.
        Returns (energies, gradients, c128 flags, gradient error bounds)."""
        x = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
        B, twop = x.shape
        e, g = np.empty(B), np.empty((B, twop))
        up, err = np.empty(B, dtype=np.int32), np.empty(B)
        flags = N.QQ_ENERGY | N.QQ_GRAD | (N.QQ_PARTITIONED if partitioned else 0)
        N.qq_evaluate_guarded(self.handle, twop // 2, B, x, flags, tol, e, g, up, err)
        return e, g, up, err

    def state(self, params, c128=False, partitioned=False):
        x = np.ascontiguousarray(params, dtype=np.float64).ravel()
        p = x.shape[0] // 2
        flags = (N.QQ_C128 if c128 else 0) | (N.QQ_PARTITIONED if partitioned else 0)
        out = np.empty(1 << self.n, dtype=np.complex128 if c128 else np.complex64)
        return N.qq_state(self.handle, p, x, flags, out)

    def probabilities(self, params, c128=False):
        x = np.ascontiguousarray(params, dtype=np.float64).ravel()
        out = np.empty(1 << self.n)
        return N.qq_probabilities(self.handle, x.shape[0] // 2, x, N.QQ_C128 if c128 else 0, out)

    def topk(self, params, k=10, c128=False):
        x = np.ascontiguousarray(params, dtype=np.float64).ravel()
        return N.qq_topk(self.handle, x.shape[0] // 2, x, N.QQ_C128 if c128 else 0, k)

    def evaluate_plain(self, params, grad=False):
        x = np.ascontiguousarray(params, dtype=np.float64).ravel()
        return N.qq_evaluate_plain(self.handle, x.shape[0] // 2, x, N.QQ_GRAD if grad else N.QQ_ENERGY)


def evaluate_many(problems, params, grad=False, options=None, workspace=None, c128=False):
    """Energies (and gradients) of many problems in one persistent launch per diagonal type.

    problems: list of Problem; params: list of [B_i, 2p_i] arrays (numpy: host path) or
    CUDA tensors (device path).  options: dict with tiles_per_chunk, max_workgroups,
    wait_limit_ms (0 = automatic).  c128: complex128 states.  Returns (energies, grads) as
    lists (grads None without grad).
    """
    import torch

    flags = N.QQ_ENERGY | (N.QQ_GRAD if grad else 0) | (N.QQ_C128 if c128 else 0)
    handles = [pb.handle for pb in problems]
    dev = len(params) > 0 and isinstance(params[0], torch.Tensor) and params[0].is_cuda
    if dev:
        xs = [x.detach().to(torch.float64).contiguous() for x in params]
        device = xs[0].device
        flags |= N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
        e = [torch.empty(x.shape[0], dtype=torch.float64, device=device) for x in xs]
        g = [torch.empty(x.shape, dtype=torch.float64, device=device) for x in xs] if grad else None
    else:
        xs = [np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64) for x in params]
        e = [np.empty(x.shape[0]) for x in xs]
        g = [np.empty(x.shape) for x in xs] if grad else None
    ps = [x.shape[1] // 2 for x in xs]
    bs = [x.shape[0] for x in xs]
    stream = None
    ws, ws_bytes = None, 0
    if dev:
        ws_bytes = N.qq_workspace_size_many(handles, ps, bs, flags, options)
        ws = workspace if workspace is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        stream = torch.cuda.current_stream(device)
    N.qq_evaluate_many(handles, ps, bs, xs, flags, options, ws, ws_bytes, stream, e, g)
    return e, g


def evaluate_many_guarded(problems, params, tol=1e-5, options=None):
    """Energies and gradients of many problems (host numpy lists) with every gradient held to `tol`
    relative: one complex64 persistent launch, then complex128 for the sets whose bound exceeds the
    tolerance.  Returns (energies, gradients, c128 flags, gradient error bounds), each a list."""
    xs = [np.atleast_2d(np.asarray(x, dtype=np.float64)) for x in params]
    bs = [x.shape[0] for x in xs]
    ps = [x.shape[1] // 2 for x in xs]
    # one packed buffer per kind (a check per buffer instead of per problem), split into views after
    flat = np.concatenate([x.reshape(-1) for x in xs]) if xs else np.empty(0)
    nb = sum(bs)
    e_all, g_all = np.empty(nb), np.empty(flat.size)
    up_all, err_all = np.empty(nb, dtype=np.int32), np.empty(nb)
    N.qq_evaluate_many_guarded_packed([pb.handle for pb in problems], ps, bs, flat, N.QQ_ENERGY | N.QQ_GRAD, options,
                                      tol, e_all, g_all, up_all, err_all)
    e, g, up, err = [], [], [], []
    o1 = o2 = 0
    for x, b in zip(xs, bs):
        e.append(e_all[o1:o1 + b])
        up.append(up_all[o1:o1 + b])
        err.append(err_all[o1:o1 + b])
        g.append(g_all[o2:o2 + x.size].reshape(x.shape))
        o1 += b
        o2 += x.size
    return e, g, up, err


def _make_autograd():
    import torch

    class QAOAEnergy(torch.autograd.Function):
        """E(x) for x[B, 2p] on the GPU; backward returns g_out[:, None] * dE/dx from the adjoint sweep."""

        @staticmethod
        def forward(ctx, params, problem, c128=False):
            need = params.requires_grad
            if need:
                e, g = problem.evaluate(params, grad=True, c128=c128)
                ctx.save_for_backward(g)
            else:
                e = problem.evaluate(params, grad=False, c128=c128)
            return e

        @staticmethod
        def backward(ctx, g_out):
            (g,) = ctx.saved_tensors
            return g_out[:, None] * g, None, None

    return QAOAEnergy


_QAOAEnergy = None


def qaoa_energy(params, problem: Problem, c128: bool = False):
    """Differentiable QAOA energy: params[B, 2p] (CUDA tensor) -> energies[B]."""
    global _QAOAEnergy
    if _QAOAEnergy is None:
        _QAOAEnergy = _make_autograd()
    return _QAOAEnergy.apply(params, problem, c128)
