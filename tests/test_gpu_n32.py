"""Full-size multi-QPU checks at n = 32 (2^32 amplitudes, 32 GiB per complex64 state).

The FP64 oracle cannot run at this size, so the checks use results that hold at
any size (1e-5 relative; energy |dE| / max(|E|, sigma_C), gradient
||dg||_inf / ||g||_inf):
  * a 4 x 8 block problem allocated one block per QPU has no cross couplings;
    its energy and gradient are the sums of the per-block oracle results, for
    the monolithic and the partitioned evaluation alike;
  * a separable instance: the closed form of a product state (and its central differences);
  * the dense N(0,1) multi-QPU workload (496 couplings, 4 QPUs of 8 variables,
    contiguous allocation, p = 2, two parameter sets): the partitioned energy,
    gradient and final state against the monolithic ones (the state compared on
    the device, ||psi_part - psi_mono||_2 <= 1e-5), and the complex64 energy and
    gradient against the complex128 generic kernel and against central differences of
    complex128 energies (forward path only), and 2000 sampled entries of its cost
    diagonal against the oracle's one-index sums (bit for bit).
Device memory: the diagonal and the cross diagonal (FP64, 32 GiB each) plus the
states of the evaluation; at most about 160 GiB at once.

At the maximum size, n = 34 (QQ_MAX_N): an integer cluster-product instance (couplings only inside
blocks, some of which straddle the 4-qubit runs of every set, so the per-tile cost tables carry
couplings between tile and base bits) whose energy is c0 plus the sum of the per-block oracle
energies; energy only (one complex64 state of 128 GiB, a 2-byte diagonal of 32 GiB, 18 GiB of
cost tables).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu

N32 = 32


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def e_rel(e, eref, sigma):
    return float(np.max(np.abs(np.asarray(e) - np.asarray(eref)) / np.maximum(np.abs(eref), sigma)))


def g_rel(g, gref):
    g, gref = np.atleast_2d(g), np.atleast_2d(gref)
    return max(float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) for a, b in zip(g, gref))


def test_n32_block_problem_monolithic_and_partitioned_vs_block_oracle():
    inst = W.cluster_product([8, 8, 8, 8], 71)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        q = W.contiguous_allocation(N32, [8, 8, 8, 8])
        cross, remote = pb.set_allocation(q, 4, [8, 8, 8, 8])
        assert cross == 0 and remote == 0
        p = 2
        x = W.random_params(p, 1, 72)
        eref = inst.c0
        gref = np.zeros(2 * p)
        for off, m in inst.meta["blocks"]:
            d = O.cost_diagonal(inst.H[off:off + m, off:off + m], None, 0.0)
            eb, gb = O.gradient(d, x[0])
            eref += eb
            gref += gb
        sig = pb.info.sigma_c
        print("monolithic", flush=True)
        e, g = pb.evaluate(x, grad=True)
        assert e_rel(e[0], eref, sig) <= 1e-5 and g_rel(g[0], gref) <= 1e-5
        print("partitioned", flush=True)
        e, g = pb.evaluate(x, grad=True, partitioned=True)
        assert e_rel(e[0], eref, sig) <= 1e-5 and g_rel(g[0], gref) <= 1e-5
    finally:
        pb.close()


def test_n32_multi_qpu_workload_partitioned_equals_monolithic():
    import torch

    inst, x, alloc = W.workload5()
    assert inst.H.shape == (N32, N32) and np.count_nonzero(np.triu(inst.H, 1)) == 496
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        caps = O.balanced_capacities(N32, 4)
        cross, remote = pb.set_allocation(alloc, 4, caps)
        ell, b = O.canonicalise(inst.H, inst.f)
        assert cross == O.cross_terms(b, alloc) == 384 and remote == 2 * cross
        sig = pb.info.sigma_c
        print("monolithic", flush=True)
        e0, g0 = pb.evaluate(x, grad=True)
        print("partitioned", flush=True)
        e1, g1 = pb.evaluate(x, grad=True, partitioned=True)
        assert e_rel(e1, e0, sig) <= 1e-5 and g_rel(g1, g0) <= 1e-5
        # final states on the device
        print("states", flush=True)
        flags = N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE
        xt = torch.tensor(x[0], device="cuda:0")
        psi0 = torch.empty(1 << N32, dtype=torch.complex64, device="cuda:0")
        N.qq_state(pb.handle, 2, xt, flags, psi0)
        psi1 = torch.empty_like(psi0)
        N.qq_state(pb.handle, 2, xt, flags | N.QQ_PARTITIONED, psi1)
        psi1 -= psi0
        diff = float(torch.linalg.vector_norm(psi1))
        norm = float(torch.linalg.vector_norm(psi0))
        del psi0, psi1
        torch.cuda.empty_cache()
        assert abs(norm - 1.0) <= 1e-5 and diff <= 1e-5, (norm, diff)
    finally:
        pb.close()


def test_n32_multi_qpu_workload_complex64_vs_complex128():
    """The same instance, first parameter set, monolithic: the complex64 specialised kernels
    (including the 64-bit-offset instances of the last, partial high set) against the complex128
    generic kernel, energy and gradient at 1e-5 relative.
    complex128 at n = 32 holds 64 GiB per state: 128 GiB for psi and lambda plus the 32 GiB diagonal."""
    inst, x, _ = W.workload5()
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        sig = pb.info.sigma_c
        print("complex64", flush=True)
        e64, g64 = pb.evaluate(x[:1], grad=True)
        print("complex128", flush=True)
        e128, g128 = pb.evaluate(x[:1], grad=True, c128=True)
        assert e_rel(e64, e128, sig) <= 1e-5, (e64, e128)
        assert g_rel(g64, g128) <= 1e-5, (g64, g128)
    finally:
        pb.close()


def p1_qubit(ell, x):
    v = np.array([1, 1], dtype=complex) / np.sqrt(2)
    for k in range(len(x) // 2):
        g, b = x[2 * k], x[2 * k + 1]
        v = np.array([1, np.exp(-1j * g * ell)]) * v
        v = np.array([[np.cos(b), -1j * np.sin(b)], [-1j * np.sin(b), np.cos(b)]]) @ v
    return abs(v[1]) ** 2


def separable_energy(ell, c0, x):
    return c0 + sum(li * p1_qubit(li, x) for li in ell)


def test_n32_separable_energy_and_gradient():
    """A separable instance (no couplings) at n = 32: the state is a product of single-qubit states, so
    E = c0 + sum_i l_i P_i(1) with each P_i from a 2 x 2 evolution, and the gradient follows from
    central differences of that closed form (h = 1e-6).  Covers every pass of the n = 32 plan,
    including the 64-bit-offset kernels of the partial high set."""
    inst = W.separable(N32, 73, scale=0.5)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        ell, _ = O.canonicalise(inst.H, inst.f)
        p = 2
        x = W.random_params(p, 2, 74)
        e, g = pb.evaluate(x, grad=True)
        sig = pb.info.sigma_c
        for b in range(x.shape[0]):
            eref = separable_energy(ell, inst.c0, x[b])
            gref = np.empty(2 * p)
            for j in range(2 * p):
                xp, xm = x[b].copy(), x[b].copy()
                xp[j] += 1e-6
                xm[j] -= 1e-6
                gref[j] = (separable_energy(ell, inst.c0, xp) - separable_energy(ell, inst.c0, xm)) / 2e-6
            assert e_rel(e[b], eref, sig) <= 1e-5, (b, e[b], eref)
            assert g_rel(g[b], gref) <= 1e-5, (b, g[b], gref)
    finally:
        pb.close()


def test_n32_dense_cost_diagonal_sampled_against_the_oracle():
    """The FP64 cost diagonal of the n = 32 multi-QPU workload (2^32 entries, canonical summation
    order): 2000 sampled entries, read on the device, equal the oracle's one-index sums bit for bit."""
    import torch

    inst, _, _ = W.workload5()
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        assert pb.info.diag_bytes == 8
        d = torch.empty(1 << N32, dtype=torch.float64, device="cuda:0")
        N.qq_cost_diagonal(pb.handle, d, N.QQ_OUT_ON_DEVICE)
        zs = np.random.default_rng(75).integers(0, 1 << N32, size=2000)
        zs[:4] = [0, 1, (1 << N32) - 1, 1 << (N32 - 1)]
        got = d[torch.tensor(zs, device="cuda:0")].cpu().numpy()
        del d
        torch.cuda.empty_cache()
        ell, b = O.canonicalise(inst.H, inst.f)
        want = np.array([O.cost_at_real(ell, b, inst.c0, int(z)) for z in zs])
        assert np.array_equal(got, want), int(np.sum(got != want))
    finally:
        pb.close()


def test_n32_dense_gradient_vs_central_differences():
    """The dense n = 32 multi-QPU workload (496 couplings, p = 2): the complex64 adjoint gradient, monolithic
    and partitioned, against five-point central differences of complex128 energies, which use the forward
    path only (the FP64 oracle needs 160 GiB of host memory and about an hour at this size).  The gradient
    here is small (||g||_inf about 2e-4 sigma_C), so the stencil is the fourth-order one with h = 1e-3:
    its truncation (h^4 / 30 times the fifth derivative) and the complex128 energies' rounding divided by
    h both stay near 1e-10, far below the bar of 1e-5 relative to ||g||_inf."""
    inst, x, alloc = W.workload5()
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        pb.set_allocation(alloc, 4, O.balanced_capacities(N32, 4))
        x0 = x[:1]
        print("complex64 gradients", flush=True)
        _, g_mono = pb.evaluate(x0, grad=True)
        _, g_part = pb.evaluate(x0, grad=True, partitioned=True)
        h = 1e-3
        fd = np.empty(4)
        for j in range(4):
            e = []
            for steps in ((2, 1), (-1, -2)):  # two complex128 states at a time: 128 GiB
                xs = np.repeat(x0, 2, axis=0)
                xs[0, j] += steps[0] * h
                xs[1, j] += steps[1] * h
                print(f"complex128 energies, component {j}, offsets {steps}", flush=True)
                e.extend(pb.evaluate(xs, c128=True))
            fd[j] = (-e[0] + 8 * e[1] - 8 * e[2] + e[3]) / (12 * h)
        print(f"fd {fd} adjoint {g_mono[0]}", flush=True)
        assert g_rel(g_mono, fd) <= 1e-5, (g_mono, fd)
        assert g_rel(g_part, fd) <= 1e-5, (g_part, fd)
    finally:
        pb.close()


def test_n34_cluster_product_energy_at_the_maximum_size():
    import torch

    torch.cuda.empty_cache()
    n = N.QQ_MAX_N
    sizes = [7, 7, 7, 7, 6]
    rng = np.random.default_rng(81)
    H = np.zeros((n, n))
    blocks, off = [], 0
    for m in sizes:
        H[off:off + m, off:off + m] = np.triu(rng.integers(-3, 4, size=(m, m))).astype(float)
        blocks.append((off, m))
        off += m
    c0 = 2.0
    pb = Problem(H, None, c0)
    try:
        assert pb.info.is_integer and pb.info.diag_bytes == 2
        p, B = 2, 1
        x = W.random_params(p, B, 82)
        print(f"n = {n}: energy-only evaluation, p = {p}", flush=True)
        e = pb.evaluate(x)
        eref = c0
        for o, m in blocks:
            d = O.cost_diagonal(H[o:o + m, o:o + m], None, 0.0)
            eref += O.gradient(d, x[0])[0]
        assert e_rel(e[0], eref, pb.info.sigma_c) <= 1e-5, (e[0], eref)
    finally:
        pb.close()
