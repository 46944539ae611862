"""Gradient evaluations with psi and lambda in alternating blocks of 2^16 amplitudes (the layout the
complex64 per-pass kernels use for n = 20 and n >= 24) against the complex128 path, which keeps
separate arrays: dense N(0,1) instances whose sets cover every geometry of the interleaved
addressing (n = 20: one high set starting at qubit 12; n = 26: a partial set at 18..25; n = 29 and
31: partial sets whose upper run starts at 25 and 27, the latter with 64-bit lane offsets), each
monolithic and partitioned; and n = 21, where a run straddles qubit 16 and the arrays stay separate.
Energy 1e-5 relative (|dE| / max(|E|, sigma_C)); gradient within the stated complex64 bound."""
import numpy as np
import pytest

from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def c64_bound(n, sigma, gmax):
    return N.QQ_GUARD_REL * gmax + N.QQ_GUARD_K * sigma * sigma * 2.0 ** -24 * 2.0 ** (-0.5 * n)


@pytest.mark.parametrize("n,p,batch", [(20, 3, 3), (21, 2, 2), (26, 2, 2), (29, 2, 1), (31, 1, 1)])
def test_interleaved_gradients_vs_complex128(n, p, batch):
    import torch

    torch.cuda.empty_cache()  # the library allocates its own workspaces here
    inst = W.dense_gaussian_upper(n, 600 + n)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        x = W.random_params(p, batch, 700 + n)
        sig = pb.info.sigma_c
        print(f"n = {n}, p = {p}, batch = {batch}: complex128 reference", flush=True)
        e128, g128 = pb.evaluate(x, grad=True, c128=True)
        checks = [("monolithic", False)]
        if n <= 29:
            M = 4
            pb.set_allocation(np.arange(n) * M // n, M)
            checks.append(("partitioned", True))
        for name, part in checks:
            print(f"n = {n}: complex64 {name}", flush=True)
            e, g = pb.evaluate(x, grad=True, partitioned=part)
            assert np.max(np.abs(e - e128) / np.maximum(np.abs(e128), sig)) <= 1e-5, (name, e, e128)
            for b in range(batch):
                gmax = float(np.max(np.abs(g128[b])))
                assert np.max(np.abs(g[b] - g128[b])) <= c64_bound(n, sig, gmax), (name, b, g[b], g128[b])
    finally:
        pb.close()
