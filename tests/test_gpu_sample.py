"""GPU tests of shot sampling from the exact distribution and of the sampled metrics (through the
C ABI).

* Shots against the oracle's inverse transform (n = 14, 100000 uniforms): every sampled index z is a
  valid inverse-transform index of the oracle's distribution, cdf(z - 1) <= u T < cdf(z) up to the
  state precision's tolerance (1e-12 complex128, 2e-6 complex64), has nonzero probability, and
  equals the oracle's index for at least 99.9% of the shots (all but boundary cases);
* at full size (n = 28, p = 8, the benchmark instance) against a cumulative sum of the library's own
  probabilities in PyTorch FP64 (tolerance 1e-9);
* device uniforms outside [0, 1) (and NaN) take the last index of nonzero probability, u = 0 the
  first;
* the metrics equal the oracle's on the same shots exactly (integer and real costs; same summation
  order);
* validation.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import sampling as S
from paper_2606_26297_amd import native as N
from paper_2606_26297_amd import workloads as W
from paper_2606_26297_amd.qaoa import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    N.lib()
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"


def check_valid(z, u, cdf, tol):
    z = z.astype(np.int64)
    t = u * cdf[-1]
    lo = np.where(z > 0, cdf[np.maximum(z - 1, 0)], 0.0)
    hi = cdf[z]
    assert np.all(lo <= t + tol), np.max(lo - t)
    assert np.all(t < hi + tol), np.max(t - hi)


@pytest.mark.parametrize("c128", [True, False], ids=["c128", "c64"])
def test_shots_match_oracle_inverse_transform(c128):
    inst = W.dense_gaussian_upper(14, 61)
    pb = Problem(inst.H, inst.f, inst.c0)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(3, 1, 62)[0]
    P = O.probabilities(O.qaoa_state(d, x))
    u = np.random.default_rng(63).uniform(0.0, 1.0, size=100_000)
    z = pb.sample(x, u, c128=c128)
    assert z.dtype == np.uint64 and z.shape == u.shape and np.all(z < 2 ** 14)
    check_valid(z, u, np.cumsum(P), 1e-12 if c128 else 2e-6)
    assert np.all(P[z.astype(np.int64)] > 0)
    assert np.mean(z == S.inverse_cdf(P, u)) >= 0.999


def test_shots_full_size_n28_against_cumulative_probabilities():
    import torch

    inst, x = W.workload3(batch=1)
    pb = Problem(inst.H, inst.f, inst.c0)
    try:
        xt = torch.tensor(x[0], device="cuda:0")
        prob = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0")
        N.qq_probabilities(pb.handle, 8, xt, N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE, prob)
        cdf = torch.cumsum(prob, 0)
        del prob
        u = np.random.default_rng(64).uniform(0.0, 1.0, size=20_000)
        ut = torch.tensor(u, device="cuda:0")
        zt = torch.empty(u.size, dtype=torch.int64, device="cuda:0")
        N.qq_sample(pb.handle, 8, xt, ut, N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE, out=zt)
        z = zt.cpu().numpy()
        assert np.all((z >= 0) & (z < (1 << 28)))
        t = ut * cdf[-1]
        hi = cdf[zt]
        lo = torch.where(zt > 0, cdf[torch.clamp(zt - 1, min=0)], torch.zeros_like(t))
        assert bool(torch.all(lo <= t + 1e-9)) and bool(torch.all(t < hi + 1e-9))
        del cdf
        torch.cuda.empty_cache()
    finally:
        pb.close()


@pytest.mark.parametrize("n", [10, 14])
def test_device_uniforms_outside_the_unit_interval_take_the_last_nonzero_index(n):
    """Device uniforms are not range-checked: values outside [0, 1), NaN, and one whose product with
    the total probability rounds up to it take the last index of nonzero probability; u = 0 takes
    the first (n = 10: one block with padding entries of zero probability; n = 14: four blocks)."""
    import torch

    inst = W.dense_gaussian_upper(n, 70)
    pb = Problem(inst.H, inst.f, inst.c0)
    x = W.random_params(2, 1, 71)[0]
    P = O.probabilities(O.qaoa_state(O.cost_diagonal(inst.H, inst.f, inst.c0), x))
    last = int(np.flatnonzero(P > 0)[-1])
    u = np.array([-0.1, 1.0, 1.5, np.nan, -np.inf, np.inf, np.nextafter(1.0, 0.0), 0.0])
    for c128 in (True, False):
        xt = torch.tensor(x, device="cuda:0")
        ut = torch.tensor(u, device="cuda:0")
        zt = torch.empty(u.size, dtype=torch.int64, device="cuda:0")
        flags = N.QQ_PARAMS_ON_DEVICE | N.QQ_OUT_ON_DEVICE | (N.QQ_C128 if c128 else 0)
        N.qq_sample(pb.handle, 2, xt, ut, flags, out=zt)
        z = zt.cpu().numpy()
        assert list(z[:7]) == [last] * 7, (c128, z)
        assert z[7] == int(S.inverse_cdf(P, [0.0])[0]), (c128, z)


@pytest.mark.parametrize("name,maker", [("int_n12", lambda: W.workload1()[0]),
                                        ("real_n14", lambda: W.unit_commitment_shaped(14, 65))])
def test_metrics_equal_the_oracles(name, maker):
    inst = maker()
    pb = Problem(inst.H, inst.f, inst.c0)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(2, 1, 66)[0]
    u = np.random.default_rng(67).uniform(0.0, 1.0, size=50_000)
    z = pb.sample(x, u)
    info = pb.info
    for margin in (0.0, 0.05 * (info.cmax - info.cmin)):
        got = pb.sample_stats(z, margin=margin, k=10)
        ref = S.sample_stats(z, d, margin, 10, info.cmin, info.argmin_index)
        for key in ("shots", "distinct", "best_index", "best_cost", "best_frequency", "best_cost_mass", "mean_cost",
                    "low_cost_mass", "exact_cost", "exact_index", "matches_exact_cost", "matches_exact_index",
                    "exact_cost_mass", "exact_index_frequency"):
            assert got[key] == ref[key], (name, margin, key, got[key], ref[key])
        assert np.array_equal(got["elite_index"], ref["elite_index"].astype(np.uint64))
        assert np.array_equal(got["elite_count"], ref["elite_count"])
        assert np.array_equal(got["elite_cost"], ref["elite_cost"])


def test_sampling_validation():
    inst = W.regular_graph_qubo(10, 68)
    pb = Problem(inst.H, inst.f, inst.c0)
    x = W.random_params(1, 1, 69)[0]
    for u in (np.array([0.5, 1.0]), np.array([-0.1]), np.array([np.nan])):
        with pytest.raises(N.QQError) as ei:
            pb.sample(x, u)
        assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError) as ei:
        N.qq_sample(pb.handle, 1, x, np.zeros(0))
    assert ei.value.status == N.QQ_E_INVALID
    with pytest.raises(N.QQError) as ei:
        N.qq_sample(pb.handle, 1, x, np.array([0.5]), flags=N.QQ_GRAD)
    assert ei.value.status == N.QQ_E_INVALID
    for idx, margin, k in (([1 << 10], 0.0, 3), ([1, 2], -1.0, 3), ([1, 2], 0.0, -1)):
        with pytest.raises(N.QQError) as ei:
            pb.sample_stats(np.array(idx, dtype=np.uint64), margin=margin, k=k)
        assert ei.value.status == N.QQ_E_INVALID
