"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute force
of the input form eq. (2), dense matrix exponentials of eq. (10)/(13), closed
forms (n = 1, separable and cluster-product instances), invariants of the
QAOA state, central finite differences, values printed in the paper (Fig. 1
cross counts, the decoding convention), and planted mistakes that a pin must
catch.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_2606_26297_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bits_of(n):
    z = np.arange(1 << n)
    return ((z[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)  # row z -> (z_1..z_n)


def brute_force_F(H, f, c0):
    """eq. (2) directly: F(z) = c0 + f.z + z^T H z for every z (no canonical form)."""
    n = H.shape[0]
    Z = bits_of(n)
    return c0 + Z @ f + np.einsum("zi,ij,zj->z", Z, H, Z)


def test_diag_integer_vs_bruteforce_exact():
    for seed in range(4):
        rng = np.random.default_rng(seed)
        n = 9
        H = rng.integers(-10, 11, size=(n, n)).astype(float)  # non-symmetric on purpose
        f = rng.integers(-5, 6, size=n).astype(float)
        c0 = float(rng.integers(-20, 21))
        d = O.cost_diagonal(H, f, c0)
        assert d.dtype == np.int64
        ref = brute_force_F(H, f, c0)
        assert np.array_equal(d.astype(np.float64), ref)


def test_workload1_diag_all_4096_strings():
    inst, _ = W.workload1()
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    assert d.shape == (4096,) and d.dtype == np.int64
    ref = brute_force_F(inst.H, inst.f, inst.c0)
    assert np.array_equal(d.astype(np.float64), ref)
    # brute-force optimum: lowest index among minimisers
    assert O.argmin_cost(d) == int(np.flatnonzero(ref == ref.min())[0])


def test_diag_real_vs_bruteforce():
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        n = 10
        H = rng.normal(size=(n, n))
        f = rng.normal(size=n)
        c0 = float(rng.normal())
        d = O.cost_diagonal(H, f, c0)
        assert d.dtype == np.float64
        ref = brute_force_F(H, f, c0)
        scale = abs(c0) + np.abs(H).sum() + np.abs(f).sum()
        assert np.max(np.abs(d - ref)) <= 1e-13 * scale


def test_cost_at_one_index_equals_the_diagonal_exactly():
    # the one-index form sums in the same canonical order, so it reproduces every FP64 entry; and
    # both agree with the brute-force z^T H z + f.z + c0 within rounding
    rng = np.random.default_rng(110)
    n = 9
    H = rng.normal(size=(n, n))
    f = rng.normal(size=n)
    c0 = float(rng.normal())
    ell, b = O.canonicalise(H, f)
    d = O.cost_diagonal_real(ell, b, c0)
    one = np.array([O.cost_at_real(ell, b, c0, z) for z in range(1 << n)])
    assert np.array_equal(one, d)
    ref = brute_force_F(H, f, c0)
    assert np.max(np.abs(one - ref)) <= 1e-13 * (abs(c0) + np.abs(H).sum() + np.abs(f).sum())


def test_real_path_equals_integer_path_on_integer_data():
    inst, _ = W.workload1()
    ell, b = O.canonicalise(inst.H, inst.f)
    dr = O.cost_diagonal_real(ell, b, inst.c0)
    di = O.cost_diagonal(inst.H, inst.f, inst.c0)
    assert np.array_equal(dr, di.astype(np.float64))


def test_bit_order_convention():
    # l_1 alone: C(z) = l_1 * z_1 and z_1 is bit 0 of the index
    n = 5
    H = np.zeros((n, n))
    H[0, 0] = 3.0
    d = O.cost_diagonal(H, None, 0.0)
    z = np.arange(1 << n)
    assert np.array_equal(d, 3 * (z & 1))
    # a coupling between variables 2 and 5 (qubits 1 and 4)
    H = np.zeros((n, n))
    H[1, 4] = 7.0
    d = O.cost_diagonal(H, None, 0.0)
    assert np.array_equal(d, 7 * (((z >> 1) & 1) & ((z >> 4) & 1)))


def test_decode_convention_golden():
    with open(os.path.join(GOLDEN, "decode_convention.json")) as fh:
        g = json.load(fh)
    for case in g["cases"]:
        n = len(case["logical"])
        assert O.index_from_display(case["display"]) == case["index"]
        assert O.bitstring(case["index"], n) == case["logical"]
        assert case["display"][::-1] == case["logical"]


def test_ising_identity_mean_and_std():
    for inst in (W.workload1()[0], W.unit_commitment_shaped(8, 5), W.regular_graph_qubo(10, 3)):
        ell, b = O.canonicalise(inst.H, inst.f)
        alpha, h, J, sigma = O.ising_coefficients(ell, b, inst.c0)
        n = inst.n
        S = 1.0 - 2.0 * bits_of(n)  # eigenvalue of Z_i on |z> is (-1)^{z_i}
        ising = alpha + S @ h + np.einsum("zi,ij,zj->z", S, J, S)
        d = O.cost_diagonal(inst.H, inst.f, inst.c0).astype(np.float64)
        scale = np.abs(d).max() + 1.0
        assert np.max(np.abs(ising - d)) <= 1e-12 * scale
        assert abs(d.mean() - alpha) <= 1e-12 * scale
        assert abs(d.std() - sigma) <= 1e-10 * scale


def pauli_x(n, q):
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    out = np.array([[1.0 + 0j]])
    for k in range(n - 1, -1, -1):  # kron order: qubit n-1 is the most significant factor
        out = np.kron(out, X if k == q else np.eye(2))
    return out


def expm_state(diag, x):
    n = int(len(diag)).bit_length() - 1
    HM = sum(pauli_x(n, q) for q in range(n))
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=complex)
    for k in range(len(x) // 2):
        g, b = x[2 * k], x[2 * k + 1]
        psi = scipy.linalg.expm(-1j * g * np.diag(np.asarray(diag, dtype=float))) @ psi
        psi = scipy.linalg.expm(-1j * b * HM) @ psi
    return psi


def test_state_vs_dense_expm():
    for seed, n, p in [(1, 3, 1), (2, 5, 2), (3, 7, 3)]:
        rng = np.random.default_rng(seed)
        H = rng.normal(size=(n, n))
        f = rng.normal(size=n)
        d = O.cost_diagonal(H, f, 0.3)
        x = rng.uniform(0, np.pi, size=2 * p)
        psi = O.qaoa_state(d, x)
        ref = expm_state(d, x)
        assert np.linalg.norm(psi - ref) <= 1e-11


def n1_closed_form(ell, c0, g, b):
    E = c0 + 0.5 * ell * (1 + np.sin(2 * b) * np.sin(g * ell))
    dg = 0.5 * ell**2 * np.sin(2 * b) * np.cos(g * ell)
    db = ell * np.cos(2 * b) * np.sin(g * ell)
    return E, np.array([dg, db])


def test_n1_closed_form_energy_and_gradient():
    for ell, c0, g, b in [(1.3, 0.2, 0.4, 0.7), (-2.5, 1.0, 2.1, 0.3), (0.7, -3.0, 1.0, 2.9)]:
        H = np.array([[ell]])
        d = O.cost_diagonal(H, None, c0)
        E, grad = O.gradient(d, [g, b])
        Eref, gref = n1_closed_form(ell, c0, g, b)
        assert abs(E - Eref) <= 1e-13 * (1 + abs(Eref))
        assert np.max(np.abs(grad - gref)) <= 1e-13 * (1 + np.abs(gref).max())


def single_qubit_p1(ell, x):
    """Prob(z_i = 1) of one qubit under prod_k RX(2 b_k) diag(1, e^{-i g_k l}) |+>."""
    v = np.array([1, 1], dtype=complex) / np.sqrt(2)
    for k in range(len(x) // 2):
        g, b = x[2 * k], x[2 * k + 1]
        v = np.array([1, np.exp(-1j * g * ell)]) * v
        v = np.array([[np.cos(b), -1j * np.sin(b)], [-1j * np.sin(b), np.cos(b)]]) @ v
    return abs(v[1]) ** 2


def test_separable_product_formula():
    inst = W.separable(12, 7)
    ell, b = O.canonicalise(inst.H, inst.f)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(3, 1, 9)[0]
    E = O.energy(d, x)
    Eref = inst.c0 + sum(ell[i] * single_qubit_p1(ell[i], x) for i in range(inst.n))
    assert abs(E - Eref) <= 1e-12 * (1 + abs(Eref))


def test_cluster_product_sum_of_blocks():
    inst = W.cluster_product([4, 3, 5], 11)
    x = W.random_params(2, 1, 12)[0]
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    E, g = O.gradient(d, x)
    Es, gs = inst.c0, np.zeros_like(x)
    for off, m in inst.meta["blocks"]:
        Hb = inst.H[off:off + m, off:off + m]
        db = O.cost_diagonal(Hb, None, 0.0)
        eb, gb = O.gradient(db, x)
        Es += eb
        gs += gb
    assert abs(E - Es) <= 1e-12 * (1 + abs(Es))
    assert np.max(np.abs(g - gs)) <= 1e-11 * (1 + np.abs(gs).max())


def test_invariants():
    inst = W.unit_commitment_shaped(9, 3)
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    ell, b = O.canonicalise(inst.H, inst.f)
    alpha, *_ = O.ising_coefficients(ell, b, inst.c0)
    scale = np.abs(d).max()
    rng = np.random.default_rng(0)
    x = rng.uniform(0, np.pi, size=6)
    psi = O.qaoa_state(d, x)
    assert abs(np.linalg.norm(psi) - 1) <= 1e-13
    # gamma = beta = 0 gives the mean of C
    assert abs(O.energy(d, np.zeros(6)) - alpha) <= 1e-12 * scale
    # beta = 0: <C> independent of gamma, P uniform
    xb = x.copy()
    xb[1::2] = 0.0
    assert abs(O.energy(d, xb) - alpha) <= 1e-12 * scale
    P = O.probabilities(O.qaoa_state(d, xb))
    assert np.max(np.abs(P - 1.0 / len(d))) <= 1e-15
    # gamma = 0: mixer acts on |+>, an eigenvector of every X_q
    xg = x.copy()
    xg[0::2] = 0.0
    assert abs(O.energy(d, xg) - alpha) <= 1e-12 * scale
    # complex conjugation: E(-x) = E(x)
    assert abs(O.energy(d, -x) - O.energy(d, x)) <= 1e-12 * scale
    # beta = pi: U_M = (-1)^n I
    n = inst.n
    phi = O.apply_phase(d, 0.3, O.qaoa_state(d, x[:4]))
    assert np.linalg.norm(O.apply_mixer(np.pi, phi) - (-1) ** n * phi) <= 1e-13


def test_integer_cost_gamma_period_2pi():
    inst, _ = W.workload1()
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = np.array([0.4, 0.7, 1.1, 0.2])
    x2 = x.copy()
    x2[0] += 2 * np.pi
    x2[2] -= 2 * np.pi
    assert np.linalg.norm(O.qaoa_state(d, x) - O.qaoa_state(d, x2)) <= 1e-9


@pytest.mark.parametrize("maker,p", [
    (lambda: W.dense_integer_symmetric(6, 3), 1),
    (lambda: W.unit_commitment_shaped(7, 4), 2),
    (lambda: W.regular_graph_qubo(8, 5), 3),
    (lambda: W.dense_gaussian_upper(7, 6), 2),
])
def test_adjoint_gradient_vs_central_fd(maker, p):
    inst = maker()
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    x = W.random_params(p, 1, 77)[0]
    E, g = O.gradient(d, x)
    assert abs(E - O.energy(d, x)) <= 1e-12 * (1 + abs(E))
    gfd = O.fd_gradient(d, x, h=1e-6)
    assert np.max(np.abs(g - gfd)) <= 1e-6 * np.abs(g).max()


def test_partitioned_equals_monolithic():
    inst, params, _ = W.workload5(n=10, qpus=2)
    q = W.contiguous_allocation(10, [5, 5])
    d = O.cost_diagonal(inst.H, inst.f, inst.c0)
    parts = O.partitioned_diagonals(inst.H, inst.f, inst.c0, q, 2)
    assert len(parts) == 3
    assert np.max(np.abs(sum(parts) - d)) <= 1e-12 * np.abs(d).max()
    for x in params:
        a = O.qaoa_state(d, x)
        bst = O.qaoa_state_multi(parts, x)
        assert np.linalg.norm(a - bst) <= 1e-11
    # integer instance: exact sum
    inst1, _ = W.workload1()
    q1 = W.contiguous_allocation(12, [4, 4, 4])
    d1 = O.cost_diagonal(inst1.H, inst1.f, inst1.c0)
    p1 = O.partitioned_diagonals(inst1.H, inst1.f, inst1.c0, q1, 3)
    assert np.array_equal(sum(p1), d1.astype(np.float64))


def test_fig1_cross_counts_golden():
    with open(os.path.join(GOLDEN, "fig1_allocation.json")) as fh:
        g = json.load(fh)

    def b_from_edges(edges):
        b = np.zeros((6, 6))
        for i, j in edges:
            b[min(i, j) - 1, max(i, j) - 1] = 1.0
        return b

    ba = b_from_edges(g["panel_a_edges"])
    for name, a in g["allocations"].items():
        q = np.zeros(6, dtype=int)
        for v in a["qpu2"]:
            q[v - 1] = 1
        assert O.validate_allocation(q, 2, [3, 3])
        assert O.cross_terms(ba, q) == a["cross_from_panel_a_edges"], name
        # the count printed in each panel is the count of that panel's drawn edges
        assert O.cross_terms(b_from_edges(a["panel_edges"]), q) == a["printed_cross"], name
        coef = int(a["printed_remote_cx"].rstrip("p"))
        for p in (1, 2, 5):
            assert O.remote_cx_estimate(a["printed_cross"], p) == coef * p


def test_allocation_rules():
    assert O.balanced_capacities(10, 3) == [4, 3, 3]
    assert O.balanced_capacities(32, 4) == [8, 8, 8, 8]
    assert O.validate_allocation([0, 0, 1, 1], 2, [2, 2])
    assert not O.validate_allocation([0, 0, 0, 1], 2, [2, 2])  # capacity exceeded
    assert not O.validate_allocation([0, 0, 0, 0], 2)  # QPU 1 unused
    assert not O.validate_allocation([0, 2, 1, 1], 2)  # out of range


def test_topk_and_ties():
    P = np.array([0.1, 0.3, 0.3, 0.05, 0.25])
    assert list(O.topk(P, 3)) == [1, 2, 4]
    assert O.argmin_cost(np.array([3, -1, 2, -1])) == 1


# --- planted mistakes: each must be caught by one of the pins above -------------------------

def test_planted_wrong_mixer_sign_is_caught():
    ell, c0, g, b = 1.3, 0.2, 0.4, 0.7
    d = O.cost_diagonal(np.array([[ell]]), None, c0)
    psi = np.full(2, 2 ** -0.5, dtype=complex)
    psi = O.apply_phase(d, g, psi)
    wrong = O.apply_mixer(b, psi, sign=-1)  # RX(-2 beta) instead of RX(2 beta)
    Eref, _ = n1_closed_form(ell, c0, g, b)
    assert abs(O.expectation(d, wrong) - Eref) > 1e-3


def test_planted_wrong_phase_sign_is_caught():
    ell, c0, g, b = 1.3, 0.2, 0.4, 0.7
    d = O.cost_diagonal(np.array([[ell]]), None, c0)
    psi = np.full(2, 2 ** -0.5, dtype=complex)
    psi = O.apply_mixer(b, O.apply_phase(d, g, psi, sign=-1))
    Eref, _ = n1_closed_form(ell, c0, g, b)
    assert abs(O.expectation(d, psi) - Eref) > 1e-3


def test_planted_dropped_transpose_term_is_caught():
    rng = np.random.default_rng(5)
    n = 6
    H = rng.integers(-5, 6, size=(n, n)).astype(float)
    ell, b = O.canonicalise(H, None)
    wrong_b = np.triu(H, 1)  # b_ij = H_ij only: drops H_ji
    wrong = O.cost_diagonal_real(ell, wrong_b, 0.0)
    assert not np.allclose(wrong, brute_force_F(H, np.zeros(n), 0.0))
