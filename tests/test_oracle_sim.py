"""Pins for the oracle simulator: each test checks it against something other
than itself (numpy Kronecker products, closed forms, invariants)."""

import itertools
import math

import numpy as np
import pytest

import oracle as O
from workloads import (KIND_CU, KIND_CX, KIND_U, H, ghz_circuit, haar_u2, layered_circuit,
                       make_gates, mixed_circuit, qft_circuit)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_dense_kron_matches_gate_by_gate(n):
    g = mixed_circuit(n, 40 + 10 * n, seed=n)
    U = O.dense_unitary(g, n)
    for x in (0, (1 << n) - 1, (1 << n) // 3):
        s = O.run(g, n, x=x)
        assert np.abs(s - U[:, x]).max() < 1e-12


def test_dense_checker_is_unitary_and_layered():
    n = 6
    g = layered_circuit(n, 4, seed=3)
    U = O.dense_unitary(g, n)
    assert np.abs(U.conj().T @ U - np.eye(1 << n)).max() < 1e-12
    assert np.abs(O.run(g, n) - U[:, 0]).max() < 1e-12


@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz_closed_form(n):
    s = O.run(ghz_circuit(n), n)
    exp = np.zeros(1 << n, dtype=np.complex128)
    exp[0] = exp[-1] = 1 / math.sqrt(2)
    assert np.abs(s - exp).max() < 1e-15
    assert np.abs(O.expect_z(s, n)).max() < 1e-15
    assert abs(O.norm(s, n) - 1) < 1e-15


@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_qft_on_basis_state_closed_form(n):
    N = 1 << n
    rev = [int(format(y, f"0{n}b")[::-1], 2) for y in range(N)]
    g = qft_circuit(n)
    for x in sorted({0, 1, (N // 2 + 1) % N, N - 1}):
        s = O.run(g, n, x=x)
        y = np.arange(N)
        exp = np.zeros(N, dtype=np.complex128)
        exp[rev] = np.exp(2j * math.pi * x * y / N) / math.sqrt(N)
        assert np.abs(s - exp).max() < 1e-13


def test_norm_preserved_long_circuit():
    n = 14
    g = layered_circuit(n, 30, seed=5)
    s = O.run(g, n)
    assert abs(O.norm(s, n) - 1.0) < 1e-12


def test_product_state_expectation_closed_form():
    n = 8
    rng = np.random.default_rng(0)
    mats = [haar_u2(rng) for _ in range(n)]
    g = make_gates([(KIND_U, q, -1, mats[q]) for q in range(n)])
    ez = O.expect_z(O.run(g, n), n)
    exp = [abs(m[0, 0]) ** 2 - abs(m[1, 0]) ** 2 for m in mats]
    assert np.abs(ez - exp).max() < 1e-14


def test_u_then_udagger_returns_start():
    n = 9
    g = mixed_circuit(n, 120, seed=9)
    inv = []
    for rec in g[::-1]:
        u = rec["u"][0::2] + 1j * rec["u"][1::2]
        m = u.reshape(2, 2).conj().T
        inv.append((int(rec["kind"]), int(rec["q0"]), int(rec["q1"]), m))
    s = O.run(g, n, x=37)
    back = O.run(make_gates(inv), n, state=s)
    exp = O.zero_state(n, 37)
    assert np.abs(back - exp).max() < 1e-13


def test_controlled_gate_acts_only_on_control_one():
    n = 3
    m = haar_u2(np.random.default_rng(4))
    g = make_gates([(KIND_CU, 2, 0, m)])
    U = O.dense_unitary(g, n)
    # control qubit 2 = 0: identity block
    for x in range(4):
        assert np.abs(U[:, x] - np.eye(8)[:, x]).max() == 0
    # control = 1: m acting on qubit 0
    assert np.allclose(U[4:6, 4:6], m, atol=1e-15)


# ----------------------------------------------------------------------------
# placement sigma and PermuteQubits data movement (paper, Section 2)

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_index_map_is_bijection_for_every_sigma(n):
    for sigma in itertools.permutations(range(n)):
        js = sorted(O.index_map(i, n, sigma) for i in range(1 << n))
        assert js == list(range(1 << n))
        # qubit q alone set -> position sigma(q)
        for q in range(n):
            assert O.index_map(1 << q, n, sigma) == 1 << sigma[q]


def test_permutation_round_trip_identity():
    n = 7
    v = O.run(mixed_circuit(n, 50, seed=2), n)
    rng = np.random.default_rng(1)
    for _ in range(10):
        s1, s2 = list(rng.permutation(n)), list(rng.permutation(n))
        w = O.permute(O.permute(v, n, list(range(n)), s1), n, s1, s2)
        back = O.permute(w, n, s2, list(range(n)))
        assert np.array_equal(back, v)


def test_single_exchange_equals_swap_gate():
    """Exchanging the positions of qubits a and b is the SWAP gate, written as
    three CNOTs and simulated gate by gate."""
    n = 6
    v = O.run(mixed_circuit(n, 40, seed=6), n)
    for a, b in [(0, 5), (1, 3), (4, 2)]:
        sigma = list(range(n))
        sigma[a], sigma[b] = b, a
        moved = O.permute(v, n, list(range(n)), sigma)
        swap = make_gates([(KIND_CX, a, b, None), (KIND_CX, b, a, None), (KIND_CX, a, b, None)])
        assert np.array_equal(moved, O.run(swap, n, state=v))


def test_gate_on_permuted_layout_commutes_with_relayout():
    """A gate on logical q applied at bit sigma(q) of the permuted vector equals
    permuting after applying it in logical order."""
    n = 7
    v = O.run(mixed_circuit(n, 30, seed=8), n)
    sigma = [3, 6, 0, 5, 1, 4, 2]
    g = mixed_circuit(n, 25, seed=11)
    phys = O.permute(v, n, list(range(n)), sigma)
    for rec in g:
        q1 = int(rec["q1"])
        O.apply_gate(phys, n, int(rec["kind"]), sigma[int(rec["q0"])], sigma[q1] if q1 >= 0 else -1,
                     rec["u"])
    logical = O.run(g, n, state=v)
    assert np.abs(O.to_logical(phys, n, sigma) - logical).max() < 1e-14


def test_expect_z_sign_convention():
    n = 4
    for x in range(1 << n):
        ez = O.expect_z(O.zero_state(n, x), n)
        assert list(ez) == [1.0 - 2 * ((x >> q) & 1) for q in range(n)]


def test_hadamard_layer_uniform_amplitudes():
    n = 10
    g = make_gates([(KIND_U, q, -1, H) for q in range(n)])
    s = O.run(g, n)
    assert np.abs(s - 1 / math.sqrt(1 << n)).max() < 1e-15
