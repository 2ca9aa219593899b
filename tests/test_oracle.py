"""Pins of the FP64 oracle simulator against closed forms, library routines,
brute force and invariants (CPU only)."""

import math

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import (Gate, ghz, qft, random_circuit, inverse, random_unitary,
                       ansatz, ansatz_params, zz_chain, qft_plus_random)

ALL_1Q = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "P")
ALL_2Q = ("CX", "CZ", "CP", "SWAP")


def _random_gate_list(n, count, rng):
    gates = []
    for _ in range(count):
        r = rng.random()
        if r < 0.45:
            name = ALL_1Q[rng.integers(len(ALL_1Q))]
            gates.append(Gate(name, int(rng.integers(n)), -1, float(rng.uniform(-4, 4))))
        elif r < 0.85:
            name = ALL_2Q[rng.integers(len(ALL_2Q))]
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate(name, a, b, float(rng.uniform(-4, 4))))
        elif r < 0.93:
            gates.append(Gate("U1", int(rng.integers(n)), -1, 0.0, -1, random_unitary(1, rng)))
        else:
            a, b = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append(Gate("U2", a, b, 0.0, -1, random_unitary(2, rng)))
    return gates


def test_gate_matrices_match_generator_definitions():
    """Each oracle matrix equals the operator built from its generator
    (expm of Pauli generators, projector sums) on 1-2 qubits."""
    rng = np.random.default_rng(1)
    for name in ALL_1Q:
        th = float(rng.uniform(-4, 4))
        g = Gate(name, 0, -1, th)
        assert np.allclose(oracle.gate_matrix(g), brute.full_operator(1, g), atol=1e-14), name
    for name in ALL_2Q:
        th = float(rng.uniform(-4, 4))
        g = Gate(name, 0, 1, th)
        assert np.allclose(oracle.gate_matrix(g), brute.full_operator(2, g), atol=1e-14), name


def test_controlled_x_orientation():
    # CX with control q0=0, target q1=1: |01> (index 1: q0=1) -> |11> (index 3)
    psi = oracle.simulate(2, [Gate("CX", 0, 1)], init=1)
    assert abs(psi[3] - 1) < 1e-15 and np.sum(np.abs(psi) ** 2) == pytest.approx(1)
    psi = oracle.simulate(2, [Gate("CX", 0, 1)], init=2)  # control 0 -> unchanged
    assert abs(psi[2] - 1) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_simulator_matches_brute_force(n):
    rng = np.random.default_rng(100 + n)
    if n == 1:
        gates = [g for g in _random_gate_list(2, 40, rng) if g.q1 < 0 and g.q0 == 0]
    else:
        gates = _random_gate_list(n, 60, rng)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    ref = brute.brute_simulate(n, gates, v)
    got = oracle.simulate(n, gates, v)
    assert np.max(np.abs(ref - got)) < 1e-13


def test_random_workload_matches_brute_force():
    gates = random_circuit(8, 12, seed=3)
    ref = brute.brute_simulate(8, gates, 5)
    got = oracle.simulate(8, gates, 5)
    assert np.max(np.abs(ref - got)) < 1e-13


@pytest.mark.parametrize("n", [2, 3, 7, 12, 20])
def test_ghz_closed_form(n):
    psi = oracle.simulate(n, ghz(n))
    assert np.max(np.abs(psi - oracle.ghz_state(n))) < 1e-14
    masks, coeffs = zz_chain(n)
    assert oracle.expect_z(n, psi, masks, coeffs) == pytest.approx(n - 1, abs=1e-12)


@pytest.mark.parametrize("n,x", [(3, 5), (6, 0), (6, 41), (10, 777), (14, 12345)])
def test_qft_closed_form_on_basis(n, x):
    psi = oracle.simulate(n, qft(n), x)
    assert np.max(np.abs(psi - oracle.qft_state(n, x))) < 1e-12


def test_qft_equals_scaled_inverse_fft():
    n = 12
    rng = np.random.default_rng(7)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    got = oracle.simulate(n, qft(n), v)
    ref = np.sqrt(v.size) * np.fft.ifft(v)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_qft_brute_force_unitary():
    n = 5
    u = brute.circuit_unitary(n, qft(n))
    N = 1 << n
    y, x = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ref = np.exp(2j * np.pi * x * y / N) / np.sqrt(N)
    assert np.max(np.abs(u - ref)) < 1e-13


def test_norm_and_inverse():
    n = 14
    gates = random_circuit(n, 20, seed=11)
    psi = oracle.simulate(n, gates, 9)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12
    back = oracle.simulate(n, inverse(gates), psi)
    assert abs(back[9] - 1) < 1e-12 * len(gates)
    assert np.sum(np.abs(back) ** 2) - abs(back[9]) ** 2 < 1e-20


def test_expect_z_on_basis_states():
    n = 6
    masks = [0b11, 0b101000, 0b1, 0b111111]
    coeffs = [0.5, -1.25, 2.0, 0.75]
    for x in (0, 1, 17, 63):
        psi = oracle.basis(n, x)
        ref = sum(c * (-1) ** bin(x & m).count("1") for m, c in zip(masks, coeffs))
        assert oracle.expect_z(n, psi, masks, coeffs) == pytest.approx(ref, abs=1e-15)


def test_prob_one_and_fidelity():
    n = 5
    psi = oracle.simulate(n, [Gate("RY", 2, -1, 1.0)])
    assert oracle.prob_one(psi, 2) == pytest.approx(math.sin(0.5) ** 2, abs=1e-15)
    fr, fn = oracle.fidelity(psi, 2.0 * psi)
    assert fr == pytest.approx(4.0) and fn == pytest.approx(1.0)


def test_param_shift_closed_form_one_qubit():
    # f(t) = <Z> after RY(t)|0> = cos t, so f'(t) = -sin t
    gates = [Gate("RY", 0, -1, 0.0, 0)]
    for t in (-2.0, 0.3, 1.1):
        g = oracle.param_shift_gradient(1, gates, [t], [1], [1.0])
        assert g[0] == pytest.approx(-math.sin(t), abs=1e-14)
    # f(t) = <X-basis after RZ>: RY(pi/2) RZ(t) RY(-pi/2)... use <Z> after H RZ(t) H
    gates = [Gate("H", 0), Gate("RZ", 0, -1, 0.0, 0), Gate("H", 0)]
    for t in (0.4, 2.5):
        g = oracle.param_shift_gradient(1, gates, [t], [1], [1.0])
        assert g[0] == pytest.approx(-math.sin(t), abs=1e-14)


def test_param_shift_matches_central_differences():
    n, layers = 5, 2
    gates = ansatz(n, layers)
    params = ansatz_params(n, layers, seed=2)[0]
    masks, coeffs = zz_chain(n)
    ps = oracle.param_shift_gradient(n, gates, params, masks, coeffs)
    h = 1e-4
    fd = np.zeros_like(ps)
    for p in range(len(params)):
        a = params.copy(); a[p] += h
        b = params.copy(); b[p] -= h
        fd[p] = (oracle.energy(n, gates, a, masks, coeffs)
                 - oracle.energy(n, gates, b, masks, coeffs)) / (2 * h)
    assert np.max(np.abs(ps - fd)) < 1e-7


def test_workload_generators_are_deterministic():
    a = random_circuit(20, 20, seed=0)
    b = random_circuit(20, 20, seed=0)
    assert a == b and len(a) > 150
    x1, g1 = qft_plus_random(28, 100, seed=0)
    x2, g2 = qft_plus_random(28, 100, seed=0)
    assert x1 == x2 and len(g1) == 28 + 378 + 14 + 100 and g1 == g2
