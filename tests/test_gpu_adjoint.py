"""Adjoint gradients on the GPU against the oracle: parameter shift (exact for
RX/RY/RZ), central finite differences, and the oracle's FP64 expectation."""

import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import ensure_built, log
from workloads import Gate, ansatz, ansatz_params, zz_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _sim(n, dtype, eb=0.0, **kw):
    from paper_2309_16979_amd import Simulator
    return Simulator(n, dtype=dtype, eb=eb, **kw)


def _layers_ckpt(n, layers, every):
    per = 3 * n   # RY + RZ on every qubit, then n CZ
    return [l * per for l in range(0, layers, every)]


@pytest.mark.parametrize("dtype,eb,tol", [("c128", 0.0, 1e-10), ("c64", 0.0, 2e-4), ("c64", 1e-6, 2e-3)])
@pytest.mark.parametrize("n,layers,ckpt_every", [(8, 2, 1), (11, 3, 2)])
def test_adjoint_matches_parameter_shift(dtype, eb, tol, n, layers, ckpt_every):
    gates = ansatz(n, layers)
    params = ansatz_params(n, layers, seed=n + layers)[0]
    masks, coeffs = zz_chain(n)
    ref_e = oracle.energy(n, gates, params, masks, coeffs)
    ref_g = oracle.param_shift_gradient(n, gates, params, masks, coeffs)
    log("adjoint", dtype, eb, n, layers)
    with _sim(n, dtype, eb, chunk_qubits=min(n, 8)) as s:
        s.init_basis(0)
        before = s.amplitudes()
        ev, g = s.adjoint(gates, params, masks, coeffs, _layers_ckpt(n, layers, ckpt_every))
        after = s.amplitudes()
        st = s.stats()
    assert ev == pytest.approx(ref_e, abs=tol * 10)
    assert np.max(np.abs(g - ref_g)) <= tol * max(1.0, np.max(np.abs(ref_g)))
    assert np.array_equal(before.view(np.uint8), after.view(np.uint8))
    assert st["bound_violations"] == 0


def test_adjoint_all_parameterised_kinds():
    """RX, RY, RZ, P and CP parameters, including one parameter feeding two gates."""
    n = 7
    rng = np.random.default_rng(4)
    gates = [Gate("H", q) for q in range(n)]
    kinds = ["RX", "RY", "RZ", "P", "CP"]
    p = 0
    for layer in range(3):
        for q in range(n):
            k = kinds[(q + layer) % 5]
            if k == "CP":
                gates.append(Gate("CP", q, (q + 1) % n, 0.0, p))
            else:
                gates.append(Gate(k, q, -1, 0.0, p))
            p += 1
        gates.append(Gate("CX", layer % n, (layer + 3) % n))
    gates.append(Gate("RY", 2, -1, 0.0, 0))   # parameter 0 feeds a second gate
    params = rng.uniform(-math.pi, math.pi, p)
    masks, coeffs = [0b11, 0b101, 1 << 6, 0b1110000], [1.0, -0.5, 0.75, 0.3]
    h = 1e-5
    fd = np.zeros(p)
    for i in range(p):
        a = params.copy(); a[i] += h
        b = params.copy(); b[i] -= h
        fd[i] = (oracle.energy(n, gates, a, masks, coeffs) - oracle.energy(n, gates, b, masks, coeffs)) / (2 * h)
    log("adjoint kinds")
    with _sim(n, "c128") as s:
        s.init_basis(5)
        ev, g = s.adjoint(gates, params, masks, coeffs, [10, 20])
    assert ev == pytest.approx(oracle.energy(n, gates, params, masks, coeffs, init=5), abs=1e-12)
    ref5 = np.zeros(p)
    for i in range(p):
        a = params.copy(); a[i] += h
        b = params.copy(); b[i] -= h
        ref5[i] = (oracle.energy(n, gates, a, masks, coeffs, init=5)
                   - oracle.energy(n, gates, b, masks, coeffs, init=5)) / (2 * h)
    assert np.max(np.abs(g - ref5)) <= 1e-8


def _sampled_params(n, layers, seed, per_layer_kind=3):
    """Per layer, `per_layer_kind` RY and as many RZ parameters on seeded
    random qubits (6 layers x 2 kinds x 3 = 36 parameters at n = 22)."""
    rng = np.random.default_rng(seed)
    out = []
    for layer in range(layers):
        for q in rng.choice(n, size=per_layer_kind, replace=False):
            out.append(2 * n * layer + 2 * int(q))
        for q in rng.choice(n, size=per_layer_kind, replace=False):
            out.append(2 * n * layer + 2 * int(q) + 1)
    return sorted(out)


def _shift_gradient_sampled(n, gates, params, masks, coeffs, which):
    """Oracle parameter-shift gradient (exact for RY, RZ) of the parameters in
    `which`, each feeding one gate: the state before that gate is simulated
    once (incrementally over the sorted parameters), then the rest of the
    circuit twice, with the angle shifted by +-pi/2."""
    bound = oracle.bind_params(gates, params)
    at = {g.param: i for i, g in enumerate(gates) if g.param >= 0}
    psi, pos, out = oracle.basis(n, 0), 0, {}
    for p in sorted(which, key=lambda p: at[p]):
        gi = at[p]
        psi = oracle.simulate(n, bound[pos:gi], psi)
        pos = gi
        vals = []
        for sh in (math.pi / 2, -math.pi / 2):
            pp = params.copy()
            pp[p] += sh
            tail = oracle.bind_params(gates[gi:], pp)
            vals.append(oracle.expect_z(n, oracle.simulate(n, tail, psi), masks, coeffs))
        out[p] = 0.5 * (vals[0] - vals[1])
    return out


@pytest.mark.timeout(900)
def test_adjoint_ansatz_n22_against_parameter_shift():
    """The n=22 ansatz (6 layers, checkpoints every 2 layers, complex64):
    36 sampled parameters, RY and RZ in every layer, against the oracle's
    parameter-shift gradient (exact for these gates) at 1e-4, and 4 of them
    against central differences (h = 1e-3, FP64). The compressed run
    (eb = 1e-4) is reported against it."""
    n, layers = 22, 6
    gates = ansatz(n, layers)
    params = ansatz_params(n, layers, seed=0)[0]
    masks, coeffs = zz_chain(n)
    ck = _layers_ckpt(n, layers, 2)
    log("adjoint n22 c64 eb=0")
    with _sim(n, "c64") as s:
        s.init_basis(0)
        ev, g = s.adjoint(gates, params, masks, coeffs, ck)
    log("adjoint n22 c64 eb=1e-4")
    with _sim(n, "c64", 1e-4, chunk_qubits=16) as s:
        s.init_basis(0)
        ev_c, g_c = s.adjoint(gates, params, masks, coeffs, ck)
    sample = _sampled_params(n, layers, seed=22)
    assert len(sample) >= 32
    assert {p % 2 for p in sample} == {0, 1} and {p // (2 * n) for p in sample} == set(range(layers))
    ps = _shift_gradient_sampled(n, gates, params, masks, coeffs, sample)
    worst = 0.0
    for i in sample:
        worst = max(worst, abs(g[i] - ps[i]))
        assert abs(g[i] - ps[i]) <= 1e-4, (i, g[i], ps[i])
    assert ev == pytest.approx(oracle.energy(n, gates, params, masks, coeffs), abs=1e-4)
    h = 1e-3
    for i in sample[:: len(sample) // 4][:4]:
        a = params.copy(); a[i] += h
        b = params.copy(); b[i] -= h
        fd = (oracle.energy(n, gates, a, masks, coeffs) - oracle.energy(n, gates, b, masks, coeffs)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-4, (i, g[i], fd)
    print("n22 adjoint: %d parameters, max |g - g_shift| %.3g; compressed eb=1e-4: max |g_c - g_shift| %.3g"
          % (len(sample), worst, max(abs(g_c[i] - ps[i]) for i in sample)))
    print("expval", ev, "compressed", ev_c)
    assert np.all(np.isfinite(g_c))


def test_torch_autograd_function():
    import torch
    from paper_2309_16979_amd import adjoint_expectation
    n, layers = 6, 2
    gates = ansatz(n, layers)
    params = torch.tensor(ansatz_params(n, layers, seed=1)[0], dtype=torch.float64, requires_grad=True)
    masks, coeffs = zz_chain(n)
    log("autograd")
    with _sim(n, "c128") as s:
        e = adjoint_expectation(params, s, gates, 0, masks, coeffs, [])
        (2.0 * e).backward()
    ref = oracle.param_shift_gradient(n, gates, params.detach().numpy(), masks, coeffs)
    assert torch.allclose(params.grad, torch.from_numpy(2.0 * ref), atol=1e-10)
