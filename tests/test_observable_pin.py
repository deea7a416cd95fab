"""Pins of the oracle's observable (the loss of the differentiated workload).

The loss is the sum of <Z_i> over a set of output qubits, with qubit i at bit
i of the read-out index (Eq. 8 fixes the bit order of the state array; the
Pauli Z is the one of Sec. 2.1).  ``oracle.core.z_weights`` and
``oracle.core.loss_z`` evaluate it through a diagonal weight vector; here the
same quantity is built independently as a dense operator from Kronecker
products of 2x2 matrices, checked on closed forms, and pushed through whole
patterns whose loss has a closed form in the angles.  A planted sign error or
a reversed bit order in the weight vector fails these pins (checked below on
planted copies).  No GPU.
"""
import itertools
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc

PAULI_Z = np.array([[1.0, 0.0], [0.0, -1.0]])
ID2 = np.eye(2)


def dense_z_sum(n: int, obs) -> np.ndarray:
    """sum_{i in obs} Z_i as a 2^n x 2^n matrix.  np.kron(A, B) puts A on
    the high bits of the index, so the factor list runs from qubit n-1 down
    to qubit 0."""
    h = np.zeros((1 << n, 1 << n))
    for i in obs:
        op = np.ones((1, 1))
        for k in range(n - 1, -1, -1):
            op = np.kron(op, PAULI_Z if k == i else ID2)
        h += op
    return h


def _subsets(n):
    out = [list(range(n))]
    if n > 1:
        out += [[0], [n - 1], list(range(0, n, 2))]
    if n > 2:
        out.append([1, n - 1])
    return out


def _random_state(g, n):
    v = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def _dense_and_closed_forms_hold(zw, lz) -> bool:
    """Every check of this file's first two tests on a given (z_weights,
    loss_z) pair; True when all hold."""
    g = np.random.default_rng(7)
    for n in range(1, 7):
        for obs in _subsets(n):
            h = dense_z_sum(n, obs)
            if not np.allclose(zw(n, obs), np.diag(h), atol=1e-12):
                return False
            for _ in range(3):
                psi = _random_state(g, n)
                if abs(lz(psi, obs) - float(np.real(np.vdot(psi, h @ psi)))) > 1e-12:
                    return False
            zero = np.zeros(1 << n, complex)
            zero[0] = 1
            ones = np.zeros(1 << n, complex)
            ones[-1] = 1
            plus = np.full(1 << n, 1 / math.sqrt(1 << n), complex)
            if abs(lz(zero, obs) - len(obs)) > 1e-12 or abs(lz(ones, obs) + len(obs)) > 1e-12:
                return False
            if abs(lz(plus, obs)) > 1e-12:
                return False
            # one qubit flipped: only its own term changes sign
            for q in range(n):
                e = np.zeros(1 << n, complex)
                e[1 << q] = 1
                want = len(obs) - 2 * (q in obs)
                if abs(lz(e, obs) - want) > 1e-12:
                    return False
    return True


def test_z_weights_equal_dense_pauli_sum_and_closed_forms():
    assert _dense_and_closed_forms_hold(oc.z_weights, oc.loss_z)


def test_default_observable_is_every_output():
    g = np.random.default_rng(3)
    for n in range(1, 6):
        psi = _random_state(g, n)
        assert oc.loss_z(psi) == pytest.approx(oc.loss_z(psi, list(range(n))), abs=1e-14)
        np.testing.assert_array_equal(oc.z_weights(n), oc.z_weights(n, list(range(n))))


def test_planted_observable_mistakes_fail_the_pins():
    def zw_bit_reversed(n, obs=None):
        obs = list(range(n)) if obs is None else list(obs)
        return oc.z_weights(n, [n - 1 - i for i in obs])

    def zw_sign(n, obs=None):
        return -oc.z_weights(n, obs)

    def zw_dropped_term(n, obs=None):
        obs = list(range(n)) if obs is None else list(obs)
        return oc.z_weights(n, obs[:-1])

    for zw in (zw_bit_reversed, zw_sign, zw_dropped_term):
        def lz(psi, obs=None, zw=zw):
            n = int(round(math.log2(psi.size)))
            return float(np.sum(zw(n, obs) * np.abs(psi) ** 2))
        assert not _dense_and_closed_forms_hold(zw, lz), zw.__name__


@pytest.mark.parametrize("n_logical", [1, 2, 3, 4])
def test_loss_of_one_ansatz_layer_is_a_cosine_sum(n_logical):
    """One layer of J(beta_q) on |+>^n then a CZ brick: CZ is diagonal, so
    <Z_q> = <+|J(beta)^dag Z J(beta)|+> = cos(beta), and the loss over obs is
    sum_{q in obs} cos(beta_q), whatever the outcome string (J(beta) =
    H diag(1, e^{i beta}); cos is even, so the sign convention of the M angle
    does not enter).  The pattern's M angles are taken in qubit order for a
    single layer."""
    g = np.random.default_rng(100 + n_logical)
    beta = g.uniform(0, 2 * math.pi, size=(1, n_logical))
    pat = W.ansatz_pattern(n_logical, 1, beta)
    alphas = pat.angles()
    assert alphas.size == n_logical
    np.testing.assert_allclose(np.cos(alphas), np.cos(beta[0]), atol=1e-12)
    subsets = [None] + [list(s) for r in range(1, n_logical + 1)
                        for s in itertools.combinations(range(n_logical), r)]
    for outcomes in (np.zeros(pat.n_meas(), np.uint8), g.integers(0, 2, pat.n_meas()).astype(np.uint8)):
        for obs in subsets:
            qs = list(range(n_logical)) if obs is None else obs
            want = sum(math.cos(beta[0, q]) for q in qs)
            for mode in (oc.MODE_OWQS, oc.MODE_EOWQS):
                assert oc.loss_at(pat, outcomes, alphas, mode=mode, obs=obs) == pytest.approx(want, abs=1e-12)
            # and the gradient: d/dalpha_q cos(alpha_q) = -sin(alpha_q) on obs, 0 elsewhere
            gs = oc.param_shift_grad(pat, outcomes, alphas, obs=obs)
            want_g = np.array([-math.sin(alphas[q]) if q in qs else 0.0 for q in range(n_logical)])
            np.testing.assert_allclose(gs, want_g, atol=1e-12)
