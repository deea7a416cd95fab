"""Pins of the reordering oracle (PROA, Sec. 4.3) on the CPU: Table I, the
Proposition of Sec. 4.3 (the reordered pattern computes the same output as
the standard form), the m >= |O| + 1 bound, and dependency order."""
import json
import os

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import proa

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def table1_pattern():
    g = json.load(open(os.path.join(GOLD, "table1_swap_proa.json")))
    cmds = [("N", q) for q in g["qubits"]] + [("E", a, b) for a, b in g["edges"]]
    cmds += [("M", q, 0.0, (), ()) for q in g["qubits"] if q not in g["outputs"]]
    return g, W.Pattern([], g["outputs"], cmds)


def test_table1_sub_states_replay():
    g, pat = table1_pattern()
    spaces, after = proa.sub_states_along(pat, g["order"])
    assert spaces == [sorted(x) for x in g["measurement_state_spaces"]]
    assert after == [sorted(sorted(s) for s in a) for a in g["sub_states_after"]]


def test_proa_finds_the_table1_order_and_the_bound():
    g, pat = table1_pattern()
    order, spaces, m, alpha = proa.proa(pat)
    assert order == g["order"]
    assert m == 3 == len(g["outputs"]) + 1


def _outcomes_for(pattern, per_qubit):
    return np.array([per_qubit[c[1]] for c in pattern.cmds if c[0] == "M"], np.uint8)


def test_reordered_patterns_compute_the_standard_form():
    g = np.random.default_rng(4303)
    for i in range(25):
        pat = W.random_standard_pattern(g, n_qubits=int(g.integers(5, 11)), n_in=int(g.integers(0, 3)),
                                        n_out=int(g.integers(1, 3)), extra_edges=int(g.integers(0, 6)))
        order, spaces, m, _ = proa.proa(pat)
        re = proa.reordered_pattern(pat, order)
        assert sorted(c for c in re.cmds if c[0] != "N") != []  # non-trivial
        per_q = {c[1]: int(g.integers(2)) for c in pat.cmds if c[0] == "M"}
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex128) if pat.inputs else None
        want, pw = oc.run(pat, _outcomes_for(pat, per_q), inp)
        got, pg = oc.run(re, _outcomes_for(re, per_q), inp)
        np.testing.assert_allclose(got, want, atol=1e-10)
        # each p is conditional on the outcomes before it; the probability of
        # the whole outcome string (their product) does not depend on the order
        assert float(np.prod(pg)) == pytest.approx(float(np.prod(pw)), rel=1e-9)
        # dependencies come first (the oracle also checks D0 on the run)
        pos = {v: k for k, v in enumerate(order)}
        for c in pat.cmds:
            if c[0] == "M":
                assert all(pos[d] < pos[c[1]] for d in list(c[3]) + list(c[4]))
        # the largest state-space of a connected graph holds at least |O| + 1 qubits
        assert len(pat.outputs) + 1 <= m <= len({c[1] for c in pat.cmds} | set(pat.inputs))


def test_cluster_reaches_the_bound():
    wl = W.cluster(rows=4, cols=6)
    std = W.standard_form(wl.pattern)
    order, spaces, m, _ = proa.proa(std)
    assert m == len(std.outputs) + 1
    re = proa.reordered_pattern(std, order)
    per_q = dict(zip([c[1] for c in wl.pattern.cmds if c[0] == "M"], wl.outcomes))
    want, _ = oc.run(std, _outcomes_for(std, per_q))
    got, _ = oc.run(re, _outcomes_for(re, per_q))
    np.testing.assert_allclose(got, want, atol=1e-10)


def test_positive_branch_ignores_dependencies():
    """EOWQS (Sec. 4.5): with every outcome 0 there are no dependencies, so any
    qubit is ready; the reordered positive branch equals the standard form's."""
    g = np.random.default_rng(4304)
    for _ in range(10):
        pat = W.random_standard_pattern(g, n_qubits=9, n_in=1, n_out=2, extra_edges=3)
        o_dep, _, m_dep, _ = proa.proa(pat)
        o_free, _, m_free, _ = proa.proa(pat, ignore_dependencies=True)
        assert m_free <= m_dep + 0  # never forced into a worse order by dependencies it ignores
        re = proa.reordered_pattern(pat, o_free, positive_branch=True)
        zeros = np.zeros(pat.n_meas(), np.uint8)
        inp = W.gaussian_state(1, g).astype(np.complex128)
        want, _ = oc.run(pat, zeros, inp)
        got, _ = oc.run(re, zeros, inp)
        np.testing.assert_allclose(got, want, atol=1e-10)


def cnot_pattern():
    """CNOT in the measurement calculus (the standard four-qubit pattern):
    inputs 1 (control), 2 (target); outputs 1, 4.  Commands in standard form:
    N3 N4, E13 E23 E34, M2 at 0, M3 at 0, then X4^{s3} Z4^{s2} Z1^{s2}."""
    cmds = [("N", 3), ("N", 4), ("E", 1, 3), ("E", 2, 3), ("E", 3, 4),
            ("M", 2, 0.0, (), ()), ("M", 3, 0.0, (), ()),
            ("X", 4, (3,)), ("Z", 4, (2,)), ("Z", 1, (2,))]
    return W.Pattern([1, 2], [1, 4], cmds)


def test_table3_cnot_state_space():
    """Table III, CNOT row: 4 qubits, m = 3 = |O| + 1 (OWQS and EOWQS)."""
    pat = cnot_pattern()
    for free in (False, True):
        order, spaces, m, _ = proa.proa(pat, ignore_dependencies=free)
        assert m == 3
    # and the pattern is a CNOT for every outcome string: |c t> -> |c, t xor c>
    order, _, _, _ = proa.proa(pat)
    re = proa.reordered_pattern(pat, order)
    for k in range(4):
        inp = np.zeros(4, np.complex128)
        inp[k] = 1.0
        c, t = k & 1, (k >> 1) & 1
        for bits in range(4):
            per_q = {2: bits & 1, 3: bits >> 1}
            out, _ = oc.run(re, _outcomes_for(re, per_q), inp)
            j = c | ((t ^ c) << 1)
            assert abs(abs(out[j]) - 1.0) < 1e-12
