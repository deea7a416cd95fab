"""Pins of the gflow oracle (exhaustive search of the definition) on the
CPU: closed cases (the J pattern, more inputs than outputs), flow patterns
(circuits, clusters), the EOWQS premise (Sec. 4.5: a measurement with a
witness has probability exactly 1/2 in the elimination oracle, for random
angles, inputs and earlier outcomes), and gflow without causal flow."""
import math

import numpy as np
import pytest

import owqs_workloads as W
from oracle import core as oc
from oracle import gflow as gf


def test_j_pattern_has_a_witness():
    pat = W.Pattern([1], [2], [("N", 2), ("E", 1, 2), ("M", 1, 0.3, (), ()), ("X", 2, (1,))])
    assert gf.certify_order(pat) == [[2]]
    assert gf.gflow_exists(pat) and gf.causal_flow_exists(pat)


def test_more_inputs_than_outputs_has_no_gflow():
    pat = W.Pattern([1, 2], [3], [("N", 3), ("E", 1, 3), ("E", 2, 3), ("M", 1, 0.0, (), ()),
                                  ("M", 2, 0.0, (), ())])
    cert = gf.certify_order(pat)
    assert cert[0] == [3] and cert[1] is None
    assert not gf.gflow_exists(pat)


def test_flow_patterns_are_certified():
    g = np.random.default_rng(4901)
    for _ in range(10):
        nl = int(g.integers(1, 5))
        pat = W.circuit_to_pattern(nl, W.random_jcz_circuit(nl, int(g.integers(1, 10)),
                                                            int(g.integers(0, 4)) if nl > 1 else 0, g))
        assert all(w is not None for w in gf.certify_order(pat))
    cl = W.cluster(rows=3, cols=4).pattern
    assert all(w is not None for w in gf.certify_order(cl))


def _random_xy_pattern(g, n):
    """Random graph on n qubits, random inputs/outputs, measurements in a
    random order at random XY angles with random domains over earlier ones."""
    qs = list(range(n))
    n_in = int(g.integers(0, 3))
    n_out = int(g.integers(1, 3))
    perm = list(g.permutation(n))
    ins, outs = sorted(perm[:n_in]), sorted(perm[n - n_out:])
    edges = {(a, b) for a in qs for b in qs if a < b and g.random() < 0.45}
    cmds = [("N", q) for q in qs if q not in ins] + [("E", a, b) for a, b in sorted(edges)]
    meas = [q for q in g.permutation(n).tolist() if q not in outs]
    done = []
    for q in meas:
        k = int(g.integers(0, min(2, len(done)) + 1))
        s = tuple(int(x) for x in g.choice(done, size=k, replace=False)) if k else ()
        cmds.append(("M", q, float(g.uniform(0, 2 * math.pi)), s, ()))
        done.append(q)
    return W.Pattern(ins, outs, cmds)


def test_a_witness_means_probability_one_half():
    """Sec. 4.5's premise, measurement by measurement: with a witness for the
    pattern's order, p = 1/2 exactly (any angles, input and earlier outcomes);
    without one, p differs from 1/2 somewhere among the draws."""
    g = np.random.default_rng(4902)
    with_w = without = off_half = 0
    for _ in range(150):
        pat = _random_xy_pattern(g, int(g.integers(3, 8)))
        cert = gf.certify_order(pat)
        inp = W.gaussian_state(len(pat.inputs), g).astype(np.complex128) if pat.inputs else None
        if inp is not None:
            inp /= np.linalg.norm(inp)   # p is relative to a unit input
        outc = g.integers(0, 2, pat.n_meas()).astype(np.uint8)
        try:
            _, probs = oc.run(pat, outc, inp)
        except oc.OracleError:
            continue   # a forced outcome of probability 0 (only where there is no witness)
        for w, p in zip(cert, probs):
            if w is not None:
                with_w += 1
                assert p == pytest.approx(0.5, abs=1e-12)
            else:
                without += 1
                off_half += abs(p - 0.5) > 1e-6
    assert with_w > 100 and without > 20 and off_half > without // 2


def test_gflow_without_causal_flow_exists():
    """A generalised flow is strictly more general: some small open graph has
    one without having a causal flow; causal flow always implies gflow."""
    g = np.random.default_rng(4903)
    found = False
    for _ in range(400):
        n = int(g.integers(3, 7))
        pat = _random_xy_pattern(g, n)
        gfl, cfl = gf.gflow_exists(pat), gf.causal_flow_exists(pat)
        assert gfl or not cfl
        found = found or (gfl and not cfl)
    assert found


def test_witness_needs_the_odd_neighbourhood():
    """Edges 0-2, 0-3, 1-2, outputs 2 and 3, measuring 0 then 1: qubit 1's only
    witness is {2, 3}, whose odd neighbourhood N(2) xor N(3) = {0,1} xor {0}
    = {1} avoids the earlier qubit 0 (their union would not)."""
    pat = W.Pattern([], [2, 3], [("N", 0), ("N", 1), ("N", 2), ("N", 3), ("E", 0, 2), ("E", 0, 3), ("E", 1, 2),
                                 ("M", 0, 0.4, (), ()), ("M", 1, 1.1, (), ())])
    assert gf.certify_order(pat) == [[2], [2, 3]]
    _, probs = oc.run(pat, [1, 0])
    np.testing.assert_allclose(probs, [0.5, 0.5], atol=1e-12)
